/*
 * recogs.h -- C ABI of the MI355X (gfx950) select / recolour / splat-render library.
 *
 * The operations follow ReCoGS (Rutayisire, Capodieci, Pellacini; arXiv 2511.18441):
 * a pre-trained 3D Gaussian Splatting scene (Sec. 3.1: covariance eq. 1, SH colour
 * eq. 2, front-to-back alpha blending eq. 3) has a region selected (Sec. 3.2) and
 * tinted (Sec. 3.3, eq. 6), is rendered with an HWC output (Sec. 4.2) and
 * differentiated w.r.t. its colour parameters (Sec. 4.1, eq. 7-8).
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers unless marked (host). The caller owns every
 *     buffer. The library allocates no device memory and keeps no device state
 *     between calls (one exception: the fixed array of recogs_unproject_noalloc);
 *     render state lives in a caller-provided workspace.
 *   - Scene arrays are structure-of-arrays "planes": plane p of an array with
 *     stride s occupies elements [p*s, p*s + n). All planes of one scene share
 *     one stride >= n.
 *   - Every call is enqueued on `stream` (NULL = the null stream) and returns a
 *     status. Argument errors are found on the host before anything is enqueued.
 *     recogs_render in its default (eager) mode synchronises `stream` once, to read
 *     the number of tile keys; the read-back calls (recogs_workspace_readback,
 *     recogs_workspace_keys_needed, recogs_batch_readback) wait for `stream`; the
 *     other calls never synchronise.
 *   - On error, recogs_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread). No call aborts or throws.
 *   - Float math on the GPU is float32; storage may be f16 / bf16 for opacity and SH.
 */
#ifndef RECOGS_H
#define RECOGS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { RECOGS_F32 = 0, RECOGS_F16 = 1, RECOGS_BF16 = 2 } recogs_dtype;

typedef enum {
    RECOGS_OK = 0,
    RECOGS_ERR_INVALID = -1,      /* bad argument (null pointer, size, shape, enum)  */
    RECOGS_ERR_CAPACITY = -2,     /* workspace too small for the tile keys of this view */
    RECOGS_ERR_UNSUPPORTED = -3,  /* valid but not supported (e.g. tile shape)        */
    RECOGS_ERR_HIP = -4           /* a HIP runtime call failed; see recogs_last_error */
} recogs_status;

/* Scene (eq. 1-2). Geometry is frozen while colours are edited (Sec. 3.3).
 *   means   float [3][stride]          world-space centres x, y, z
 *   cov3d   float [6][stride]          3D covariance xx, xy, xz, yy, yz, zz (eq. 1)
 *   opacity storage [stride]           activated opacity sigma in (0, 1)
 *   sh      storage [(deg+1)^2*3][stride]  SH coefficients, plane = k*3 + channel,
 *                                      k = l*l + l + m, real SH with Condon-Shortley
 *                                      phase; displayed colour = max(0, f + 1/2). */
typedef struct {
    int64_t n;
    int64_t stride;
    int32_t sh_degree;   /* 0..3 */
    int32_t storage;     /* recogs_dtype of opacity and sh */
    const float *means;
    const float *cov3d;
    const void *opacity;
    const void *sh;
} recogs_scene;

/* Pinhole camera (host struct). World -> camera m = R mu + t, axes x right, y down,
 * z forward. Pixel (px, py) has its centre at (px + 1/2, py + 1/2); a point projects
 * to (fx m_x / m_z + cx, fy m_y / m_z + cy). Points with depth <= znear are culled. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];          /* row-major */
    float t[3];
    float znear;
} recogs_camera;

/* Selection (host struct): a Gaussian is selected when its depth is > znear, its
 * projected centre lies in the closed disk (cx, cy, radius) [pixels] and its DC
 * colour Y00 C0 + 1/2 lies in the closed ball (ref, color_radius). */
typedef struct {
    float cx, cy, radius;
    float ref[3];
    float color_radius;
} recogs_select_params;

/* Render options (host struct). */
typedef struct {
    int32_t tile_w, tile_h;      /* sort tile: 8x8, 16x16, 32x8, 32x16 or 32x32 */
    int32_t px_per_thread;       /* 1, 2 or 4 pixels per blend thread. Where tile_h is a multiple
                                    of 8 * px_per_thread the blend runs one wave per 8 x
                                    8*px_per_thread block of a tile; otherwise one workgroup
                                    per tile. Outputs are bit-identical for every shape. */
    float bg[3];                 /* background colour */
    /* Optional fused recolour (all three NULL = off): selected Gaussians display
     * max(0, M (f + 1/2) + b) instead of max(0, f + 1/2). Device pointers:
     * mask uint8 [n], M float [9] row-major, b float [3]. */
    const uint8_t *mask;
    const float *M;
    const float *b;
    int32_t keep_backward_state; /* 1: store what recogs_render_backward needs (per-Gaussian colour
                                    state, per-pixel final transmittance and list count); 0: the
                                    workspace's final_T / nproc are not written */
    /* Stage timing with HIP events recorded on `stream`.
     * 0: off. 1: events between all stages; this call waits for its blend and writes the
     * durations to ws->stage_ms. 2: the blend's duration, accumulated without waiting:
     * events are recorded just before and after the blend launch only (an event between
     * two kernels delays the second one's dispatch by microseconds), and the duration
     * of the workspace's previous mode-2 call (complete by then) is added to
     * ws->stage_ms_sum[8] with ws->profiled_frames incremented, at this call's
     * key-count read-back; recogs_workspace_profile_flush adds the last one. Mode 2
     * creates its event objects on first use; recogs_workspace_release destroys them. */
    int32_t profile_stages;
    /* How the (tile, depth, index) order of the tile lists is produced; all give the
     * same order. 0 (default): sort the Gaussians with keys by depth (32-bit keys),
     * emit their tile keys in that order, then stable-sort the tile ids (the LSD
     * depth digits sorted before the keys are duplicated). 1: emit 64-bit keys
     * (tile << 32) | depth bits in index order and radix-sort them. 2: emit the tile
     * ids in index order, stable-sort them, then sort each tile's list by depth with
     * one workgroup (lists of up to 8,192 keys in LDS, longer ones through memory). */
    int32_t sort_mode;
    /* 1: no host synchronisation (the render may be captured in a HIP graph). The
     * key count, capacity decision and overflow flag stay on the device: a view with
     * more keys than ws->key_capacity draws only the background, and
     * recogs_workspace_readback reports num_keys / num_visible afterwards
     * (num_keys > key_capacity: overflowed). Needs sort_mode 0 or 2; profile_stages 0 or 2.
     * 0: the render reads the key count back once (eager capacity check). */
    int32_t graph_mode;
    /* Output layout (Sec. 4.2 compares the two). 0 (default): image float [H][W][3]
     * (HWC, the layout the paper switches the rasteriser to). 1: float [3][H][W] (CHW,
     * the rasteriser's original layout); the values are the same bits, only the
     * addresses differ. recogs_render_backward needs an HWC render. */
    int32_t output_chw;
    /* Rough depth map (Sec. 3.2): with depth_map non-NULL (device float [H][W]) the blend
     * also writes, per pixel, the float32 depth of the blended splat that takes the
     * transmittance from >= depth_tau to < depth_tau (front to back, eq. 3), and 0 where
     * the transmittance never falls below depth_tau before the pixel stops. Needs
     * 0 < depth_tau <= 1 (INVALID otherwise) and a tile whose height is a multiple of
     * 8 * px_per_thread (UNSUPPORTED otherwise); single-view renders only (batch
     * workspaces reject it). NULL: no depth map, depth_tau ignored. */
    float *depth_map;
    float depth_tau;
    /* Which tiles list a splat (the paper renders with the original 3DGS rasteriser,
     * Sec. 4; its extent is not stated there). 0 (default): every tile meeting the box
     * that holds all pixels where alpha >= 1/255 (2 ln(255 sigma) + 1/64 of the conic's
     * quadratic form), so tiles never change a pixel and every tile shape draws the
     * same bits. 1: the 3DGS rasteriser's square, for comparison with it: radius
     * r = ceil(3 sqrt(lambda_max)) pixels, lambda_max = (a + c)/2 +
     * sqrt(max(0.1, ((a - c)/2)^2 + b^2)) of the 2D covariance [[a, b], [b, c]], tiles
     * floor((x - r) / tile_w) up to, not including, floor((x + r + tile_w - 1) / tile_w)
     * around x = u - 1/2 (the same in y), clipped to the image's tiles; a splat then
     * reaches only the pixels of the tiles that list it, so the image depends on the
     * tile shape. Either rule gives no tiles to a splat with 255 sigma < 1. INVALID
     * otherwise. */
    int32_t extent_rule;
    /* Backward only (ignored by the render): optional device scratch of at least
     * recogs_backward_scratch_bytes bytes, 256-byte aligned, caller-owned, its contents
     * not kept between calls (so calls that share one scratch must not overlap). Given,
     * and where the tile height is a multiple of 8 * px_per_thread, the backward
     * replays each 8 x 8*px_per_thread block of a tile with its own wave, which walks
     * the tile's list without waiting for the others (as the forward blend does), and
     * the tile's workgroup then adds the blocks' parts of each (Gaussian, tile)
     * gradient in block order; NULL: one workgroup per tile whose waves step through
     * the list together. Both are deterministic and give the same gradients up to
     * float32 summation order. INVALID: too small or misaligned. */
    void *bwd_scratch;
    size_t bwd_scratch_bytes;
} recogs_render_opts;

/* Workspace: caller-provided device memory carved by recogs_workspace_init. It holds
 * the per-Gaussian splat records, the tile keys and their sort buffers, the tile
 * ranges and the per-pixel state the backward replays. A workspace must outlive the
 * backward that follows its render and must not be shared by concurrent renders.
 * Fields are filled by the library; callers only read them. Offsets are bytes from
 * `base`. */
typedef struct {
    void *base;
    size_t bytes;
    int64_t n_cap;
    int32_t width, height, tile_w, tile_h;
    int64_t key_capacity;
    int32_t tiles_x, tiles_y;
    /* buffer offsets */
    size_t off_rec, off_bwd, off_gpart, off_zbits, off_rect, off_count, off_offset, off_scan;
    size_t off_keys0, off_keys1, off_vals0, off_vals1, off_hist, off_sort_count;
    size_t off_ranges, off_final_T, off_nproc, off_header;
    size_t off_dkeys0, off_dkeys1, off_dvals0, off_dvals1, off_dhist, off_esum, off_efirst;
    size_t scan_chunks, sort_chunks;
    /* results of the last render, valid when it returned RECOGS_OK (or CAPACITY) */
    int64_t num_keys;            /* K: tile keys emitted */
    int64_t num_visible;         /* V: Gaussians with at least one tile key */
    int32_t sort_mode;           /* sort_mode of the last render */
    int32_t key_bytes;           /* 8: sorted keys are (tile << 32) | depth bits; 4: tile ids */
    int32_t sorted_in_alt;       /* 1 if the sorted keys/values are in keys1/vals1 */
    int32_t sort_passes;         /* passes over the K keys */
    int32_t depth_passes;        /* sort_mode 0: passes over the V depth keys after the count scan's (which orders them by their low 8 depth bits) */
    int32_t key_bits;            /* significant bits sorted: tile bits + depth bits */
    int32_t depth_bits;
    uint32_t depth_min_bits;     /* smallest float32 depth bit pattern among keys */
    int32_t last_n;
    /* with profile_stages: milliseconds of [0] preprocess, [1] scan, [2] key-count read-back,
     * [3] depth sort (sort_mode 0), [4] key emission, [5] key sort, [6] tile ranges,
     * [7] per-tile depth sort (sort_mode 2), [8] blend */
    float stage_ms[9];
    /* with profile_stages = 2: [8] sums the blend's milliseconds over profiled_frames
     * calls (the other entries stay 0); zeroed by recogs_workspace_init */
    double stage_ms_sum[9];
    int64_t profiled_frames;
    void *profile_state;         /* host-side event objects of mode 2 (library-owned) */
    /* incremented by every recogs_render call on this workspace that passes its argument
     * checks (zeroed by recogs_workspace_init): a caller that keeps a render's state for a
     * later backward can tell whether another render has overwritten it since */
    int64_t generation;
} recogs_workspace;

/* ---- support --------------------------------------------------------------- */

/* Bytes of device memory a workspace needs for scenes of up to n Gaussians,
 * width x height images, the given tile shape and up to key_capacity tile keys. */
size_t recogs_workspace_bytes(int64_t n, int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                              int64_t key_capacity);

/* Carve `dev_mem` (>= recogs_workspace_bytes(...) bytes, 256-byte aligned) into *ws.
 * Errors: INVALID for null pointers, bad sizes or too few bytes. */
recogs_status recogs_workspace_init(recogs_workspace *ws, void *dev_mem, size_t bytes, int64_t n,
                                    int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                                    int64_t key_capacity);

/* After a graph_mode render: wait for it and fill ws->num_keys (keys the view needs),
 * ws->num_visible and ws->depth_min_bits from the device header. */
recogs_status recogs_workspace_readback(recogs_workspace *ws, hipStream_t stream);

/* Tile keys the workspace's last render needed (eager or graph mode, whether or not they
 * fitted ws->key_capacity), read from the device header into *out_keys (host). Waits for
 * `stream`. 0 before the first render and for an empty scene. INVALID: NULL or
 * uninitialised workspace, NULL out_keys. A render that returned CAPACITY is repeated
 * with a workspace of at least this many keys. */
recogs_status recogs_workspace_keys_needed(const recogs_workspace *ws, int64_t *out_keys, hipStream_t stream);

/* Wait for the workspace's last profile_stages = 2 render and add its stage durations
 * to stage_ms_sum / profiled_frames. OK when nothing is pending. */
recogs_status recogs_workspace_profile_flush(recogs_workspace *ws);

/* Destroy the event objects that profile_stages = 2 created (no-op otherwise). Call it
 * before re-initialising or dropping a workspace that was profiled in mode 2; the
 * device memory stays the caller's. */
void recogs_workspace_release(recogs_workspace *ws);

/* eq. (1): cov3d = R S S^T R^T from log-scales float [3][stride] and quaternions
 * float [4][stride] (w, x, y, z; normalised here). Output float [6][stride]. */
recogs_status recogs_prepare_covariance(const float *log_scales, const float *quats, float *cov3d,
                                        int64_t n, int64_t stride, hipStream_t stream);

/* ---- the path ---------------------------------------------------------------- */

/* Selection (Sec. 3.2 stand-in): mask uint8 [n] (1 = selected) and *count (device
 * int32, overwritten) = number selected. */
recogs_status recogs_select(const recogs_scene *scene, const recogs_camera *cam,
                            const recogs_select_params *params, uint8_t *mask, int32_t *count,
                            hipStream_t stream);

/* Recolour (Sec. 3.3, eq. 6 generalised): for every selected i the displayed colour
 * becomes M (f + 1/2) + b for every view direction, realised on coefficients as
 * C'_k = M C_k (k >= 1) and C'_0 = M C_0 + ((M - I) 1/2 + b) / Y00.
 * Reads scene->sh, writes dst_sh (same dtype, degree and stride; may equal
 * scene->sh). copy_unselected = 1 also copies unselected Gaussians' coefficients;
 * 0 leaves them untouched in dst_sh. M float [9] row-major and b float [3] are device
 * pointers; f16/bf16 results are rounded to nearest even. */
recogs_status recogs_recolor(const recogs_scene *scene, void *dst_sh, const uint8_t *mask,
                             const float *M, const float *b, int32_t copy_unselected,
                             hipStream_t stream);

/* Render (eq. 2-3; HWC output, Sec. 4.2): EWA projection, tile binning with a
 * (tile, depth) key sort, front-to-back compositing with early termination.
 * image float [height][width][3]. ws must have been initialised for at least this n,
 * the camera's size and opts' tile shape. Synchronises the stream once.
 * Errors: INVALID / UNSUPPORTED before any launch; CAPACITY when more tile keys are
 * needed than ws->key_capacity (ws->num_keys then holds the number needed and the
 * image is not written); HIP. */
recogs_status recogs_render(const recogs_scene *scene, const recogs_camera *cam,
                            const recogs_render_opts *opts, recogs_workspace *ws, float *image,
                            hipStream_t stream);

/* Bytes of the scratch the backward's block form needs (opts->bwd_scratch) for this
 * workspace and opts' tile shape and px_per_thread, with B blocks per tile: a float4
 * per block and key of ws->key_capacity, rounded up to 256 bytes, then B * (capacity / 64
 * + tiles + 2) flag words of 16 bytes. 0 where the shape has no block form or an
 * argument is NULL / unsupported. */
size_t recogs_backward_scratch_bytes(const recogs_workspace *ws, const recogs_render_opts *opts);

/* Backward of the render and of the fused recolour (eq. 8, restricted to opacity,
 * SH DC and the recolour matrix). Needs the workspace of the matching render (run
 * with keep_backward_state = 1, no other render on the workspace since) and its output
 * image. dL_dimage float [H][W][3].
 * Outputs: dL_dopacity float [n], dL_dsh_dc float [3][n] (gradient w.r.t. the DC
 * coefficients C_0 of each channel), dL_dM float [9] (zero when no fused recolour).
 * accumulate 0: they are overwritten; 1: this view's gradients are added to them (a
 * loss summed over views: render and backward each view in turn, accumulate 0 for the
 * first); INVALID otherwise. No atomics: every sum is taken in a fixed order, so results
 * are bit-identical between runs. The backward uses the workspace's sorted-key buffers
 * (keys0/keys1) as per-key gradient scratch; the tile lists and the rest of the
 * render's state stay valid, so it may be called again on the same render. After a
 * graph_mode render it needs no recogs_workspace_readback and does not synchronise
 * either: the key count is read on the device, and a render that overflowed its key
 * capacity (no tile lists) gives zero gradients (the overflow shows in the read-back).
 * INVALID: a render read back as overflowed, no kept state, a CHW render, another
 * scene size, NULL pointers, bad accumulate or bwd_scratch. */
recogs_status recogs_render_backward(const recogs_scene *scene, const recogs_camera *cam,
                                     const recogs_render_opts *opts, const recogs_workspace *ws,
                                     const float *image, const float *dL_dimage, float *dL_dopacity,
                                     float *dL_dsh_dc, float *dL_dM, int32_t accumulate, hipStream_t stream);

/* L2 loss of an image against a target (the differentiable form's loss, an analog of
 * eq. 4 with its gradient, eq. 7): loss (device float, overwritten) = scale * sum (y - t)^2 and
 * dL_dimage = 2 scale (y - t), over `count` floats. scale = 1 / count gives the mean.
 * The workgroups' sums are added to the loss with float atomics, so its last bits may
 * change between runs; the gradient does not. */
recogs_status recogs_loss_l2(const float *image, const float *target, int64_t count, float scale,
                             float *dL_dimage, float *loss, hipStream_t stream);

/* ---- background optimiser (Sec. 3.3, 4.1) -------------------------------------- */

/* The backward of recogs_render_backward with the gradient of every SH coefficient
 * instead of the DC term only: the optimiser of Sec. 3.3 refits the SH coefficients
 * (Sec. 4.1 keeps only dL/dC_l^m of the rasteriser's gradients, eq. 8). The colour of
 * eq. 2 is linear in the coefficients, so dL/dC_{k,c} = Y_k(d) g_c, with d the view
 * direction of the Gaussian's centre and g the colour gradient through the clamp and,
 * for Gaussians the fused recolour selected, through M (g = M^T gh).
 * dL_dsh: device float [3 (sh_degree + 1)^2][scene.stride], plane k * 3 + c: the scene's
 * SH layout, so an optimiser can step the coefficient planes with it directly. Entries
 * 0..n-1 of every plane are written (zero for Gaussians that reach no pixel); the
 * padding entries n..stride-1 are left as they are.
 * Everything else (arguments, accumulate, requirements, determinism, errors) as for
 * recogs_render_backward; the DC planes equal its dL_dsh_dc bit for bit. */
recogs_status recogs_render_backward_sh(const recogs_scene *scene, const recogs_camera *cam,
                                        const recogs_render_opts *opts, const recogs_workspace *ws,
                                        const float *image, const float *dL_dimage, float *dL_dopacity,
                                        float *dL_dsh, float *dL_dM, int32_t accumulate, hipStream_t stream);

/* L1 term of the loss of eq. 4, with the gradient Sec. 4.1 writes out (eq. 7):
 * loss (device float, overwritten) = scale * sum |y - t| and
 * dL_dimage = scale * sign(y - t) (sign(0) = 0), over `count` floats; scale = 1 / count
 * gives the mean. Device pointers of any alignment. The loss's last bits may change
 * between runs (float atomics, as recogs_loss_l2); recogs_loss_l1_dssim sums in a fixed
 * order. INVALID: count < 0, NULL pointer. */
recogs_status recogs_loss_l1(const float *image, const float *target, int64_t count, float scale,
                             float *dL_dimage, float *loss, hipStream_t stream);

/* SSIM term of eq. 4, lambda (1 - SSIM), over two HWC float images [height][width][3]:
 * per channel, local means, variances and covariance under the 11 x 11 Gaussian window
 * (sigma 1.5, zero outside the image), S = (2 mu_y mu_t + C1)(2 s_yt + C2) /
 * ((mu_y^2 + mu_t^2 + C1)(s_y^2 + s_t^2 + C2)), C1 = 0.01^2, C2 = 0.03^2, averaged over
 * all pixels and channels. loss (device float, overwritten) = weight (1 - SSIM);
 * dL_dimage = -weight dSSIM/dimage, written (accumulate 0) or added (accumulate 1, so
 * that eq. 7 is recogs_loss_l1 with scale (1 - lambda) / count, then this with weight
 * lambda). workspace: device scratch of recogs_dssim_workspace_bytes (9 floats per
 * pixel, then 6 per 16 x 16 tile of the image), 4-byte aligned. The loss is summed in a
 * fixed order (the same bits on every run). INVALID: bad size, flag, pointer or
 * workspace. */
size_t recogs_dssim_workspace_bytes(int32_t width, int32_t height);
recogs_status recogs_loss_dssim(const float *image, const float *target, int32_t width, int32_t height, float weight,
                                float *dL_dimage, int32_t accumulate, float *loss, void *workspace,
                                size_t workspace_bytes, hipStream_t stream);

/* Both terms of the loss of eq. 4 in one pass, with the gradient of eq. 7:
 * loss (device float, overwritten) = l1_scale * sum |y - t| + weight (1 - SSIM) and
 * dL_dimage = l1_scale * sign(y - t) - weight dSSIM/dimage, written (accumulate 0) or
 * added (accumulate 1); eq. 4 with lambda is l1_scale = (1 - lambda) / (3 width height),
 * weight = lambda. Images, SSIM and workspace as for recogs_loss_dssim. The gradient has
 * the bits of recogs_loss_l1 (scale l1_scale) followed by recogs_loss_dssim with
 * accumulate 1; both sums of the loss are taken in a fixed order (the same bits on every
 * run), where recogs_loss_l1 adds its per-workgroup sums atomically. INVALID as for
 * recogs_loss_dssim. */
recogs_status recogs_loss_l1_dssim(const float *image, const float *target, int32_t width, int32_t height,
                                   float l1_scale, float weight, float *dL_dimage, int32_t accumulate, float *loss,
                                   void *workspace, size_t workspace_bytes, hipStream_t stream);

/* One Adam step over `count` float parameters (the optimiser that moves the SH
 * coefficients toward the edited views, Sec. 3.3): m <- beta1 m + (1 - beta1) g,
 * v <- beta2 v + (1 - beta2) g^2, param <- param - lr (m / c1) / (sqrt(v / c2) + eps) with
 * c1 = 1 - beta1^step, c2 = 1 - beta2^step. param, m, v are updated in place (device,
 * caller-owned; m and v start at zero), grad is read; step counts from 1.
 * INVALID: count < 0, step < 1, beta outside [0, 1), eps <= 0, NULL pointer. */
recogs_status recogs_adam_step(float *param, const float *grad, float *m, float *v, int64_t count, float lr,
                               float beta1, float beta2, float eps, int32_t step, hipStream_t stream);

/* recogs_render_backward_sh followed by recogs_adam_step on the scene's SH, fused: the
 * gradient of every coefficient of each Gaussian goes straight into its Adam update
 * (the same arithmetic as the two calls, so the same bits) and never to memory. The
 * scene's SH planes (scene->sh, float32 storage, [3 (deg + 1)^2][stride]) are updated
 * in place; m and v (device float, same layout, zero at step 1) are the moments.
 * Columns n..stride-1 are left untouched. dL_dopacity and dL_dM are written as by
 * recogs_render_backward_sh (overwritten). UNSUPPORTED: storage other than float32;
 * otherwise the errors of the two calls. */
recogs_status recogs_render_backward_sh_adam(const recogs_scene *scene, const recogs_camera *cam,
                                             const recogs_render_opts *opts, const recogs_workspace *ws,
                                             const float *image, const float *dL_dimage, float *dL_dopacity, float *dL_dM,
                                             float *m, float *v, float lr, float beta1, float beta2, float eps,
                                             int32_t step, hipStream_t stream);

/* ---- pixel selection (Sec. 3.2, 3.3) ----------------------------------------- */

/* Unprojection of a 2D selection to a world point cloud (Sec. 3.2, 3D selection).
 * Takes the pixels with mask != 0, keep != 0 (the uniform sample the method draws,
 * e.g. 70% of the selection; keep NULL = every pixel) and depth > 0 (pixels without a
 * surface are skipped), in row-major pixel order, and writes each one's world point
 * X = R^T (m - t), m = d ((x + 1/2 - cx) / fx, (y + 1/2 - cy) / fy, 1), d its depth
 * (camera-space z, as the rough depth map of the render holds it). Device pointers:
 * mask, keep uint8 [H][W]; depth float [H][W]; points float [3][capacity] (planar, the
 * layout of scene means); count uint32 [1] receives the number of selected pixels,
 * which may exceed capacity (points past capacity are not written). workspace: device
 * memory of recogs_unproject_workspace_bytes(W, H) bytes, 4-byte aligned, overwritten.
 * No host synchronisation. INVALID: bad camera, capacity, pointer or workspace. */
size_t recogs_unproject_workspace_bytes(int32_t width, int32_t height);
recogs_status recogs_unproject(const recogs_camera *cam, const uint8_t *mask, const uint8_t *keep, const float *depth,
                               float *points, int64_t capacity, uint32_t *count, void *workspace,
                               size_t workspace_bytes, hipStream_t stream);

/* recogs_unproject for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same arguments,
 * results and errors, without the workspace. Its per-workgroup counts live in a fixed
 * device array of the library (256 KB on each GPU it runs on, held until the process
 * ends), which covers images of at most 67,108,864 pixels (e.g. 8192 x 8192); larger
 * images are refused with INVALID before any launch. The call allocates nothing and every
 * count it uses is written before it is read, so nothing carries over between calls; but
 * all calls on one GPU share the array, so calls that overlap in time on one GPU (other
 * streams or threads) race and must be serialised by the caller. HIP: the array's device
 * address could not be obtained. */
recogs_status recogs_unproject_noalloc(const recogs_camera *cam, const uint8_t *mask, const uint8_t *keep,
                                       const float *depth, float *points, int64_t capacity, uint32_t *count,
                                       hipStream_t stream);

/* A point cloud drawn into a view as its selection mask (Sec. 3.2: the cloud is drawn
 * as screen-space squares of one size, depth-tested against the rough depth map;
 * Sec. 3.3: the mask of each training view). Point i (points float [3][stride], n of
 * them) at m = R X + t is skipped when m_z <= znear; otherwise the square of side
 * quad_px around (u, v) = (fx m_x / m_z + cx, fy m_y / m_z + cy) covers the pixels whose
 * centres lie in [u - quad_px/2, u + quad_px/2) x [v - quad_px/2, v + quad_px/2), and a
 * covered pixel is marked where depth (float [H][W], or NULL = no test) is 0 or
 * m_z <= depth (1 + depth_eps). mask uint8 [H][W] is overwritten: 1 marked, 0 not.
 * INVALID: bad camera, n < 0, stride < n, quad_px not in (0, 64], depth_eps < 0, NULL
 * pointer. */
recogs_status recogs_reproject_mask(const recogs_camera *cam, const float *points, int64_t n, int64_t stride,
                                    float quad_px, const float *depth, float depth_eps, uint8_t *mask,
                                    hipStream_t stream);

/* The edit of Sec. 3.3 (eq. 6's colour filter on pixels): out = t c per channel where
 * mask != 0, c elsewhere. image, out float [pixels][3] (HWC; out may be image); mask
 * uint8 [pixels]; t: host float [3], read during the call. INVALID: pixels < 0, NULL
 * pointer, t not finite. */
recogs_status recogs_tint(const float *image, const uint8_t *mask, const float t[3], float *out, int64_t pixels,
                          hipStream_t stream);

/* Statistical outlier removal of the unprojected cloud (Sec. 3.2, Fig. 2 caption: the
 * mean distance to 16 neighbours, a standard-deviation scale of 0.007). For each of
 * the n points (points float [3][stride], finite coordinates) D_i = mean Euclidean
 * distance to its k nearest other points (to all others when n - 1 < k; 0 when n = 1);
 * with mu and sigma the mean and population standard deviation of D over the cloud,
 * point i is kept iff D_i <= mu + std_ratio sigma. Outputs (device, overwritten):
 * mean_dist float [n] = D; keep uint8 [n] (1 kept); out_count uint32 [1] = kept count;
 * out_points float [3][out_stride] (NULL = no compaction) = the kept points in input
 * order. The nearest neighbours are exact (a hashed-grid search with a whole-cloud
 * scan for points far from the rest). workspace: recogs_outlier_workspace_bytes(n)
 * bytes of device memory, 256-byte aligned, overwritten. No host synchronisation.
 * INVALID: n < 0, stride < n, out_stride < n, std_ratio < 0, NULL pointer, workspace
 * too small or misaligned; UNSUPPORTED: k not one of 4, 8, 16, 32. */
size_t recogs_outlier_workspace_bytes(int64_t n);
recogs_status recogs_remove_outliers(const float *points, int64_t n, int64_t stride, int32_t k, float std_ratio,
                                     float *mean_dist, uint8_t *keep, float *out_points, int64_t out_stride,
                                     uint32_t *out_count, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- batched form ------------------------------------------------------------ */

/* One render of a batch (host struct): a scene, a camera, an optional fused recolour
 * (device mask uint8 [scene.n], M float [9], b float [3]; all NULL = none) and the
 * output image float [H][W][3] (device). Views may share scenes. */
typedef struct {
    recogs_scene scene;
    recogs_camera cam;
    const uint8_t *mask;
    const float *M;
    const float *b;
    float *image;
} recogs_batch_view;

/* Batch workspace: device memory carved by recogs_batch_init (filled by the library). */
typedef struct {
    void *base;
    size_t bytes;
    int32_t nviews, tile_w, tile_h, px_per_thread;
    int32_t storage, sh_degree;
    int64_t pairs;               /* sum over views of the scene sizes */
    int64_t tiles;               /* sum over views of the tile counts */
    int64_t key_capacity;
    int32_t tile_bits;           /* significant bits of the global tile ids */
    int32_t persistent_blocks;   /* workgroups of the persistent blend */
    uint32_t preprocess_blocks;
    int32_t reserved;
    size_t off_views, off_vtab, off_rec, off_zbits, off_rect, off_count, off_offset;
    size_t off_dkeys0, off_dkeys1, off_dvals0, off_dvals1, off_scan, off_esum, off_efirst, off_sort_count;
    size_t off_keys0, off_keys1, off_vals0, off_vals1, off_header, off_hist, off_dhist, off_ranges, off_order;
    size_t scan_chunks;
    /* filled by recogs_batch_readback */
    int64_t num_keys;            /* keys the batch needs */
    int64_t num_visible;         /* (view, Gaussian) pairs with keys */
    int32_t overflow;            /* 1: num_keys > key_capacity, nothing was rendered */
    int32_t sorted_in_alt;
} recogs_batch_workspace;

/* Bytes for a batch of these views with the given tile shape and key capacity
 * (0 on invalid arguments). */
size_t recogs_batch_workspace_bytes(const recogs_batch_view *views /* host [nviews] */, int32_t nviews,
                                    int32_t tile_w, int32_t tile_h, int64_t key_capacity);

/* Carve dev_mem for the batch and upload its view table (a synchronous copy; the views'
 * device pointers are captured here and used by every recogs_render_batch call).
 * opts: tile shape, px_per_thread and background; all views must share the storage
 * dtype and SH degree of their scenes. Errors: INVALID / UNSUPPORTED / HIP. */
recogs_status recogs_batch_init(recogs_batch_workspace *ws, void *dev_mem, size_t bytes,
                                const recogs_batch_view *views, int32_t nviews, const recogs_render_opts *opts,
                                int64_t key_capacity);

/* Render every view of the batch (an analog of the paper's concurrent editor streams,
 * Sec. 4): one preprocess over all (view, Gaussian) pairs, one count scan, one depth
 * sort, one emission of global tile keys, one tile sort, one persistent blend whose
 * workgroups take tiles largest-list-first from an atomic queue. Enqueues work only:
 * no host synchronisation, no allocation, no memset nodes -- the call can be captured
 * in a HIP graph and replayed. When the keys exceed the capacity nothing is drawn and
 * the overflow flag is set (see recogs_batch_readback). */
recogs_status recogs_render_batch(const recogs_batch_workspace *ws, hipStream_t stream);

/* Synchronises `stream` and reads the key count and overflow flag of the last batch. */
recogs_status recogs_batch_readback(recogs_batch_workspace *ws, hipStream_t stream);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *recogs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RECOGS_H */
