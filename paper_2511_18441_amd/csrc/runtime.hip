// Host side of the C ABI declared in include/recogs.h: argument validation,
// workspace carving and the launch sequence of each call.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "optim_device.hpp"

namespace recogs {
// launchers (kernels_*.hip)
void launch_covariance(const float *, const float *, float *, int64_t, int64_t, hipStream_t);
void launch_select(int, const SceneDev &, const CamDev &, const recogs_select_params &, uint8_t *, int32_t *, hipStream_t);
void launch_recolor(int, const SceneDev &, int, void *, const uint8_t *, const float *, const float *, int, hipStream_t);
void launch_fill_u32(uint32_t *, uint32_t, int64_t, hipStream_t);
void launch_fill_u32_dyn(uint32_t *, uint32_t, const uint32_t *, uint32_t, int64_t, hipStream_t);
void launch_preprocess(int, int, const SceneDev &, const CamDev &, const RecolorDev &, int, SplatRec *, float4 *,
                       uint32_t *, uint2 *, uint32_t *, hipStream_t, uint32_t *, int64_t);
void launch_scan(const uint32_t *, const uint32_t *, uint32_t *, int64_t, uint64_t *, uint32_t *, uint32_t *, uint32_t *,
                 uint32_t *, uint32_t *, uint32_t *, int64_t, hipStream_t, const ScanEmit *, const ScanSort * = nullptr);
void launch_emit(const uint32_t *, const uint32_t *, const uint2 *, const uint32_t *, int64_t, int, uint64_t *, uint32_t *,
                 hipStream_t);
void launch_emit_compacted(const uint32_t *, uint32_t, const uint2 *, const uint32_t *, const uint32_t *, uint32_t, int,
                           uint32_t *, uint32_t *, hipStream_t, const uint32_t *, const uint32_t *, const uint32_t *,
                           const uint4 *, int, const KeyCount * = nullptr);
void launch_tile_depth_sort(const uint2 *, uint32_t, uint32_t *, const uint32_t *, const uint32_t *, uint32_t *, uint32_t *,
                            hipStream_t);
void launch_emit_sorted(const uint32_t *, uint32_t, const uint2 *, uint2 *, int, uint32_t *, uint32_t *, uint32_t *,
                        uint32_t, uint32_t *, uint32_t *, hipStream_t, const uint32_t *, const uint32_t *,
                        const uint32_t *, const uint4 *, int, int = 0, const KeyCount * = nullptr);
uint32_t emit_blocks(uint32_t K);
size_t sort_count_words(uint64_t K_max);
void launch_ranges(const uint64_t *, uint32_t, uint2 *, hipStream_t);
void launch_ranges32(const uint32_t *, uint32_t, uint2 *, hipStream_t, const uint32_t *);
bool launch_blend(int, int, int, int, const uint2 *, const uint32_t *, const SplatRec *, int, int, int, const float *,
                  float *, int, float *, uint32_t *, const uint32_t *, float, float *, hipStream_t);
int sort_passes(int total_bits);
int radix_sort_tile_depth64(uint64_t *, uint32_t *, uint64_t *, uint32_t *, uint32_t, uint32_t, int, int, uint32_t *,
                            uint32_t *, hipStream_t);
int radix_sort_u32(uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t, uint32_t, int, uint32_t *, uint32_t *,
                   hipStream_t, const EmitFold * = nullptr, bool = false);
bool launch_blend_bwd(int, int, int, int, const uint2 *, const uint32_t *, const SplatRec *, const uint2 *, const uint32_t *,
                      int, int, int, const float *, const float *, const uint32_t *, float4 *, hipStream_t);
void launch_grad_finish(const float4 *, const uint32_t *, const float4 *, const uint32_t *, int64_t, const float *, float *,
                        float *, float *, float *, int, const float *, int64_t, const CamDev &, int, hipStream_t, float *,
                        float *, float *, const AdamArgs *, uint64_t, const uint32_t *);
uint32_t bwd_blocks(int, int, int);
bool launch_blend_bwd_blocks(int, int, int, int, const uint2 *, const uint32_t *, const SplatRec *, const uint2 *,
                             const uint32_t *, int, int, int, const float *, const float *, const uint32_t *, float4 *,
                             ulonglong2 *, uint32_t, uint32_t, float4 *, hipStream_t);
void launch_loss_l2(const float *, const float *, int64_t, float, float *, float *, hipStream_t);
void launch_loss_l1(const float *, const float *, int64_t, float, float *, float *, hipStream_t);
void launch_adam(float *, const float *, float *, float *, int64_t, float, float, float, float, float, float, hipStream_t);
void launch_dssim(const float *, const float *, int, int, float, float *, int, float *, float *, hipStream_t, int, float);
size_t dssim_scratch_floats(int, int);
uint32_t unproject_blocks(int64_t);
int64_t unproject_scratch_max_pixels();
uint32_t *unproject_scratch_ptr(hipError_t *);
void launch_unproject(const CamDev &, const uint8_t *, const uint8_t *, const float *, int64_t, uint32_t *, uint32_t *,
                      float *, int64_t, hipStream_t);
void launch_reproject(const CamDev &, const float *, int64_t, int64_t, float, const float *, float, uint8_t *, hipStream_t);
void launch_tint(const float *, const uint8_t *, const float *, float *, int64_t, hipStream_t);
size_t outlier_workspace_bytes(int64_t);
bool launch_outliers(const float *, int64_t, int64_t, int, float, float *, uint8_t *, float *, int64_t, uint32_t *, void *,
                     hipStream_t);
int radix_sort_u32_dyn(uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t, const uint32_t *, const uint32_t *, int,
                       uint32_t *, uint32_t *, hipStream_t, const EmitFold * = nullptr, int = 0, bool = false,
                       bool = false);
KeyCount key_sort_first_count(uint32_t *, uint32_t, int);
void launch_preprocess_batch(int, int, uint32_t, const ViewDev *, int, SplatRec *, uint32_t *, uint2 *, uint32_t *,
                             hipStream_t);
void launch_tile_order(const uint2 *, uint32_t, uint32_t *, uint32_t *, uint32_t *, hipStream_t);
bool launch_blend_persistent(int, int, int, uint32_t, const ViewDev *, int, const uint2 *, const uint32_t *,
                             const SplatRec *, const uint32_t *, uint32_t, uint32_t *, hipStream_t);
}  // namespace recogs

using namespace recogs;

namespace {

thread_local char g_err[512] = "";

recogs_status fail(recogs_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

recogs_status hip_check(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RECOGS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return RECOGS_OK;
}

#define RECOGS_TRY_HIP(call)                                                                          \
    do {                                                                                              \
        const hipError_t _e = (call);                                                                 \
        if (_e != hipSuccess) return fail(RECOGS_ERR_HIP, "%s: %s", #call, hipGetErrorString(_e));     \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool tile_supported(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 32 && th == 8) || (tw == 32 && th == 16) ||
           (tw == 32 && th == 32);
}

// Computes every offset of the workspace; returns total bytes.
size_t layout(recogs_workspace *ws, int64_t n, int32_t W, int32_t H, int32_t tw, int32_t th, int64_t cap) {
    const int64_t tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    const int64_t T = tiles_x * tiles_y;
    const int64_t P = (int64_t)W * H;
    const int64_t nn = n > 0 ? n : 1;
    const int64_t scan_chunks = (nn + kScanChunk - 1) / kScanChunk;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
    ws->off_rec = take(sizeof(SplatRec) * nn);
    ws->off_bwd = take(sizeof(float4) * nn);
    ws->off_gpart = take(sizeof(float) * 9 * (size_t)((nn + 255) / 256));
    ws->off_zbits = take(4 * nn);
    ws->off_rect = take(8 * nn);
    ws->off_count = take(4 * nn);
    ws->off_offset = take(4 * nn);
    ws->off_keys0 = take(8 * (size_t)(cap > 0 ? cap : 1));
    ws->off_keys1 = take(8 * (size_t)(cap > 0 ? cap : 1));
    ws->off_vals0 = take(4 * (size_t)(cap > 0 ? cap : 1));
    ws->off_vals1 = take(4 * (size_t)(cap > 0 ? cap : 1));
    ws->off_final_T = take(4 * (size_t)P);
    ws->off_nproc = take(4 * (size_t)P);
    ws->off_dkeys0 = take(4 * nn);
    ws->off_dkeys1 = take(4 * nn);
    ws->off_dvals0 = take(4 * nn);
    ws->off_dvals1 = take(4 * nn);
    // scan partials per chunk: key count (u64), count with keys, depth min, depth max
    ws->off_scan = take(20 * (size_t)scan_chunks);
    ws->off_efirst = take(4 * ((size_t)emit_blocks((uint32_t)(cap > 0 ? cap : 1)) + 1));
    // radix digit-count matrix [256][chunks], shared by the depth sort (up to n keys) and
    // the key sort (up to cap keys)
    ws->off_sort_count = take(4 * std::max(sort_count_words((uint64_t)nn), sort_count_words((uint64_t)(cap > 0 ? cap : 1))));
    // zeroed each render: header; histograms; key counts of the depth-ordered emission
    // chunks (summed by the depth sort's last pass); tile ranges
    ws->off_header = take(4 * H_WORDS);
    ws->off_hist = take(4 * 256 * kMaxPasses);
    ws->off_dhist = take(4 * 256 * kMaxPasses);
    ws->off_esum = take(4 * (size_t)((nn + kEmitChunk - 1) / kEmitChunk));
    ws->off_ranges = take(8 * (size_t)T);
    ws->scan_chunks = (size_t)scan_chunks;
    ws->sort_chunks = std::max(sort_count_words((uint64_t)nn), sort_count_words((uint64_t)(cap > 0 ? cap : 1))) / 256;
    ws->tiles_x = (int32_t)tiles_x;
    ws->tiles_y = (int32_t)tiles_y;
    return o;
}

template <typename T> T *at(const recogs_workspace *ws, size_t off) { return (T *)((char *)ws->base + off); }

// Stage timing. Mode 1 uses the thread's own events and waits for the blend; mode 2
// brackets the blend with one of the workspace's two event pairs, does not wait, and
// harvests the other pair (recorded by the previous call, complete once this call's
// read-back returned).
// Stage events: 0 start, then the end of [0] preprocess, [1] scan, [2] key-count read-back,
// [3] depth sort, [4] key emission, [5] key sort, [6] tile ranges, [7] per-tile depth sort,
// [8] blend (kStages stages, kStages + 1 events; the blend is the last).
constexpr int kStages = 9;
constexpr int kBlendStage = kStages - 1;
struct ProfileSet {
    hipEvent_t ev[kStages + 1];
    bool pending;
};
struct ProfileState {
    ProfileSet set[2];
    int cur;
};

void harvest(recogs_workspace *ws, ProfileSet &p) {
    if (!p.pending) return;
    p.pending = false;
    if (hipEventSynchronize(p.ev[kBlendStage + 1]) != hipSuccess) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.ev[kBlendStage], p.ev[kBlendStage + 1]) == hipSuccess)
        ws->stage_ms_sum[kBlendStage] += ms;
    ws->profiled_frames += 1;
}

struct StageTimer {
    hipEvent_t own[kStages + 1] = {};
    bool own_ready = false;
    hipEvent_t *ev = nullptr;
    ProfileSet *set = nullptr;
    int mode = 0;
    hipStream_t st = nullptr;
    recogs_status start(int m, recogs_workspace *ws, hipStream_t s) {
        mode = m;
        st = s;
        set = nullptr;
        if (mode == 0) return RECOGS_OK;
        if (mode == 1) {
            if (!own_ready) {
                for (auto &e : own)
                    if (hipEventCreate(&e) != hipSuccess) return fail(RECOGS_ERR_HIP, "hipEventCreate failed");
                own_ready = true;
            }
            ev = own;
            return mark(0);
        }
        ProfileState *ps = (ProfileState *)ws->profile_state;
        if (!ps) {
            ps = (ProfileState *)calloc(1, sizeof(ProfileState));
            if (!ps) return fail(RECOGS_ERR_INVALID, "host allocation of profile state failed");
            for (auto &ps_set : ps->set)
                for (auto &e : ps_set.ev)
                    if (hipEventCreate(&e) != hipSuccess) return fail(RECOGS_ERR_HIP, "hipEventCreate failed");
            ws->profile_state = ps;
        }
        set = &ps->set[ps->cur];
        harvest(ws, *set);  // left over from two calls ago (normally already harvested)
        ev = set->ev;
        return RECOGS_OK;
    }
    // mode 2 records only the blend's bracket: each event between two kernels delays the
    // second one's dispatch by a few microseconds
    recogs_status mark(int k) {
        if (mode == 0 || (mode == 2 && k < kBlendStage)) return RECOGS_OK;
        if (hipEventRecord(ev[k], st) != hipSuccess) return fail(RECOGS_ERR_HIP, "hipEventRecord failed");
        return RECOGS_OK;
    }
    // after the key-count read-back: the previous mode-2 call has completed
    void after_readback(recogs_workspace *ws) {
        if (mode != 2) return;
        ProfileState *ps = (ProfileState *)ws->profile_state;
        harvest(ws, ps->set[ps->cur ^ 1]);
    }
    recogs_status finish(recogs_workspace *ws, int last) {
        if (mode == 2) {
            ProfileState *ps = (ProfileState *)ws->profile_state;
            set->pending = true;
            ps->cur ^= 1;
            return RECOGS_OK;
        }
        if (mode != 1) return RECOGS_OK;
        if (hipEventSynchronize(ev[last]) != hipSuccess) return fail(RECOGS_ERR_HIP, "hipEventSynchronize failed");
        for (int k = 0; k < kStages; ++k) {
            float ms = 0.f;
            if (k < last && hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) ms = 0.f;
            ws->stage_ms[k] = ms;
        }
        return RECOGS_OK;
    }
};
thread_local StageTimer g_timer;

recogs_status check_scene(const recogs_scene *sc) {
    if (!sc) return fail(RECOGS_ERR_INVALID, "scene is NULL");
    if (sc->n < 0) return fail(RECOGS_ERR_INVALID, "scene n = %lld < 0", (long long)sc->n);
    if (sc->n > 0x3fffffffLL) return fail(RECOGS_ERR_UNSUPPORTED, "scene n = %lld exceeds 2^30-1", (long long)sc->n);
    if (sc->stride < sc->n) return fail(RECOGS_ERR_INVALID, "scene stride %lld < n %lld", (long long)sc->stride, (long long)sc->n);
    if (sc->sh_degree < 0 || sc->sh_degree > 3) return fail(RECOGS_ERR_INVALID, "sh_degree %d not in 0..3", sc->sh_degree);
    if (sc->storage < RECOGS_F32 || sc->storage > RECOGS_BF16) return fail(RECOGS_ERR_INVALID, "storage dtype %d unknown", sc->storage);
    if (sc->n > 0 && (!sc->means || !sc->opacity || !sc->sh))
        return fail(RECOGS_ERR_INVALID, "scene means/opacity/sh pointer is NULL");
    return RECOGS_OK;
}

recogs_status check_camera(const recogs_camera *c) {
    if (!c) return fail(RECOGS_ERR_INVALID, "camera is NULL");
    if (c->width <= 0 || c->height <= 0 || c->width > 32768 || c->height > 32768)
        return fail(RECOGS_ERR_INVALID, "image size %dx%d out of range 1..32768", c->width, c->height);
    if (!(c->fx > 0.f) || !(c->fy > 0.f) || !std::isfinite(c->fx) || !std::isfinite(c->fy))
        return fail(RECOGS_ERR_INVALID, "focal lengths must be finite and > 0");
    if (!std::isfinite(c->cx) || !std::isfinite(c->cy) || !std::isfinite(c->znear))
        return fail(RECOGS_ERR_INVALID, "principal point / znear not finite");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(c->R[k])) return fail(RECOGS_ERR_INVALID, "camera R not finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->t[k])) return fail(RECOGS_ERR_INVALID, "camera t not finite");
    return RECOGS_OK;
}

CamDev make_cam(const recogs_camera &c, int tw, int th, int extent_rule = 0) {
    CamDev d;
    d.extent_rule = extent_rule;
    for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy; d.znear = c.znear;
    d.limx = kFrustumClamp * (0.5f * (float)c.width) / c.fx;
    d.limy = kFrustumClamp * (0.5f * (float)c.height) / c.fy;
    // camera centre -R^T t, in double then rounded
    for (int k = 0; k < 3; ++k)
        d.campos[k] = (float)(-((double)c.R[0 * 3 + k] * c.t[0] + (double)c.R[1 * 3 + k] * c.t[1] + (double)c.R[2 * 3 + k] * c.t[2]));
    d.W = c.width; d.H = c.height; d.tw = tw; d.th = th;
    d.tiles_x = (c.width + tw - 1) / tw;
    d.tiles_y = (c.height + th - 1) / th;
    return d;
}

SceneDev make_scene(const recogs_scene &s) {
    SceneDev d;
    d.n = s.n; d.stride = s.stride; d.means = s.means; d.cov3d = s.cov3d; d.opacity = s.opacity; d.sh = s.sh;
    return d;
}

int bits_for(uint64_t v) {  // bits needed to represent values 0..v
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

recogs_status check_opts(const recogs_render_opts *o) {
    if (!o) return fail(RECOGS_ERR_INVALID, "render opts is NULL");
    if (!tile_supported(o->tile_w, o->tile_h))
        return fail(RECOGS_ERR_UNSUPPORTED, "tile %dx%d not one of 16x16, 8x8, 32x8, 32x16, 32x32", o->tile_w, o->tile_h);
    if (o->sort_mode < 0 || o->sort_mode > 2) return fail(RECOGS_ERR_INVALID, "sort_mode %d not 0, 1 or 2", o->sort_mode);
    if (o->graph_mode != 0 && o->graph_mode != 1) return fail(RECOGS_ERR_INVALID, "graph_mode %d not 0 or 1", o->graph_mode);
    if (o->graph_mode && o->sort_mode == 1) return fail(RECOGS_ERR_UNSUPPORTED, "graph_mode needs sort_mode 0 or 2");
    if (o->graph_mode && o->profile_stages == 1)
        return fail(RECOGS_ERR_UNSUPPORTED, "graph_mode renders do not wait: use profile_stages 0 or 2");
    if (o->profile_stages < 0 || o->profile_stages > 2)
        return fail(RECOGS_ERR_INVALID, "profile_stages %d not 0, 1 or 2", o->profile_stages);
    if (o->px_per_thread != 1 && o->px_per_thread != 2 && o->px_per_thread != 4)
        return fail(RECOGS_ERR_UNSUPPORTED, "px_per_thread %d not one of 1, 2, 4", o->px_per_thread);
    if (o->output_chw != 0 && o->output_chw != 1) return fail(RECOGS_ERR_INVALID, "output_chw %d not 0 or 1", o->output_chw);
    if (o->extent_rule != 0 && o->extent_rule != 1) return fail(RECOGS_ERR_INVALID, "extent_rule %d not 0 or 1", o->extent_rule);
    if (o->depth_map && !region_shape(o->tile_w, o->tile_h, o->px_per_thread))
        return fail(RECOGS_ERR_UNSUPPORTED, "depth_map needs tile_h a multiple of 8 * px_per_thread (%dx%d, %d)",
                    o->tile_w, o->tile_h, o->px_per_thread);
    if (o->depth_map && !(o->depth_tau > 0.f && o->depth_tau <= 1.f))
        return fail(RECOGS_ERR_INVALID, "depth_tau %g not in (0, 1]", (double)o->depth_tau);
    const bool any = o->mask || o->M || o->b;
    if (any && !(o->mask && o->M && o->b)) return fail(RECOGS_ERR_INVALID, "fused recolour needs mask, M and b together");
    return RECOGS_OK;
}

recogs_status check_ws(const recogs_workspace *ws, const recogs_scene *sc, const recogs_camera *cam,
                       const recogs_render_opts *o) {
    if (!ws || !ws->base) return fail(RECOGS_ERR_INVALID, "workspace is NULL or not initialised");
    if (sc->n > ws->n_cap) return fail(RECOGS_ERR_INVALID, "scene n %lld > workspace capacity %lld", (long long)sc->n, (long long)ws->n_cap);
    if (cam->width != ws->width || cam->height != ws->height)
        return fail(RECOGS_ERR_INVALID, "camera %dx%d != workspace %dx%d", cam->width, cam->height, ws->width, ws->height);
    if (o->tile_w != ws->tile_w || o->tile_h != ws->tile_h)
        return fail(RECOGS_ERR_INVALID, "tile %dx%d != workspace tile %dx%d", o->tile_w, o->tile_h, ws->tile_w, ws->tile_h);
    return RECOGS_OK;
}

}  // namespace

// The rest of a render in graph mode: no host synchronisation. Counts, the depth
// minimum, the capacity decision and the overflow flag stay in the workspace header;
// grids are sized for n Gaussians and key_capacity keys and workgroups past the live
// counts return at once (sort mode 0, all 32 depth bits above the minimum).
static recogs_status render_async(const recogs_scene *scene, const recogs_camera *cam, const recogs_render_opts *opts,
                                  recogs_workspace *ws, float *image, hipStream_t stream, const CamDev &cd,
                                  StageTimer &tm) {
    recogs_status s;
    const int64_t n = scene->n;
    const int ntiles = cd.tiles_x * cd.tiles_y;
    const uint32_t cap = (uint32_t)ws->key_capacity;
    const int mode = opts->sort_mode;
    uint32_t *hdr = at<uint32_t>(ws, ws->off_header);
    uint32_t *dk0 = at<uint32_t>(ws, ws->off_dkeys0), *dk1 = at<uint32_t>(ws, ws->off_dkeys1);
    uint32_t *dv0 = at<uint32_t>(ws, ws->off_dvals0), *dv1 = at<uint32_t>(ws, ws->off_dvals1);
    uint32_t *t0 = at<uint32_t>(ws, ws->off_keys0), *t1 = at<uint32_t>(ws, ws->off_keys1);
    uint32_t *v0 = at<uint32_t>(ws, ws->off_vals0), *v1 = at<uint32_t>(ws, ws->off_vals1);
    uint32_t *hist = at<uint32_t>(ws, ws->off_hist), *dhist = at<uint32_t>(ws, ws->off_dhist);
    uint32_t *scount = at<uint32_t>(ws, ws->off_sort_count);
    uint2 *ranges = at<uint2>(ws, ws->off_ranges);
    const int tbits = bits_for((uint64_t)(ntiles - 1));
    ws->num_keys = -1;   // known after recogs_workspace_readback
    ws->num_visible = -1;
    ws->last_n = (int32_t)n;
    ws->sort_mode = mode;
    ws->depth_bits = 32;
    ws->depth_min_bits = 0;
    ws->key_bits = tbits + 32;
    ws->sort_passes = sort_passes(tbits);
    ws->depth_passes = mode == 0 ? sort_passes(24) : 0;   // after the scan's pass
    ws->key_bytes = 4;
    int alt = 0;
    if (n > 0 && cap > 0) {
        // the emission counts the key sort's first digit (KeyCount)
        const KeyCount kc = key_sort_first_count(scount, cap, tbits);
        if (mode == 0) {
            // the depth order's rectangles go to keys1, free until the key sort (cap entries;
            // past them the view overflows and emits nothing)
            uint2 *srect = (uint2 *)t1;
            const EmitFold ef{at<uint2>(ws, ws->off_rect), srect, at<uint32_t>(ws, ws->off_esum), cap};
            // the scan left the pairs ordered by their low 8 depth bits in dkeys1 (digit
            // totals in dhist[0..255]); three passes over the upper 24 bits remain
            // (the passes load their chunks below n before the live count V arrives: at worst
            // the n - V pairs past it are read for nothing)
            const int dalt = radix_sort_u32_dyn(dk1, dv1, dk0, dv0, (uint32_t)n, hdr + H_V, nullptr, 24, dhist + 256,
                                                scount, stream, &ef, 8, false, true);
            uint32_t *order = dalt ? dv0 : dv1, *spare = dalt ? dv1 : dv0;
            if ((s = tm.mark(4)) != RECOGS_OK) return s;
            launch_emit_sorted(order, (uint32_t)n, at<uint2>(ws, ws->off_rect), srect, cd.tiles_x,
                               at<uint32_t>(ws, ws->off_esum), spare, at<uint32_t>(ws, ws->off_efirst), cap, t0, v0, stream,
                               hdr + H_V, hdr + H_KEFF, hdr, nullptr, 1, 1, &kc);
        } else {
            if ((s = tm.mark(4)) != RECOGS_OK) return s;
            launch_emit_compacted(dv0, (uint32_t)n, (const uint2 *)dk0, dv1, at<uint32_t>(ws, ws->off_efirst), cap,
                                  cd.tiles_x, t0, v0, stream, hdr + H_V, hdr + H_KEFF, hdr, nullptr, 1, &kc);
        }
        if ((s = tm.mark(5)) != RECOGS_OK) return s;
        alt = radix_sort_u32_dyn(t0, v0, t1, v1, cap, hdr + H_KEFF, nullptr, tbits, hist, scount, stream, nullptr, 0, true);
        if ((s = tm.mark(6)) != RECOGS_OK) return s;
        launch_ranges32(alt ? t1 : t0, cap, ranges, stream, hdr + H_KEFF);
        if ((s = tm.mark(7)) != RECOGS_OK) return s;
        if (mode == 2)
            launch_tile_depth_sort(ranges, (uint32_t)ntiles, alt ? v1 : v0, at<uint32_t>(ws, ws->off_zbits), hdr,
                                   alt ? t0 : t1, alt ? v0 : v1, stream);
    } else {
        for (int k = 4; k <= 7; ++k)
            if ((s = tm.mark(k)) != RECOGS_OK) return s;
    }
    if ((s = tm.mark(kBlendStage)) != RECOGS_OK) return s;
    ws->sorted_in_alt = alt;
    if ((s = hip_check("emit/sort/ranges")) != RECOGS_OK) return s;
    if (!launch_blend(opts->tile_w, opts->tile_h, opts->px_per_thread, ntiles, ranges, alt ? v1 : v0,
                      at<SplatRec>(ws, ws->off_rec), cam->width, cam->height, cd.tiles_x, opts->bg, image, opts->output_chw,
                      opts->keep_backward_state ? at<float>(ws, ws->off_final_T) : nullptr,
                      opts->keep_backward_state ? at<uint32_t>(ws, ws->off_nproc) : nullptr,
                      at<uint32_t>(ws, ws->off_zbits), opts->depth_tau, opts->depth_map, stream))
        return fail(RECOGS_ERR_UNSUPPORTED, "no blend kernel for this tile / px_per_thread");
    if ((s = tm.mark(kBlendStage + 1)) != RECOGS_OK) return s;
    if ((s = hip_check("blend")) != RECOGS_OK) return s;
    return tm.finish(ws, kBlendStage + 1);
}

extern "C" {

const char *recogs_last_error(void) { return g_err; }

size_t recogs_workspace_bytes(int64_t n, int32_t width, int32_t height, int32_t tile_w, int32_t tile_h, int64_t key_capacity) {
    if (n < 0 || width <= 0 || height <= 0 || !tile_supported(tile_w, tile_h) || key_capacity < 0) return 0;
    recogs_workspace ws;
    memset(&ws, 0, sizeof(ws));
    return layout(&ws, n, width, height, tile_w, tile_h, key_capacity);
}

recogs_status recogs_workspace_init(recogs_workspace *ws, void *dev_mem, size_t bytes, int64_t n, int32_t width,
                                    int32_t height, int32_t tile_w, int32_t tile_h, int64_t key_capacity) {
    g_err[0] = 0;
    if (!ws || !dev_mem) return fail(RECOGS_ERR_INVALID, "workspace struct or memory is NULL");
    if ((uintptr_t)dev_mem % kAlign) return fail(RECOGS_ERR_INVALID, "workspace memory not 256-byte aligned");
    if (n < 0 || width <= 0 || height <= 0 || key_capacity < 0)
        return fail(RECOGS_ERR_INVALID, "bad workspace sizes");
    if (key_capacity > 0x3fffffffLL) return fail(RECOGS_ERR_UNSUPPORTED, "key capacity above 2^30-1");
    if (!tile_supported(tile_w, tile_h)) return fail(RECOGS_ERR_UNSUPPORTED, "tile %dx%d unsupported", tile_w, tile_h);
    memset(ws, 0, sizeof(*ws));
    const size_t need = layout(ws, n, width, height, tile_w, tile_h, key_capacity);
    if (bytes < need) return fail(RECOGS_ERR_INVALID, "workspace has %zu bytes, needs %zu", bytes, need);
    ws->base = dev_mem;
    ws->bytes = bytes;
    ws->n_cap = n;
    ws->width = width; ws->height = height; ws->tile_w = tile_w; ws->tile_h = tile_h;
    ws->key_capacity = key_capacity;
    return RECOGS_OK;
}

recogs_status recogs_workspace_profile_flush(recogs_workspace *ws) {
    g_err[0] = 0;
    if (!ws) return fail(RECOGS_ERR_INVALID, "workspace is NULL");
    ProfileState *ps = (ProfileState *)ws->profile_state;
    if (!ps) return RECOGS_OK;
    harvest(ws, ps->set[ps->cur]);      // older
    harvest(ws, ps->set[ps->cur ^ 1]);  // latest
    return RECOGS_OK;
}

recogs_status recogs_workspace_readback(recogs_workspace *ws, hipStream_t stream) {
    g_err[0] = 0;
    if (!ws || !ws->base) return fail(RECOGS_ERR_INVALID, "workspace not initialised");
    uint32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    RECOGS_TRY_HIP(hipMemcpyAsync(h, at<uint32_t>(ws, ws->off_header), sizeof(h), hipMemcpyDeviceToHost, stream));
    RECOGS_TRY_HIP(hipStreamSynchronize(stream));
    const bool any = ws->last_n > 0;
    ws->num_keys = any ? (int64_t)((uint64_t)h[H_K_LO] | ((uint64_t)h[H_K_HI] << 32)) : 0;
    ws->num_visible = any ? h[H_V] : 0;
    ws->depth_min_bits = any ? h[H_ZMIN_RAW] : 0;
    return RECOGS_OK;
}

recogs_status recogs_workspace_keys_needed(const recogs_workspace *ws, int64_t *out_keys, hipStream_t stream) {
    g_err[0] = 0;
    if (!ws || !ws->base) return fail(RECOGS_ERR_INVALID, "workspace not initialised");
    if (!out_keys) return fail(RECOGS_ERR_INVALID, "out_keys is NULL");
    if (ws->generation == 0 || ws->last_n == 0) {  // no render yet, or an empty scene
        *out_keys = 0;
        return RECOGS_OK;
    }
    uint32_t h[2] = {0, 0};
    RECOGS_TRY_HIP(hipMemcpyAsync(h, at<uint32_t>(ws, ws->off_header) + H_K_LO, sizeof(h), hipMemcpyDeviceToHost, stream));
    RECOGS_TRY_HIP(hipStreamSynchronize(stream));
    *out_keys = (int64_t)((uint64_t)h[0] | ((uint64_t)h[1] << 32));
    return RECOGS_OK;
}

void recogs_workspace_release(recogs_workspace *ws) {
    if (!ws || !ws->profile_state) return;
    ProfileState *ps = (ProfileState *)ws->profile_state;
    for (auto &st : ps->set)
        for (auto &e : st.ev)
            if (e) (void)hipEventDestroy(e);
    free(ps);
    ws->profile_state = nullptr;
}

recogs_status recogs_prepare_covariance(const float *log_scales, const float *quats, float *cov3d, int64_t n,
                                        int64_t stride, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0 || stride < n) return fail(RECOGS_ERR_INVALID, "n / stride invalid");
    if (n > 0 && (!log_scales || !quats || !cov3d)) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    launch_covariance(log_scales, quats, cov3d, n, stride, stream);
    return hip_check("covariance");
}

recogs_status recogs_select(const recogs_scene *scene, const recogs_camera *cam, const recogs_select_params *params,
                            uint8_t *mask, int32_t *count, hipStream_t stream) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_scene(scene)) != RECOGS_OK) return s;
    if ((s = check_camera(cam)) != RECOGS_OK) return s;
    if (!params || !count || (scene->n > 0 && !mask)) return fail(RECOGS_ERR_INVALID, "params / mask / count is NULL");
    launch_fill_u32((uint32_t *)count, 0u, 1, stream);
    launch_select(scene->storage, make_scene(*scene), make_cam(*cam, 16, 16), *params, mask, count, stream);
    return hip_check("select");
}

recogs_status recogs_recolor(const recogs_scene *scene, void *dst_sh, const uint8_t *mask, const float *M, const float *b,
                             int32_t copy_unselected, hipStream_t stream) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_scene(scene)) != RECOGS_OK) return s;
    if (scene->n > 0 && (!dst_sh || !mask || !M || !b)) return fail(RECOGS_ERR_INVALID, "dst_sh / mask / M / b is NULL");
    const int ncoef = (scene->sh_degree + 1) * (scene->sh_degree + 1);
    launch_recolor(scene->storage, make_scene(*scene), ncoef, dst_sh, mask, M, b, copy_unselected, stream);
    return hip_check("recolor");
}

recogs_status recogs_render(const recogs_scene *scene, const recogs_camera *cam, const recogs_render_opts *opts,
                            recogs_workspace *ws, float *image, hipStream_t stream) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_scene(scene)) != RECOGS_OK) return s;
    if ((s = check_camera(cam)) != RECOGS_OK) return s;
    if ((s = check_opts(opts)) != RECOGS_OK) return s;
    if ((s = check_ws(ws, scene, cam, opts)) != RECOGS_OK) return s;
    if (!image) return fail(RECOGS_ERR_INVALID, "image is NULL");
    if (scene->n > 0 && !scene->cov3d) return fail(RECOGS_ERR_INVALID, "scene cov3d is NULL");

    const int64_t n = scene->n;
    const CamDev cd = make_cam(*cam, opts->tile_w, opts->tile_h, opts->extent_rule);
    const int ntiles = cd.tiles_x * cd.tiles_y;
    uint32_t *hdr = at<uint32_t>(ws, ws->off_header);
    SplatRec *rec = at<SplatRec>(ws, ws->off_rec);
    ++ws->generation;
    float4 *bwd = at<float4>(ws, ws->off_bwd);
    uint32_t *zb = at<uint32_t>(ws, ws->off_zbits);
    uint2 *rect = at<uint2>(ws, ws->off_rect);
    uint32_t *cnt = at<uint32_t>(ws, ws->off_count);
    uint32_t *off = at<uint32_t>(ws, ws->off_offset);
    uint2 *ranges = at<uint2>(ws, ws->off_ranges);

    StageTimer &tm = g_timer;
    for (int k = 0; k < kStages; ++k) ws->stage_ms[k] = 0.f;
    if ((s = tm.start(opts->profile_stages, ws, stream)) != RECOGS_OK) return s;
    const int mode = opts->sort_mode;
    uint32_t *dk0 = at<uint32_t>(ws, ws->off_dkeys0), *dk1 = at<uint32_t>(ws, ws->off_dkeys1);
    uint32_t *dv0 = at<uint32_t>(ws, ws->off_dvals0), *dv1 = at<uint32_t>(ws, ws->off_dvals1);
    // the preprocess launch also zeroes the header, the digit totals, the emission sums
    // and the tile ranges (adjacent)
    RecolorDev rc{opts->mask, opts->M, opts->b};
    launch_preprocess(scene->storage, scene->sh_degree, make_scene(*scene), cd, rc, opts->keep_backward_state, rec, bwd, zb,
                      rect, cnt, stream, hdr, (int64_t)((ws->off_ranges - ws->off_header) / 4) + 2 * (int64_t)ntiles);
    if ((s = tm.mark(1)) != RECOGS_OK) return s;
    {
        const size_t sc_n = ws->scan_chunks;
        uint64_t *pk = at<uint64_t>(ws, ws->off_scan);
        uint32_t *pv = (uint32_t *)(pk + sc_n);
        // tile-first order: the compaction carries rectangles (over both depth-key buffers,
        // adjacent), key offsets (dvals1) and the emission blocks' owners
        const ScanEmit em{rect, (uint2 *)dk0, dv1, at<uint32_t>(ws, ws->off_efirst)};
        // depth-first order: the scan also does the depth sort's first pass, on the low 8
        // raw depth bits (the minimum is not known yet; raw bits give the same order), into
        // dkeys1
        const ScanSort so{at<uint32_t>(ws, ws->off_sort_count), at<uint32_t>(ws, ws->off_dhist), dk1, dv1};
        launch_scan(cnt, zb, off, n, pk, pv, pv + sc_n, pv + 2 * sc_n, dk0, dv0, hdr, ws->key_capacity, stream,
                    mode == 2 ? &em : nullptr, mode == 0 ? &so : nullptr);
    }
    if ((s = tm.mark(2)) != RECOGS_OK) return s;
    if ((s = hip_check("preprocess/scan")) != RECOGS_OK) return s;
    if (opts->graph_mode) return render_async(scene, cam, opts, ws, image, stream, cd, tm);

    uint32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    RECOGS_TRY_HIP(hipMemcpyAsync(h, hdr, sizeof(h), hipMemcpyDeviceToHost, stream));
    RECOGS_TRY_HIP(hipStreamSynchronize(stream));
    tm.after_readback(ws);
    if ((s = tm.mark(3)) != RECOGS_OK) return s;
    const uint64_t K = n > 0 ? ((uint64_t)h[H_K_LO] | ((uint64_t)h[H_K_HI] << 32)) : 0;
    const uint32_t V = n > 0 ? h[H_V] : 0;
    ws->num_keys = (int64_t)K;
    ws->num_visible = V;
    ws->last_n = (int32_t)n;
    ws->sort_mode = mode;
    if ((int64_t)K > ws->key_capacity)
        return fail(RECOGS_ERR_CAPACITY, "view needs %llu tile keys, workspace holds %lld", (unsigned long long)K,
                    (long long)ws->key_capacity);
    const uint32_t zmin = ~h[H_ZMIN], zmax = h[H_ZMAX];
    const int dbits = K ? bits_for((uint64_t)(zmax - zmin)) : 0;
    const int tbits = bits_for((uint64_t)(ntiles - 1));
    const int key_bits = mode == 1 ? tbits + dbits : tbits;
    ws->depth_bits = dbits;
    ws->depth_min_bits = zmin;
    ws->key_bits = tbits + dbits;
    ws->sort_passes = K ? sort_passes(key_bits) : 0;
    // sort mode 0: raw depth bits up to the highest one in which the depths differ; the
    // scan sorted bits 0-7, the depth sort takes the rest
    const int rbits = K ? bits_for((uint64_t)(zmin ^ zmax)) : 0;
    const int rest_bits = rbits > 8 ? rbits - 8 : 0;
    ws->depth_passes = (mode == 0 && V) ? sort_passes(rest_bits) : 0;
    ws->key_bytes = mode == 1 ? 8 : 4;

    // (histograms, emission sums and tile ranges zeroed by the preprocess launch)
    uint32_t *hist = at<uint32_t>(ws, ws->off_hist), *dhist = at<uint32_t>(ws, ws->off_dhist);
    uint32_t *scount = at<uint32_t>(ws, ws->off_sort_count);

    uint64_t *k0 = at<uint64_t>(ws, ws->off_keys0), *k1 = at<uint64_t>(ws, ws->off_keys1);
    uint32_t *v0 = at<uint32_t>(ws, ws->off_vals0), *v1 = at<uint32_t>(ws, ws->off_vals1);
    int alt = 0;
    if (K > 0 && mode == 0) {
        // the rest of the depth sort of the V Gaussians with keys (the scan left them ordered
        // by their low 8 depth bits in dkeys1); its last pass gathers the depth-ordered
        // rectangles (8 bytes each) into keys1, free until the key sort (K <= cap, so
        // V <= cap), and sums the emission chunks' counts
        uint32_t *t0 = (uint32_t *)k0, *t1 = (uint32_t *)k1;
        uint2 *srect = (uint2 *)k1;
        const EmitFold ef{rect, srect, at<uint32_t>(ws, ws->off_esum), (uint32_t)ws->key_capacity};
        const int dalt = radix_sort_u32_dyn(dk1, dv1, dk0, dv0, V, nullptr, nullptr, rest_bits, dhist + 256, scount,
                                            stream, &ef, 8);
        uint32_t *order = dalt ? dv0 : dv1, *spare = dalt ? dv1 : dv0;
        if ((s = tm.mark(4)) != RECOGS_OK) return s;
        // per-Gaussian key offsets go to the depth-value buffer the sort left free; with no
        // pass left (depths equal above bit 7) the emission does its own reduce
        const KeyCount kc = key_sort_first_count(scount, (uint32_t)K, key_bits);
        launch_emit_sorted(order, V, rect, srect, cd.tiles_x, at<uint32_t>(ws, ws->off_esum), spare,
                           at<uint32_t>(ws, ws->off_efirst), (uint32_t)K, t0, v0, stream, nullptr, nullptr, nullptr,
                           nullptr, 1, rest_bits > 0 ? 1 : 0, &kc);
        if ((s = tm.mark(5)) != RECOGS_OK) return s;
        alt = radix_sort_u32(t0, v0, t1, v1, (uint32_t)K, 0u, key_bits, hist, scount, stream, nullptr, true);
        if ((s = tm.mark(6)) != RECOGS_OK) return s;
        launch_ranges32(alt ? t1 : t0, (uint32_t)K, ranges, stream, nullptr);
        if ((s = tm.mark(7)) != RECOGS_OK) return s;
    } else if (K > 0 && mode == 2) {
        // tile-first: keys of the index-ordered compaction, a stable sort by tile, then each
        // tile's list sorted by depth
        uint32_t *t0 = (uint32_t *)k0, *t1 = (uint32_t *)k1;
        if ((s = tm.mark(4)) != RECOGS_OK) return s;
        const KeyCount kc = key_sort_first_count(scount, (uint32_t)K, key_bits);
        launch_emit_compacted(dv0, V, (const uint2 *)dk0, dv1, at<uint32_t>(ws, ws->off_efirst), (uint32_t)K, cd.tiles_x,
                              t0, v0, stream, nullptr, nullptr, nullptr, nullptr, 1, &kc);
        if ((s = tm.mark(5)) != RECOGS_OK) return s;
        alt = radix_sort_u32(t0, v0, t1, v1, (uint32_t)K, 0u, key_bits, hist, scount, stream, nullptr, true);
        if ((s = tm.mark(6)) != RECOGS_OK) return s;
        launch_ranges32(alt ? t1 : t0, (uint32_t)K, ranges, stream, nullptr);
        if ((s = tm.mark(7)) != RECOGS_OK) return s;
        launch_tile_depth_sort(ranges, (uint32_t)ntiles, alt ? v1 : v0, zb, hdr, alt ? t0 : t1, alt ? v0 : v1, stream);
    } else if (K > 0) {
        if ((s = tm.mark(4)) != RECOGS_OK) return s;
        launch_emit(cnt, off, rect, zb, n, cd.tiles_x, k0, v0, stream);
        if ((s = tm.mark(5)) != RECOGS_OK) return s;
        alt = radix_sort_tile_depth64(k0, v0, k1, v1, (uint32_t)K, zmin, dbits, key_bits, hist, scount, stream);
        if ((s = tm.mark(6)) != RECOGS_OK) return s;
        launch_ranges(alt ? k1 : k0, (uint32_t)K, ranges, stream);
        if ((s = tm.mark(7)) != RECOGS_OK) return s;
    } else {
        for (int k = 4; k <= 7; ++k)
            if ((s = tm.mark(k)) != RECOGS_OK) return s;
    }
    if ((s = tm.mark(kBlendStage)) != RECOGS_OK) return s;
    ws->sorted_in_alt = alt;
    if ((s = hip_check("emit/sort/ranges")) != RECOGS_OK) return s;
    if (!launch_blend(opts->tile_w, opts->tile_h, opts->px_per_thread, ntiles, ranges, alt ? v1 : v0, rec, cam->width,
                      cam->height, cd.tiles_x, opts->bg, image, opts->output_chw,
                      opts->keep_backward_state ? at<float>(ws, ws->off_final_T) : nullptr,
                      opts->keep_backward_state ? at<uint32_t>(ws, ws->off_nproc) : nullptr,
                      at<uint32_t>(ws, ws->off_zbits), opts->depth_tau, opts->depth_map, stream))
        return fail(RECOGS_ERR_UNSUPPORTED, "no blend kernel for this tile / px_per_thread");
    if ((s = tm.mark(kBlendStage + 1)) != RECOGS_OK) return s;
    if ((s = hip_check("blend")) != RECOGS_OK) return s;
    return tm.finish(ws, kBlendStage + 1);
}

// The block backward's scratch for this workspace and launch shape: per block of a tile,
// one float4 per key of capacity, then a 16-byte (written flags, count) word per 64 keys
// of capacity and per tile (plus two). 0 bytes: the shape has no block form.
static size_t bwd_flag_stride(const recogs_workspace *ws) {
    return (size_t)ws->key_capacity / 64 + (size_t)ws->tiles_x * (size_t)ws->tiles_y + 2;
}
static size_t backward_scratch_bytes(const recogs_workspace *ws, const recogs_render_opts *o) {
    const uint32_t nr = bwd_blocks(o->tile_w, o->tile_h, o->px_per_thread);
    if (!nr || !ws || ws->key_capacity <= 0) return 0;
    return align_up(16 * (size_t)nr * (size_t)ws->key_capacity) + 16 * (size_t)nr * bwd_flag_stride(ws);
}

// The backward of both entry points: out = dL/dC0 [3][n], or with all_bands
// dL/dSH [3 (deg + 1)^2][scene stride].
static recogs_status backward_impl(const recogs_scene *scene, const recogs_camera *cam, const recogs_render_opts *opts,
                                   const recogs_workspace *ws, const float *image, const float *dL_dimage,
                                   float *dL_dopacity, float *out, float *dL_dM, int32_t accumulate, bool all_bands,
                                   hipStream_t stream, float *am = nullptr, float *av = nullptr,
                                   const AdamArgs *adam = nullptr) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_scene(scene)) != RECOGS_OK) return s;
    if ((s = check_camera(cam)) != RECOGS_OK) return s;
    if ((s = check_opts(opts)) != RECOGS_OK) return s;
    if ((s = check_ws(ws, scene, cam, opts)) != RECOGS_OK) return s;
    if (!opts->keep_backward_state) return fail(RECOGS_ERR_INVALID, "render must keep backward state for the backward");
    if (opts->output_chw) return fail(RECOGS_ERR_UNSUPPORTED, "the backward takes an HWC render (output_chw 0)");
    if (ws->last_n != scene->n) return fail(RECOGS_ERR_INVALID, "workspace holds a render of %d Gaussians, scene has %lld", ws->last_n, (long long)scene->n);
    // after a graph_mode render not read back, the key count stays on the device (no host
    // synchronisation here either); a render that overflowed emitted no key, so every
    // tile list is empty and the gradients are zero
    const bool dyn_keys = ws->num_keys < 0;
    if (ws->num_keys > ws->key_capacity) return fail(RECOGS_ERR_INVALID, "the render overflowed its key capacity");
    if (!image || !dL_dimage || !dL_dM || (scene->n > 0 && (!dL_dopacity || (!out && !adam))))
        return fail(RECOGS_ERR_INVALID, "NULL image / gradient pointer");
    if (accumulate != 0 && accumulate != 1) return fail(RECOGS_ERR_INVALID, "accumulate %d not 0 or 1", accumulate);
    const int64_t n = scene->n;
    const int ntiles = ws->tiles_x * ws->tiles_y;
    const uint32_t *koff = at<uint32_t>(ws, ws->off_offset);
    const uint32_t *vals = ws->sorted_in_alt ? at<uint32_t>(ws, ws->off_vals1) : at<uint32_t>(ws, ws->off_vals0);
    // the block form when the caller gives its scratch, else one workgroup per tile with
    // a barrier per batch of the list
    const uint32_t nr = bwd_blocks(opts->tile_w, opts->tile_h, opts->px_per_thread);
    const bool blocks = opts->bwd_scratch && nr > 0;
    if (blocks && opts->bwd_scratch_bytes < backward_scratch_bytes(ws, opts))
        return fail(RECOGS_ERR_INVALID, "bwd_scratch of %zu bytes, the block backward needs %zu", opts->bwd_scratch_bytes,
                    backward_scratch_bytes(ws, opts));
    if (blocks && (uintptr_t)opts->bwd_scratch % kAlign) return fail(RECOGS_ERR_INVALID, "bwd_scratch not 256-byte aligned");
    // per-(Gaussian, tile) gradient slots, 16 bytes per key: the span of both sorted-key
    // buffers (adjacent, 16 bytes per key of capacity), which the backward does not read
    float4 *gk = at<float4>(ws, ws->off_keys0);
    if (ws->num_keys > 0 || dyn_keys) {
        bool ok;
        if (blocks) {   // writes every slot
            const size_t cap = (size_t)ws->key_capacity;
            float4 *sub = (float4 *)opts->bwd_scratch;
            ulonglong2 *fw = (ulonglong2 *)((char *)opts->bwd_scratch + align_up(16 * (size_t)nr * cap));
            ok = launch_blend_bwd_blocks(opts->tile_w, opts->tile_h, opts->px_per_thread, ntiles,
                                         at<uint2>(ws, ws->off_ranges), vals, at<SplatRec>(ws, ws->off_rec),
                                         at<uint2>(ws, ws->off_rect), koff, cam->width, cam->height, ws->tiles_x, image,
                                         dL_dimage, at<uint32_t>(ws, ws->off_nproc), sub, fw, (uint32_t)cap,
                                         (uint32_t)bwd_flag_stride(ws), gk, stream);
        } else if (dyn_keys) {
            launch_fill_u32_dyn((uint32_t *)gk, 0u, at<uint32_t>(ws, ws->off_header) + H_KEFF, 4u,
                                4 * ws->key_capacity, stream);
            ok = launch_blend_bwd(opts->tile_w, opts->tile_h, opts->px_per_thread, ntiles, at<uint2>(ws, ws->off_ranges),
                                  vals, at<SplatRec>(ws, ws->off_rec), at<uint2>(ws, ws->off_rect), koff, cam->width,
                                  cam->height, ws->tiles_x, image, dL_dimage, at<uint32_t>(ws, ws->off_nproc), gk, stream);
        } else {
            launch_fill_u32((uint32_t *)gk, 0u, 4 * ws->num_keys, stream);
            ok = launch_blend_bwd(opts->tile_w, opts->tile_h, opts->px_per_thread, ntiles, at<uint2>(ws, ws->off_ranges),
                                  vals, at<SplatRec>(ws, ws->off_rec), at<uint2>(ws, ws->off_rect), koff, cam->width,
                                  cam->height, ws->tiles_x, image, dL_dimage, at<uint32_t>(ws, ws->off_nproc), gk, stream);
        }
        if (!ok) return fail(RECOGS_ERR_UNSUPPORTED, "no backward kernel for this tile / px_per_thread");
    }
    const CamDev cd = make_cam(*cam, opts->tile_w, opts->tile_h);
    launch_grad_finish(gk, koff, at<float4>(ws, ws->off_bwd), at<uint32_t>(ws, ws->off_count), n, opts->M, dL_dopacity, out,
                       dL_dM, at<float>(ws, ws->off_gpart), all_bands ? scene->sh_degree : -1, scene->means,
                       scene->stride, cd, accumulate, stream, adam ? (float *)scene->sh : nullptr, am, av, adam,
                       (uint64_t)ws->key_capacity, at<uint32_t>(ws, ws->off_header) + H_OVERFLOW);
    return hip_check("backward");
}

size_t recogs_backward_scratch_bytes(const recogs_workspace *ws, const recogs_render_opts *opts) {
    if (!ws || !opts || !tile_supported(opts->tile_w, opts->tile_h)) return 0;
    return backward_scratch_bytes(ws, opts);
}

recogs_status recogs_render_backward(const recogs_scene *scene, const recogs_camera *cam, const recogs_render_opts *opts,
                                     const recogs_workspace *ws, const float *image, const float *dL_dimage,
                                     float *dL_dopacity, float *dL_dsh_dc, float *dL_dM, int32_t accumulate,
                                     hipStream_t stream) {
    return backward_impl(scene, cam, opts, ws, image, dL_dimage, dL_dopacity, dL_dsh_dc, dL_dM, accumulate, false, stream);
}

recogs_status recogs_render_backward_sh(const recogs_scene *scene, const recogs_camera *cam,
                                        const recogs_render_opts *opts, const recogs_workspace *ws, const float *image,
                                        const float *dL_dimage, float *dL_dopacity, float *dL_dsh, float *dL_dM,
                                        int32_t accumulate, hipStream_t stream) {
    return backward_impl(scene, cam, opts, ws, image, dL_dimage, dL_dopacity, dL_dsh, dL_dM, accumulate, true, stream);
}

recogs_status recogs_render_backward_sh_adam(const recogs_scene *scene, const recogs_camera *cam,
                                             const recogs_render_opts *opts, const recogs_workspace *ws,
                                             const float *image, const float *dL_dimage, float *dL_dopacity, float *dL_dM,
                                             float *m, float *v, float lr, float beta1, float beta2, float eps,
                                             int32_t step, hipStream_t stream) {
    g_err[0] = 0;
    if (!scene) return fail(RECOGS_ERR_INVALID, "scene is NULL");
    if (scene->storage != RECOGS_F32) return fail(RECOGS_ERR_UNSUPPORTED, "the fused Adam step updates float32 SH only");
    if (step < 1) return fail(RECOGS_ERR_INVALID, "step %d < 1", step);
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(RECOGS_ERR_INVALID, "beta1, beta2 must lie in [0, 1) and eps > 0");
    if (scene->n > 0 && (!m || !v)) return fail(RECOGS_ERR_INVALID, "NULL moment pointer");
    const double c1 = 1.0 - std::pow((double)beta1, (double)step), c2 = 1.0 - std::pow((double)beta2, (double)step);
    const AdamArgs a{lr, beta1, beta2, eps, (float)(1.0 / c1), (float)(1.0 / c2)};
    return backward_impl(scene, cam, opts, ws, image, dL_dimage, dL_dopacity, nullptr, dL_dM, 0, true, stream, m, v, &a);
}

recogs_status recogs_loss_l2(const float *image, const float *target, int64_t count, float scale, float *dL_dimage,
                             float *loss, hipStream_t stream) {
    g_err[0] = 0;
    if (count < 0) return fail(RECOGS_ERR_INVALID, "count < 0");
    if (!loss || (count > 0 && (!image || !target || !dL_dimage))) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    launch_fill_u32((uint32_t *)loss, 0u, 1, stream);
    launch_loss_l2(image, target, count, scale, dL_dimage, loss, stream);
    return hip_check("loss_l2");
}

recogs_status recogs_loss_l1(const float *image, const float *target, int64_t count, float scale, float *dL_dimage,
                             float *loss, hipStream_t stream) {
    g_err[0] = 0;
    if (count < 0) return fail(RECOGS_ERR_INVALID, "count < 0");
    if (!loss || (count > 0 && (!image || !target || !dL_dimage))) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    launch_fill_u32((uint32_t *)loss, 0u, 1, stream);
    launch_loss_l1(image, target, count, scale, dL_dimage, loss, stream);
    return hip_check("loss_l1");
}

size_t recogs_dssim_workspace_bytes(int32_t width, int32_t height) {
    return sizeof(float) * dssim_scratch_floats(width, height);
}

recogs_status recogs_loss_dssim(const float *image, const float *target, int32_t width, int32_t height, float weight,
                                float *dL_dimage, int32_t accumulate, float *loss, void *workspace, size_t workspace_bytes,
                                hipStream_t stream) {
    g_err[0] = 0;
    if (width <= 0 || height <= 0) return fail(RECOGS_ERR_INVALID, "image %dx%d", width, height);
    if (accumulate != 0 && accumulate != 1) return fail(RECOGS_ERR_INVALID, "accumulate %d not 0 or 1", accumulate);
    if (!image || !target || !dL_dimage || !loss || !workspace) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    if (workspace_bytes < recogs_dssim_workspace_bytes(width, height))
        return fail(RECOGS_ERR_INVALID, "workspace of %zu bytes, needs %zu", workspace_bytes,
                    recogs_dssim_workspace_bytes(width, height));
    if (reinterpret_cast<uintptr_t>(workspace) % 4) return fail(RECOGS_ERR_INVALID, "workspace not 4-byte aligned");
    launch_dssim(image, target, width, height, weight, dL_dimage, accumulate, loss, (float *)workspace, stream, 0, 0.f);
    return hip_check("loss_dssim");
}

recogs_status recogs_loss_l1_dssim(const float *image, const float *target, int32_t width, int32_t height, float l1_scale,
                                   float weight, float *dL_dimage, int32_t accumulate, float *loss, void *workspace,
                                   size_t workspace_bytes, hipStream_t stream) {
    g_err[0] = 0;
    if (width <= 0 || height <= 0) return fail(RECOGS_ERR_INVALID, "image %dx%d", width, height);
    if (accumulate != 0 && accumulate != 1) return fail(RECOGS_ERR_INVALID, "accumulate %d not 0 or 1", accumulate);
    if (!image || !target || !dL_dimage || !loss || !workspace) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    if (workspace_bytes < recogs_dssim_workspace_bytes(width, height))
        return fail(RECOGS_ERR_INVALID, "workspace of %zu bytes, needs %zu", workspace_bytes,
                    recogs_dssim_workspace_bytes(width, height));
    if (reinterpret_cast<uintptr_t>(workspace) % 4) return fail(RECOGS_ERR_INVALID, "workspace not 4-byte aligned");
    launch_dssim(image, target, width, height, weight, dL_dimage, accumulate, loss, (float *)workspace, stream, 1, l1_scale);
    return hip_check("loss_l1_dssim");
}

recogs_status recogs_adam_step(float *param, const float *grad, float *m, float *v, int64_t count, float lr, float beta1,
                               float beta2, float eps, int32_t step, hipStream_t stream) {
    g_err[0] = 0;
    if (count < 0) return fail(RECOGS_ERR_INVALID, "count < 0");
    if (step < 1) return fail(RECOGS_ERR_INVALID, "step %d < 1", step);
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(RECOGS_ERR_INVALID, "beta1, beta2 must lie in [0, 1) and eps > 0");
    if (count > 0 && (!param || !grad || !m || !v)) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    const double c1 = 1.0 - std::pow((double)beta1, (double)step), c2 = 1.0 - std::pow((double)beta2, (double)step);
    launch_adam(param, grad, m, v, count, lr, beta1, beta2, eps, (float)(1.0 / c1), (float)(1.0 / c2), stream);
    return hip_check("adam_step");
}

size_t recogs_unproject_workspace_bytes(int32_t width, int32_t height) {
    if (width <= 0 || height <= 0) return 0;
    return align_up((size_t)4 * ((size_t)unproject_blocks((int64_t)width * height) + 1));
}

recogs_status recogs_unproject(const recogs_camera *cam, const uint8_t *mask, const uint8_t *keep, const float *depth,
                               float *points, int64_t capacity, uint32_t *count, void *workspace, size_t workspace_bytes,
                               hipStream_t stream) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_camera(cam)) != RECOGS_OK) return s;
    if (capacity < 0 || capacity > 0xffffffffLL) return fail(RECOGS_ERR_INVALID, "capacity %lld not in 0..2^32-1", (long long)capacity);
    if (!mask || !depth || !count || !workspace || (capacity > 0 && !points)) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    if (workspace_bytes < recogs_unproject_workspace_bytes(cam->width, cam->height))
        return fail(RECOGS_ERR_INVALID, "workspace of %zu bytes, needs %zu", workspace_bytes,
                    recogs_unproject_workspace_bytes(cam->width, cam->height));
    if (reinterpret_cast<uintptr_t>(workspace) % 4) return fail(RECOGS_ERR_INVALID, "workspace not 4-byte aligned");
    launch_unproject(make_cam(*cam, 16, 16), mask, keep, depth, (int64_t)cam->width * cam->height, (uint32_t *)workspace,
                     count, points, capacity, stream);
    return hip_check("unproject");
}

recogs_status recogs_unproject_noalloc(const recogs_camera *cam, const uint8_t *mask, const uint8_t *keep,
                                       const float *depth, float *points, int64_t capacity, uint32_t *count,
                                       hipStream_t stream) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_camera(cam)) != RECOGS_OK) return s;
    if (capacity < 0 || capacity > 0xffffffffLL) return fail(RECOGS_ERR_INVALID, "capacity %lld not in 0..2^32-1", (long long)capacity);
    if (!mask || !depth || !count || (capacity > 0 && !points)) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    const int64_t P = (int64_t)cam->width * cam->height;
    if (P > unproject_scratch_max_pixels())
        return fail(RECOGS_ERR_INVALID, "image of %lld pixels exceeds the %lld this call's fixed scratch covers",
                    (long long)P, (long long)unproject_scratch_max_pixels());
    hipError_t e = hipSuccess;
    uint32_t *part = unproject_scratch_ptr(&e);
    if (!part) return fail(RECOGS_ERR_HIP, "device address of the unprojection scratch: %s", hipGetErrorString(e));
    launch_unproject(make_cam(*cam, 16, 16), mask, keep, depth, P, part, count, points, capacity, stream);
    return hip_check("unproject_noalloc");
}

recogs_status recogs_reproject_mask(const recogs_camera *cam, const float *points, int64_t n, int64_t stride,
                                    float quad_px, const float *depth, float depth_eps, uint8_t *mask,
                                    hipStream_t stream) {
    g_err[0] = 0;
    recogs_status s;
    if ((s = check_camera(cam)) != RECOGS_OK) return s;
    if (n < 0 || n > 0x7fffffffLL || stride < n) return fail(RECOGS_ERR_INVALID, "n %lld / stride %lld", (long long)n, (long long)stride);
    if (!(quad_px > 0.f && quad_px <= 64.f)) return fail(RECOGS_ERR_INVALID, "quad_px %g not in (0, 64]", (double)quad_px);
    if (!(depth_eps >= 0.f && std::isfinite(depth_eps))) return fail(RECOGS_ERR_INVALID, "depth_eps %g not finite and >= 0", (double)depth_eps);
    if (!mask || (n > 0 && !points)) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    launch_reproject(make_cam(*cam, 16, 16), points, n, stride, quad_px, depth, depth_eps, mask, stream);
    return hip_check("reproject_mask");
}

recogs_status recogs_tint(const float *image, const uint8_t *mask, const float t[3], float *out, int64_t pixels,
                          hipStream_t stream) {
    g_err[0] = 0;
    if (pixels < 0) return fail(RECOGS_ERR_INVALID, "pixels < 0");
    if (!t || (pixels > 0 && (!image || !mask || !out))) return fail(RECOGS_ERR_INVALID, "NULL pointer");
    if (!std::isfinite(t[0]) || !std::isfinite(t[1]) || !std::isfinite(t[2])) return fail(RECOGS_ERR_INVALID, "tint not finite");
    launch_tint(image, mask, t, out, pixels, stream);
    return hip_check("tint");
}

size_t recogs_outlier_workspace_bytes(int64_t n) {
    if (n < 0 || n > 0x7fffffffLL) return 0;
    return outlier_workspace_bytes(n);
}

recogs_status recogs_remove_outliers(const float *points, int64_t n, int64_t stride, int32_t k, float std_ratio,
                                     float *mean_dist, uint8_t *keep, float *out_points, int64_t out_stride,
                                     uint32_t *out_count, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0 || n > 0x7fffffffLL || stride < n) return fail(RECOGS_ERR_INVALID, "n %lld / stride %lld", (long long)n, (long long)stride);
    if (k != 4 && k != 8 && k != 16 && k != 32) return fail(RECOGS_ERR_UNSUPPORTED, "k = %d not one of 4, 8, 16, 32", k);
    if (!(std_ratio >= 0.f) || !std::isfinite(std_ratio)) return fail(RECOGS_ERR_INVALID, "std_ratio %g not finite and >= 0", (double)std_ratio);
    if (!out_count || !workspace || (n > 0 && (!points || !mean_dist || !keep)))
        return fail(RECOGS_ERR_INVALID, "NULL pointer");
    if (out_points && out_stride < n) return fail(RECOGS_ERR_INVALID, "out_stride %lld < n %lld", (long long)out_stride, (long long)n);
    if (workspace_bytes < outlier_workspace_bytes(n))
        return fail(RECOGS_ERR_INVALID, "workspace of %zu bytes, needs %zu", workspace_bytes, outlier_workspace_bytes(n));
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(RECOGS_ERR_INVALID, "workspace not 256-byte aligned");
    launch_outliers(points, n, stride, k, std_ratio, mean_dist, keep, out_points, out_stride, out_count, workspace, stream);
    return hip_check("remove_outliers");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
namespace {

constexpr int kMaxViews = 4096;

recogs_status check_batch(const recogs_batch_view *views, int32_t nviews) {
    if (!views || nviews <= 0 || nviews > kMaxViews) return fail(RECOGS_ERR_INVALID, "batch of %d views (1..%d)", nviews, kMaxViews);
    char msg[sizeof(g_err)];
    for (int v = 0; v < nviews; ++v) {
        recogs_status s;
        if ((s = check_scene(&views[v].scene)) != RECOGS_OK || (s = check_camera(&views[v].cam)) != RECOGS_OK) {
            memcpy(msg, g_err, sizeof(msg));
            return fail(s, "view %d: %s", v, msg);
        }
        if (views[v].scene.n > 0 && !views[v].scene.cov3d) return fail(RECOGS_ERR_INVALID, "view %d: cov3d is NULL", v);
        if (!views[v].image) return fail(RECOGS_ERR_INVALID, "view %d: image is NULL", v);
        const bool any = views[v].mask || views[v].M || views[v].b;
        if (any && !(views[v].mask && views[v].M && views[v].b))
            return fail(RECOGS_ERR_INVALID, "view %d: fused recolour needs mask, M and b together", v);
        if (views[v].scene.storage != views[0].scene.storage || views[v].scene.sh_degree != views[0].scene.sh_degree)
            return fail(RECOGS_ERR_UNSUPPORTED, "view %d: all scenes of a batch share storage dtype and SH degree", v);
    }
    return RECOGS_OK;
}

size_t batch_layout(recogs_batch_workspace *ws, const recogs_batch_view *views, int32_t nviews, int32_t tw, int32_t th,
                    int64_t cap) {
    int64_t P = 0, T = 0;
    for (int v = 0; v < nviews; ++v) {
        P += views[v].scene.n;
        T += (int64_t)((views[v].cam.width + tw - 1) / tw) * ((views[v].cam.height + th - 1) / th);
    }
    const int64_t pp = P > 0 ? P : 1;
    const int64_t cc = cap > 0 ? cap : 1;
    const int64_t scan_chunks = (pp + kScanChunk - 1) / kScanChunk;

    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
    ws->off_views = take(sizeof(ViewDev) * (size_t)nviews);
    ws->off_vtab = take(sizeof(uint4) * (size_t)nviews);
    ws->off_rec = take(sizeof(SplatRec) * (size_t)pp);
    ws->off_zbits = take(4 * (size_t)pp);
    ws->off_rect = take(8 * (size_t)pp);
    ws->off_count = take(4 * (size_t)pp);
    ws->off_offset = take(4 * (size_t)pp);
    ws->off_dkeys0 = take(4 * (size_t)pp);
    ws->off_dkeys1 = take(4 * (size_t)pp);
    ws->off_dvals0 = take(4 * (size_t)pp);
    ws->off_dvals1 = take(4 * (size_t)pp);
    ws->off_scan = take(20 * (size_t)scan_chunks);
    ws->off_esum = take(4 * (size_t)((pp + kEmitChunk - 1) / kEmitChunk));
    ws->off_efirst = take(4 * ((size_t)emit_blocks((uint32_t)cc) + 1));
    ws->off_sort_count = take(4 * std::max(sort_count_words((uint64_t)pp), sort_count_words((uint64_t)cc)));
    ws->off_keys0 = take(4 * (size_t)cc);
    ws->off_keys1 = take(4 * (size_t)cc);
    ws->off_vals0 = take(4 * (size_t)cc);
    ws->off_vals1 = take(4 * (size_t)cc);
    ws->off_order = take(4 * (size_t)(T > 0 ? T : 1));
    // zeroed each batch (contiguous): header, histograms, tile ranges
    ws->off_header = take(4 * H_WORDS);
    ws->off_hist = take(4 * 256 * kMaxPasses);
    ws->off_dhist = take(4 * 256 * kMaxPasses);
    ws->off_ranges = take(8 * (size_t)(T > 0 ? T : 1));
    ws->scan_chunks = (size_t)scan_chunks;
    ws->pairs = P;
    ws->tiles = T;
    return o;
}

}  // namespace

extern "C" {

size_t recogs_batch_workspace_bytes(const recogs_batch_view *views, int32_t nviews, int32_t tile_w, int32_t tile_h,
                                    int64_t key_capacity) {
    if (check_batch(views, nviews) != RECOGS_OK || !tile_supported(tile_w, tile_h) || key_capacity < 0) return 0;
    recogs_batch_workspace ws;
    memset(&ws, 0, sizeof(ws));
    return batch_layout(&ws, views, nviews, tile_w, tile_h, key_capacity);
}

recogs_status recogs_batch_init(recogs_batch_workspace *ws, void *dev_mem, size_t bytes, const recogs_batch_view *views,
                                int32_t nviews, const recogs_render_opts *opts, int64_t key_capacity) {
    g_err[0] = 0;
    recogs_status s;
    if (!ws || !dev_mem) return fail(RECOGS_ERR_INVALID, "workspace struct or memory is NULL");
    if ((uintptr_t)dev_mem % kAlign) return fail(RECOGS_ERR_INVALID, "workspace memory not 256-byte aligned");
    if ((s = check_batch(views, nviews)) != RECOGS_OK) return s;
    if ((s = check_opts(opts)) != RECOGS_OK) return s;
    if (opts->depth_map) return fail(RECOGS_ERR_UNSUPPORTED, "batch renders write no depth map");
    if (key_capacity < 0 || key_capacity > 0x7fffffffLL) return fail(RECOGS_ERR_UNSUPPORTED, "key capacity not in 0..2^31-1");
    memset(ws, 0, sizeof(*ws));
    const size_t need = batch_layout(ws, views, nviews, opts->tile_w, opts->tile_h, key_capacity);
    if (bytes < need) return fail(RECOGS_ERR_INVALID, "batch workspace has %zu bytes, needs %zu", bytes, need);
    if (ws->pairs > 0x7fffffffLL) return fail(RECOGS_ERR_UNSUPPORTED, "batch of %lld pairs exceeds 2^31-1", (long long)ws->pairs);
    if (ws->tiles > (1LL << 30)) return fail(RECOGS_ERR_UNSUPPORTED, "batch of %lld tiles exceeds 2^30", (long long)ws->tiles);
    ws->base = dev_mem;
    ws->bytes = bytes;
    ws->nviews = nviews;
    ws->tile_w = opts->tile_w;
    ws->tile_h = opts->tile_h;
    ws->px_per_thread = opts->px_per_thread;
    ws->storage = views[0].scene.storage;
    ws->sh_degree = views[0].scene.sh_degree;
    ws->key_capacity = key_capacity;
    ws->tile_bits = bits_for((uint64_t)(ws->tiles > 0 ? ws->tiles - 1 : 0));
    int dev = 0, cus = 0;
    RECOGS_TRY_HIP(hipGetDevice(&dev));
    RECOGS_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    ws->persistent_blocks = (cus > 0 ? cus : 256) * 8;
    // view table
    ViewDev *vd = (ViewDev *)calloc((size_t)nviews, sizeof(ViewDev));
    uint4 *vt = (uint4 *)calloc((size_t)nviews, sizeof(uint4));
    if (!vd || !vt) {
        free(vd);
        free(vt);
        return fail(RECOGS_ERR_INVALID, "host allocation of the view table failed");
    }
    uint32_t pair = 0, blk = 0, tile = 0;
    for (int v = 0; v < nviews; ++v) {
        const recogs_batch_view &bv = views[v];
        vd[v].sc = make_scene(bv.scene);
        vd[v].cam = make_cam(bv.cam, opts->tile_w, opts->tile_h, opts->extent_rule);
        vd[v].rc = RecolorDev{bv.mask, bv.M, bv.b};
        vd[v].image = bv.image;
        for (int c = 0; c < 3; ++c) vd[v].bg[c] = opts->bg[c];
        vd[v].pair_base = pair;
        vd[v].blk_base = blk;
        vd[v].tile_base = tile;
        vd[v].ntiles = (uint32_t)(vd[v].cam.tiles_x * vd[v].cam.tiles_y);
        vt[v] = make_uint4(pair, tile, (uint32_t)vd[v].cam.tiles_x, 0u);
        pair += (uint32_t)bv.scene.n;
        blk += (uint32_t)((bv.scene.n + 255) / 256);
        tile += vd[v].ntiles;
    }
    ws->preprocess_blocks = blk;
    hipError_t e1 = hipMemcpy((char *)dev_mem + ws->off_views, vd, sizeof(ViewDev) * (size_t)nviews, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy((char *)dev_mem + ws->off_vtab, vt, sizeof(uint4) * (size_t)nviews, hipMemcpyHostToDevice);
    free(vd);
    free(vt);
    if (e1 != hipSuccess || e2 != hipSuccess)
        return fail(RECOGS_ERR_HIP, "uploading the view table: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    return RECOGS_OK;
}

recogs_status recogs_render_batch(const recogs_batch_workspace *ws, hipStream_t stream) {
    g_err[0] = 0;
    if (!ws || !ws->base || ws->nviews <= 0) return fail(RECOGS_ERR_INVALID, "batch workspace not initialised");
    auto B = [&](size_t off) { return (char *)ws->base + off; };
    uint32_t *hdr = (uint32_t *)B(ws->off_header);
    const ViewDev *views = (const ViewDev *)B(ws->off_views);
    SplatRec *rec = (SplatRec *)B(ws->off_rec);
    uint32_t *zb = (uint32_t *)B(ws->off_zbits), *cnt = (uint32_t *)B(ws->off_count), *off = (uint32_t *)B(ws->off_offset);
    uint2 *rect = (uint2 *)B(ws->off_rect);
    uint32_t *dk0 = (uint32_t *)B(ws->off_dkeys0), *dk1 = (uint32_t *)B(ws->off_dkeys1);
    uint32_t *dv0 = (uint32_t *)B(ws->off_dvals0), *dv1 = (uint32_t *)B(ws->off_dvals1);
    uint32_t *k0 = (uint32_t *)B(ws->off_keys0), *k1 = (uint32_t *)B(ws->off_keys1);
    uint32_t *v0 = (uint32_t *)B(ws->off_vals0), *v1 = (uint32_t *)B(ws->off_vals1);
    uint32_t *hist = (uint32_t *)B(ws->off_hist), *dhist = (uint32_t *)B(ws->off_dhist);
    uint32_t *scount = (uint32_t *)B(ws->off_sort_count);
    uint2 *ranges = (uint2 *)B(ws->off_ranges);
    const uint32_t P = (uint32_t)ws->pairs, T = (uint32_t)ws->tiles, cap = (uint32_t)ws->key_capacity;
    // header, histograms and ranges are contiguous
    launch_fill_u32(hdr, 0u, (int64_t)((ws->off_ranges - ws->off_header) / 4) + 2 * (int64_t)T, stream);
    launch_preprocess_batch(ws->storage, ws->sh_degree, ws->preprocess_blocks, views, ws->nviews, rec, zb, rect, cnt, stream);
    {
        const size_t sc_n = ws->scan_chunks;
        uint64_t *pk = (uint64_t *)B(ws->off_scan);
        uint32_t *pv = (uint32_t *)(pk + sc_n);
        launch_scan(cnt, zb, off, P, pk, pv, pv + sc_n, pv + 2 * sc_n, dk0, dv0, hdr, ws->key_capacity, stream, nullptr);
    }
    // depth sort of the pairs with keys over all 32 depth bits above the minimum
    const int dalt = radix_sort_u32_dyn(dk0, dv0, dk1, dv1, P, hdr + H_V, hdr + H_ZMIN_RAW, 32, dhist, scount, stream);
    launch_emit_sorted(dalt ? dv1 : dv0, P, rect, (uint2 *)dk0, 0, (uint32_t *)B(ws->off_esum), dalt ? dv0 : dv1,
                       (uint32_t *)B(ws->off_efirst), cap, k0, v0, stream, hdr + H_V, hdr + H_KEFF, hdr,
                       (const uint4 *)B(ws->off_vtab), ws->nviews);
    const int alt = radix_sort_u32_dyn(k0, v0, k1, v1, cap, hdr + H_KEFF, nullptr, ws->tile_bits, hist, scount, stream);
    launch_ranges32(alt ? k1 : k0, cap, ranges, stream, hdr + H_KEFF);
    launch_tile_order(ranges, T, hdr + H_ORDER_HIST, hdr + H_ORDER_CUR, (uint32_t *)B(ws->off_order), stream);
    if (!launch_blend_persistent(ws->tile_w, ws->tile_h, ws->px_per_thread, (uint32_t)ws->persistent_blocks, views,
                                 ws->nviews, ranges, alt ? v1 : v0, rec, (const uint32_t *)B(ws->off_order), T,
                                 hdr + H_QUEUE, stream))
        return fail(RECOGS_ERR_UNSUPPORTED, "no persistent blend for this tile / px_per_thread");
    return hip_check("render_batch");
}

recogs_status recogs_batch_readback(recogs_batch_workspace *ws, hipStream_t stream) {
    g_err[0] = 0;
    if (!ws || !ws->base) return fail(RECOGS_ERR_INVALID, "batch workspace not initialised");
    uint32_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    RECOGS_TRY_HIP(hipMemcpyAsync(h, (char *)ws->base + ws->off_header, sizeof(h), hipMemcpyDeviceToHost, stream));
    RECOGS_TRY_HIP(hipStreamSynchronize(stream));
    ws->num_keys = (int64_t)((uint64_t)h[H_K_LO] | ((uint64_t)h[H_K_HI] << 32));
    ws->num_visible = h[H_V];
    ws->overflow = (int32_t)h[H_OVERFLOW];
    ws->sorted_in_alt = ws->tile_bits > 0 ? (sort_passes(ws->tile_bits) & 1) : 0;
    return RECOGS_OK;
}

}  // extern "C"
