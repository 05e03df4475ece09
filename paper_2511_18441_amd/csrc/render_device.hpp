// Device functions shared by the single-view and the batched render kernels
// (preprocess of one Gaussian, blend of one tile).
#pragma once

#include "recogs_internal.hpp"

namespace recogs {

// Real SH basis (eq. 2), degree <= DEG, at unit direction (x, y, z).
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    Y[0] = kSH0;
    if constexpr (DEG >= 1) {
        Y[1] = -kSH1 * y; Y[2] = kSH1 * z; Y[3] = -kSH1 * x;
    }
    if constexpr (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kSH2a * x * y; Y[5] = -kSH2a * y * z; Y[6] = kSH2b * (2.f * zz - xx - yy);
        Y[7] = -kSH2a * x * z; Y[8] = kSH2c * (xx - yy);
        if constexpr (DEG >= 3) {
            Y[9] = -kSH3a * y * (3.f * xx - yy); Y[10] = kSH3b * x * y * z;
            Y[11] = -kSH3c * y * (4.f * zz - xx - yy); Y[12] = kSH3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
            Y[13] = -kSH3c * x * (4.f * zz - xx - yy); Y[14] = kSH3e * z * (xx - yy);
            Y[15] = -kSH3a * x * (xx - 3.f * yy);
        }
    }
}

// The basis at the view direction d = (mu - campos) / |mu - campos| of a centre mu: the
// forward colour and the SH gradients of the backward use these same values.
template <int DEG>
__device__ __forceinline__ void view_basis(const CamDev &cam, float mx, float my, float mz, float *Y) {
    float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
    const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= inv; dy *= inv; dz *= inv;
    sh_basis<DEG>(dx, dy, dz, Y);
}

// ---------------------------------------------------------------------------
// Preprocess: one thread per Gaussian.
//   m = R mu + t (compensated); cull depth <= znear.
//   EWA: J at the 1.3x-frustum-clamped position, Sigma2D = J R Sigma R^T J^T + 0.3 I.
//   Cull det <= 0 and 255 sigma < 1. Box of q <= 2 ln(255 sigma) + 1/64 -> pixel range
//   [ceil(u - ex - 1/2), floor(u + ex - 1/2)] clipped -> tile rectangle and count.
//   Extent rule 1 instead lists the tiles of the 3DGS rasteriser's square: radius
//   r = ceil(3 sqrt(lambda_max)), lambda_max = (A + C)/2 + sqrt(max(0.1, ((A - C)/2)^2 + B^2))
//   (the discriminant as a sum of squares: no cancellation), tiles floor((x - r) / tw) up
//   to floor((x + r + tw - 1) / tw) exclusive around x = u - 1/2 (the same in y), clipped
//   to the grid. The record keeps the box: the blend's region test stays exact.
//   Colour max(0, f + 1/2) or, for selected Gaussians of a fused recolour,
//   max(0, M (f + 1/2) + b).
// Writes the splat record, depth bits, packed tile rectangle and count (the count
// scan reduces the depth range). The colour is evaluated for every Gaussian, so its
// coefficient loads go out with the position and covariance loads, ahead of the culls.
// ---------------------------------------------------------------------------
// Gaussian i of the scene, outputs at index o (o = i for one view; the (view,
// Gaussian) pair index in a batch).
template <int DT, int DEG>
__device__ __forceinline__ void preprocess_one(const SceneDev &sc, const CamDev &cam, const RecolorDev &rc, int keep_bwd,
                                               int64_t i, int64_t o, SplatRec *__restrict__ rec, float4 *__restrict__ bwd,
                                               uint32_t *__restrict__ zbits, uint2 *__restrict__ rect,
                                               uint32_t *__restrict__ count) {
    uint32_t cnt = 0, zb = 0;
    uint2 rr = make_uint2(0u, 0u);
    {
        const int64_t S = sc.stride;
        const float mx = sc.means[i], my = sc.means[S + i], mz = sc.means[2 * S + i];
        // colour (eq. 2) at the view direction of the centre, for every Gaussian: its
        // coefficient loads are issued with the others, before any cull decision
        constexpr int NC = (DEG + 1) * (DEG + 1);
        float f[3];
        {
            float Y[16];
            view_basis<DEG>(cam, mx, my, mz, Y);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < NC; ++k) acc += Store<DT>::ld(sc.sh, (int64_t)(k * 3 + c) * S + i) * Y[k];
                f[c] = acc + 0.5f;
            }
        }
        const float z = dot3c(cam.R[6], mx, cam.R[7], my, cam.R[8], mz, cam.t[2]);
        zb = __float_as_uint(z);
        if (z > cam.znear) {
            const float x = dot3c(cam.R[0], mx, cam.R[1], my, cam.R[2], mz, cam.t[0]);
            const float y = dot3c(cam.R[3], mx, cam.R[4], my, cam.R[5], mz, cam.t[1]);
            const float iz = 1.0f / z;
            const float xc = fminf(cam.limx, fmaxf(-cam.limx, x * iz)) * z;
            const float yc = fminf(cam.limy, fmaxf(-cam.limy, y * iz)) * z;
            const float j00 = cam.fx * iz, j02 = -cam.fx * xc * iz * iz;
            const float j11 = cam.fy * iz, j12 = -cam.fy * yc * iz * iz;
            // T = J R (2 x 3)
            const float a0 = j00 * cam.R[0] + j02 * cam.R[6], a1 = j00 * cam.R[1] + j02 * cam.R[7],
                        a2 = j00 * cam.R[2] + j02 * cam.R[8];
            const float b0 = j11 * cam.R[3] + j12 * cam.R[6], b1 = j11 * cam.R[4] + j12 * cam.R[7],
                        b2 = j11 * cam.R[5] + j12 * cam.R[8];
            const float c00 = sc.cov3d[i], c01 = sc.cov3d[S + i], c02 = sc.cov3d[2 * S + i];
            const float c11 = sc.cov3d[3 * S + i], c12 = sc.cov3d[4 * S + i], c22 = sc.cov3d[5 * S + i];
            // Sigma T^T columns
            const float sa0 = c00 * a0 + c01 * a1 + c02 * a2, sa1 = c01 * a0 + c11 * a1 + c12 * a2,
                        sa2 = c02 * a0 + c12 * a1 + c22 * a2;
            const float sb0 = c00 * b0 + c01 * b1 + c02 * b2, sb1 = c01 * b0 + c11 * b1 + c12 * b2,
                        sb2 = c02 * b0 + c12 * b1 + c22 * b2;
            const float A = a0 * sa0 + a1 * sa1 + a2 * sa2 + kDilation;
            const float B = a0 * sb0 + a1 * sb1 + a2 * sb2;
            const float C = b0 * sb0 + b1 * sb1 + b2 * sb2 + kDilation;
            const float det = A * C - B * B;
            if (det > 0.f && det < INFINITY) {
                const float sigma = Store<DT>::ldc(sc.opacity, i);
                if (255.f * sigma >= 1.f) {
                    const float level = 2.f * logf(255.f * sigma) + kQSlack;
                    const float ex = sqrtf(level * A), ey = sqrtf(level * C);
                    const float u = cam.fx * (x / z) + cam.cx, v = cam.fy * (y / z) + cam.cy;
                    if (cam.extent_rule == 0) {
                        const float fx0 = fmaxf(ceilf(u - ex - 0.5f), 0.f), fx1 = fminf(floorf(u + ex - 0.5f), (float)(cam.W - 1));
                        const float fy0 = fmaxf(ceilf(v - ey - 0.5f), 0.f), fy1 = fminf(floorf(v + ey - 0.5f), (float)(cam.H - 1));
                        if (fx0 <= fx1 && fy0 <= fy1) {
                            const uint32_t tx0 = (uint32_t)fx0 / cam.tw, tx1 = (uint32_t)fx1 / cam.tw;
                            const uint32_t ty0 = (uint32_t)fy0 / cam.th, ty1 = (uint32_t)fy1 / cam.th;
                            cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                            rr = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
                        }
                    } else {
                        const float hd = 0.5f * (A - C);
                        const float lam = 0.5f * (A + C) + sqrtf(fmaxf(0.1f, hd * hd + B * B));
                        const float r = ceilf(3.f * sqrtf(lam));
                        const float xc = u - 0.5f, yc = v - 0.5f;
                        const float twf = (float)cam.tw, thf = (float)cam.th;
                        // tile sizes are powers of two: the divisions are exact
                        const float gx = (float)cam.tiles_x, gy = (float)cam.tiles_y;
                        const float ax = fminf(fmaxf(floorf((xc - r) / twf), 0.f), gx);
                        const float bx = fminf(fmaxf(floorf((xc + r + (twf - 1.f)) / twf), 0.f), gx);
                        const float ay = fminf(fmaxf(floorf((yc - r) / thf), 0.f), gy);
                        const float by = fminf(fmaxf(floorf((yc + r + (thf - 1.f)) / thf), 0.f), gy);
                        if (bx > ax && by > ay) {
                            const uint32_t tx0 = (uint32_t)ax, tx1 = (uint32_t)bx - 1u;
                            const uint32_t ty0 = (uint32_t)ay, ty1 = (uint32_t)by - 1u;
                            cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                            rr = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
                        }
                    }
                    if (cnt > 0) {
                        float pre[3] = {f[0], f[1], f[2]};
                        uint32_t flags = 0;
                        if (rc.mask && rc.mask[i]) {
                            flags |= 8u;
#pragma unroll
                            for (int r = 0; r < 3; ++r)
                                pre[r] = rc.M[r * 3] * f[0] + rc.M[r * 3 + 1] * f[1] + rc.M[r * 3 + 2] * f[2] + rc.b[r];
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) flags |= (pre[c] > 0.f ? 1u : 0u) << c;
                        // conic = inverse 2D covariance, folded into a base-2 exponent
                        const float idet = 1.0f / det;
                        const float ca = C * idet, cb = -B * idet, cc = A * idet;
                        SplatRec s;
                        s.r0 = make_float4(u, v, ex, ey);
                        s.r1 = make_float4(-0.5f * kLog2e * ca, -kLog2e * cb, -0.5f * kLog2e * cc, log2f(sigma));
                        s.r2 = make_float4(fmaxf(pre[0], 0.f), fmaxf(pre[1], 0.f), fmaxf(pre[2], 0.f), sigma);
                        rec[o] = s;
                        if (keep_bwd) bwd[o] = make_float4(f[0], f[1], f[2], __uint_as_float(flags));
                    }
                }
            }
        }
        count[o] = cnt;
        rect[o] = rr;
        zbits[o] = zb;
    }
}

constexpr int kBlendBatch = 128;   // splat records staged per LDS batch (small enough for 8 waves per SIMD)

// LDS staging of one batch: only what the per-pixel loop reads (the extent box is
// used at staging, for the wave mask, and not kept). One 48-byte record per splat,
// so a wave reads all of it from one address register.
struct BlendRec {
    float2 uv;        // projected centre
    uint32_t mask;    // wave regions the alpha >= 1/255 box meets
    uint32_t pad;
    float4 r1;        // base-2 conic terms and log2 sigma
    float4 rgb;       // colour (w unused)
};
struct BlendStage {
    BlendRec r[kBlendBatch];
};

// Final colour of one pixel (index p = y W + x of an image of HW pixels): HWC, or CHW
// with chw (the two layouts of Sec. 4.2).
__device__ __forceinline__ void store_pixel(float *__restrict__ image, int64_t p, int64_t HW, int chw, float r, float g,
                                            float b) {
    if (chw) {
        image[p] = r;
        image[HW + p] = g;
        image[2 * HW + p] = b;
    } else {
        image[p * 3 + 0] = r;
        image[p * 3 + 1] = g;
        image[p * 3 + 2] = b;
    }
}

// One splat record applied to the PPT pixels of a thread (eq. 3, front to back).
// `idx` is the record's 1-based position in its tile list (kept, with STATE, as the
// count up to the last blended entry). With DEPTH, cross[j] takes the position of the
// blended splat that takes the pixel's transmittance from >= tau to < tau (the rough
// depth of Sec. 3.2; at most one splat per pixel does, as T only decreases). Two
// compares and a select; a per-pixel flag in a lane mask instead of the compare of T
// measured slower (its mask updates put scalar instructions between the vector ones).
template <int PPT, bool STATE, bool DEPTH = false>
__device__ __forceinline__ void blend_step(const BlendRec &b, float pxc, const float *pyc, float *T, float *C0, float *C1,
                                           float *C2, uint32_t *last, uint32_t idx, uint32_t *cross = nullptr,
                                           float tau = 0.f) {
#pragma clang fp contract(off)
    const float2 uv = b.uv;
    const float4 r1 = b.r1, r2 = b.rgb;
    const ExpRow er = exp_row(r1, pxc - uv.x);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const float e = exp_at(er, r1, pyc[j] - uv.y);
        const float a = fminf(kAlphaMax, __builtin_amdgcn_exp2f(e));
        const float Tn = __builtin_fmaf(-a, T[j], T[j]);   // T (1 - alpha), rounded once
        // A stopped pixel (T < 0) needs no test of its own: its T' = T (1 - alpha) is
        // negative too, so `stop` holds, nothing is blended and T stays -|T| = T.
        const bool ok = !(e < kLog2AlphaMin);
        const bool stop = Tn < kTMin;
        const bool bl = ok && !stop;
        const float wgt = bl ? a * T[j] : 0.f;
        C0[j] = __builtin_fmaf(r2.x, wgt, C0[j]);
        C1[j] = __builtin_fmaf(r2.y, wgt, C1[j]);
        C2[j] = __builtin_fmaf(r2.z, wgt, C2[j]);
        if constexpr (STATE) last[j] = bl ? idx : last[j];
        if constexpr (DEPTH) cross[j] = (bl && Tn < tau && T[j] >= tau) ? idx : cross[j];
        const float Ts = stop ? -fabsf(T[j]) : Tn;   // two selects: this form compiles to v_cndmask
        T[j] = ok ? Ts : T[j];
    }
}

// One tile (local index `tile` of a W x H image with tiles_x tiles per row) whose
// sorted list is vals[rg.x, rg.y). With STATE the final transmittance and the
// per-pixel count of list entries up to the last blended one are written (the
// backward replays them); finalT / nproc are then non-null.
//
// Per pixel the transmittance T carries the state: T > 0 while compositing; at the
// splat that would take it below 1e-4 it becomes -T (stopped, |T| is final). Every
// lane evaluates every splat its wave takes, and selects leave a pixel that is
// stopped, below the alpha threshold or stopping unchanged (C + r * 0 == C exactly),
// so the per-pixel arithmetic is that of eq. 3 with no divergent branches.
template <int TW, int TH, int PPT, bool STATE>
__device__ __forceinline__ void blend_tile(int tile, uint2 rg, const uint32_t *__restrict__ vals,
                                           const SplatRec *__restrict__ rec, int W, int H, int tiles_x, float bg0,
                                           float bg1, float bg2, float *__restrict__ image, int chw,
                                           float *__restrict__ finalT, uint32_t *__restrict__ nproc, BlendStage &sm) {
#pragma clang fp contract(off)
    using Map = TileMap<TW, TH, PPT>;
    constexpr int NT = Map::NT;
    constexpr int BATCH = kBlendBatch;
    const int tx0 = (tile % tiles_x) * TW, ty0 = (tile / tiles_x) * TH;
    const int t = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(Map::wave(t));
    int lx, lrow;
    Map::pixel(t, lx, lrow);
    const int px = tx0 + lx;
    const float pxc = (float)px + 0.5f;
    float pyc[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
    uint32_t last[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = ty0 + lrow * PPT + j;
        pyc[j] = (float)py + 0.5f;
        T[j] = (px < W && py < H) ? 1.f : -1.f;  // pixels outside the image start stopped
        C0[j] = C1[j] = C2[j] = 0.f;
        last[j] = 0;
    }

    for (uint32_t start = rg.x; start < rg.y; start += BATCH) {
        bool stopped = true;
#pragma unroll
        for (int j = 0; j < PPT; ++j) stopped = stopped && !(T[j] > 0.f);
        if (__syncthreads_and(stopped)) break;
        for (int q = t; q < BATCH; q += NT) {
            const uint32_t k = start + q;
            if (k < rg.y) {
                const SplatRec s = rec[vals[k]];
                BlendRec b;
                b.uv = make_float2(s.r0.x, s.r0.y);
                b.mask = Map::wave_mask(s.r0, s.r1, (float)tx0, (float)ty0);
                b.pad = 0u;
                b.r1 = s.r1;
                b.rgb = s.r2;
                sm.r[q] = b;
            }
        }
        __syncthreads();
        const int nb = (int)min((uint32_t)BATCH, rg.y - start);
        const uint32_t krel0 = start + 1 - rg.x;
        // the batch's records this wave takes, as a scalar bit set per 64 records; the
        // loop walks its set bits in order
        constexpr int L = NT < 64 ? NT : 64;   // lanes of a wave (a workgroup may be a partial wave)
        uint64_t todo[BATCH / 64];
#pragma unroll
        for (int c = 0; c < BATCH / 64; ++c) {
            todo[c] = 0;
#pragma unroll
            for (int sub = 0; sub < 64 / L; ++sub) {
                const int q = c * 64 + sub * L + (int)lane_id();
                todo[c] |= wave_ballot(q < nb && ((sm.r[q].mask >> w) & 1u)) << (sub * L);
            }
        }
        bool quit = false;
#pragma unroll
        for (int c = 0; c < BATCH / 64; ++c) {
            uint64_t mm = todo[c];
            while (mm && !quit) {
                const int q = c * 64 + (int)__builtin_ctzll(mm);
                mm &= mm - 1;
                bool alive = false;
#pragma unroll
                for (int j = 0; j < PPT; ++j) alive = alive || T[j] > 0.f;
                if (!wave_ballot(alive)) {
                    quit = true;
                    break;
                }
                blend_step<PPT, STATE>(sm.r[q], pxc, pyc, T, C0, C1, C2, last, krel0 + (uint32_t)q);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = ty0 + lrow * PPT + j;
        if (px < W && py < H) {
            const int64_t p = (int64_t)py * W + px;
            const float Tf = fabsf(T[j]);
            store_pixel(image, p, (int64_t)W * H, chw, __builtin_fmaf(Tf, bg0, C0[j]), __builtin_fmaf(Tf, bg1, C1[j]),
                        __builtin_fmaf(Tf, bg2, C2[j]));
            if constexpr (STATE) {
                finalT[p] = Tf;
                nproc[p] = last[j];
            }
        }
    }
}

// Region form of the same blend: one wave, alone in its workgroup, composites the
// 8 x 8*PPT pixel region `sub` of tile `tile` (regions numbered row-major, TW / 8 per
// row). It reads the tile's whole list 64 records at a time, one per lane, and takes
// those that pass region_hit for its own region, in list order (compacted into the
// first LDS slots, with their list positions where STATE or DEPTH needs them). No barrier couples
// the regions of a tile: a region whose pixels have all stopped retires at once, so
// the sort tile can be larger than the region without the early-stopped pixels
// holding the rest. The per-pixel arithmetic and the list positions kept with STATE
// are those of blend_tile, so both forms give bit-identical outputs. With DEPTH the
// rough depth map (Sec. 3.2) is written too: per pixel, the float32 depth (zbits, per
// record) of the splat whose blending takes T below tau, 0 where none does.
constexpr int kRegionUnroll = 4;

template <int TW, int TH, int PPT, bool STATE, bool DEPTH = false>
__device__ __forceinline__ void blend_region(int tile, int sub, uint2 rg, const uint32_t *__restrict__ vals,
                                             const SplatRec *__restrict__ rec, int W, int H, int tiles_x, float bg0,
                                             float bg1, float bg2, float *__restrict__ image, int chw,
                                             float *__restrict__ finalT, uint32_t *__restrict__ nproc,
                                             BlendRec *sm /* [64] */, const uint32_t *__restrict__ zbits = nullptr,
                                             float tau = 0.f, float *__restrict__ depth = nullptr) {
#pragma clang fp contract(off)
    static_assert(TW % 8 == 0 && TH % (8 * PPT) == 0, "regions of 8 x 8*PPT pixels");
    const int l = (int)lane_id();
    const int bx = (tile % tiles_x) * TW + (sub % (TW / 8)) * 8;
    const int by = (tile / tiles_x) * TH + (sub / (TW / 8)) * 8 * PPT;
    const int px = bx + (l & 7);
    const float pxc = (float)px + 0.5f;
    const float x0 = (float)bx + 0.5f, x1 = x0 + 7.f;
    const float y0 = (float)by + 0.5f, y1 = y0 + (float)(8 * PPT - 1);
    float pyc[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
    uint32_t last[PPT], cross[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = by + (l >> 3) * PPT + j;
        pyc[j] = (float)py + 0.5f;
        T[j] = (px < W && py < H) ? 1.f : -1.f;  // pixels outside the image start stopped
        C0[j] = C1[j] = C2[j] = 0.f;
        last[j] = 0;
        cross[j] = 0;
    }
    // Software pipeline over chunks of 64 list entries (one per lane): the records of
    // chunk c are in registers while chunk c - 1 is composited, and the list values of
    // chunk c + 1 are on their way, so the two dependent loads are off the critical path.
    float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, p2 = p0;
    uint32_t vnext = 0;
    {
        const uint32_t k = rg.x + (uint32_t)l;
        if (k < rg.y) {
            const SplatRec *s = rec + vals[k];
            p0 = s->r0; p1 = s->r1; p2 = s->r2;
        }
        if (k + 64u < rg.y) vnext = vals[k + 64u];
    }
    for (uint32_t start = rg.x; start < rg.y; start += 64) {
        bool alive = false;
#pragma unroll
        for (int j = 0; j < PPT; ++j) alive = alive || T[j] > 0.f;
        if (!wave_ballot(alive)) break;
        const bool hit = start + (uint32_t)l < rg.y && region_hit(p0, p1, x0, x1, y0, y1);
        const uint64_t mm = wave_ballot(hit);
        if (hit) {   // compacted in list order: slot = passing lanes below this one
            const uint32_t slot = rank_below(mm);
            sm[slot].uv = make_float2(p0.x, p0.y);
            sm[slot].r1 = p1;
            sm[slot].rgb = p2;
            if constexpr (STATE || DEPTH) sm[slot].pad = start + 1u - rg.x + (uint32_t)l;   // 1-based list position
        }
        const int nh = (int)__builtin_popcountll(mm);
        wave_sync();   // the lanes' LDS writes before any lane reads
        {
            const uint32_t k = start + 64u + (uint32_t)l;
            if (k < rg.y) {
                const SplatRec *s = rec + vnext;
                p0 = s->r0; p1 = s->r1; p2 = s->r2;
            }
            if (k + 64u < rg.y) vnext = vals[k + 64u];
        }
        // kRegionUnroll records per liveness check: consecutive slots, so their LDS
        // addresses are one base plus immediate offsets
        for (int q = 0; q < nh; q += kRegionUnroll) {
            bool live = false;
#pragma unroll
            for (int j = 0; j < PPT; ++j) live = live || T[j] > 0.f;
            if (!wave_ballot(live)) break;
            // the group's LDS base as an opaque vector value: kept in one register for
            // the group (a copy per step otherwise), the records at immediate offsets
            uint32_t off = (uint32_t)q * (uint32_t)sizeof(BlendRec);
            asm volatile("" : "+v"(off));
            const BlendRec *g = reinterpret_cast<const BlendRec *>(reinterpret_cast<const char *>(sm) + off);
#pragma unroll
            for (int u = 0; u < kRegionUnroll; ++u)
                if (q + u < nh)
                    blend_step<PPT, STATE, DEPTH>(g[u], pxc, pyc, T, C0, C1, C2, last, (STATE || DEPTH) ? g[u].pad : 0u,
                                                  cross, tau);
        }
        wave_sync();   // all reads of this chunk before the next chunk's writes
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = by + (l >> 3) * PPT + j;
        if (px < W && py < H) {
            const int64_t p = (int64_t)py * W + px;
            const float Tf = fabsf(T[j]);
            store_pixel(image, p, (int64_t)W * H, chw, __builtin_fmaf(Tf, bg0, C0[j]), __builtin_fmaf(Tf, bg1, C1[j]),
                        __builtin_fmaf(Tf, bg2, C2[j]));
            if constexpr (STATE) {
                finalT[p] = Tf;
                nproc[p] = last[j];
            }
            if constexpr (DEPTH) depth[p] = cross[j] ? __uint_as_float(zbits[vals[rg.x + cross[j] - 1u]]) : 0.f;
        }
    }
}

}  // namespace recogs
