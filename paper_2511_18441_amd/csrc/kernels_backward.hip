// Backward of the blend and of the colour / fused-recolour step (eq. 8 restricted to
// opacity, SH DC and the recolour matrix), and the L2 loss gradient.
//
// Per-tile recomputation: a workgroup replays its tile's sorted list front to back
// for each pixel, over the entries the forward processed (it stored their count),
// taking the same threshold decisions with the same float32 arithmetic. With the
// forward output y, the colour behind splat i is R_i = y - A_i - rgb_i alpha_i T_i
// (A_i: colour accumulated in front of it), and
//   dL/drgb_i   += alpha_i T_i g
//   dL/dalpha_i  = g . (rgb_i T_i - R_i / (1 - alpha_i))
//   dL/dsigma_i += dL/dalpha_i G_i(p)   (0 where alpha is clamped at 0.99)
// Per splat the workgroup's pixels are summed per wave (shuffles), then one atomic
// per wave adds to the Gaussian's accumulator.
#include "recogs_internal.hpp"

namespace recogs {

template <int TW, int TH, int PPT>
__global__ __launch_bounds__(TW *TH / PPT) void k_blend_bwd(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                                           const SplatRec *__restrict__ rec, int W, int H, int tiles_x,
                                                           const float *__restrict__ image, const float *__restrict__ dldy,
                                                           const uint32_t *__restrict__ nproc,
                                                           float4 *__restrict__ acc) {
#pragma clang fp contract(off)
    using Map = TileMap<TW, TH, PPT>;
    constexpr int NT = Map::NT;
    constexpr int BATCH = 256;
    __shared__ float4 s_r0[BATCH], s_r1[BATCH], s_r2[BATCH];
    __shared__ uint32_t s_gid[BATCH];
    __shared__ uint8_t s_mask[BATCH];
    const int tile = blockIdx.x;
    const int tx0 = (tile % tiles_x) * TW, ty0 = (tile / tiles_x) * TH;
    const int t = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(Map::wave(t));
    int lx, lrow;
    Map::pixel(t, lx, lrow);
    const int px = tx0 + lx;
    const float pxc = (float)px + 0.5f;
    float pyc[PPT], T[PPT], A0[PPT], A1[PPT], A2[PPT], y0[PPT], y1[PPT], y2[PPT], g0[PPT], g1[PPT], g2[PPT];
    uint32_t np[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = ty0 + lrow * PPT + j;
        pyc[j] = (float)py + 0.5f;
        T[j] = 1.f; A0[j] = A1[j] = A2[j] = 0.f;
        np[j] = 0;
        y0[j] = y1[j] = y2[j] = g0[j] = g1[j] = g2[j] = 0.f;
        if (px < W && py < H) {
            const int64_t p = (int64_t)py * W + px;
            np[j] = nproc[p];
            y0[j] = image[p * 3]; y1[j] = image[p * 3 + 1]; y2[j] = image[p * 3 + 2];
            g0[j] = dldy[p * 3]; g1[j] = dldy[p * 3 + 1]; g2[j] = dldy[p * 3 + 2];
        }
    }
    uint32_t npmax = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) npmax = max(npmax, np[j]);

    const uint2 rg = ranges[tile];
    for (uint32_t start = rg.x; start < rg.y; start += BATCH) {
        if (__syncthreads_and(start - rg.x >= npmax)) break;
        for (int q = t; q < BATCH; q += NT) {
            const uint32_t k = start + q;
            if (k < rg.y) {
                const uint32_t gid = vals[k];
                const SplatRec s = rec[gid];
                s_r0[q] = s.r0; s_r1[q] = s.r1; s_r2[q] = s.r2;
                s_gid[q] = gid;
                s_mask[q] = (uint8_t)Map::wave_mask(s.r0, (float)tx0, (float)ty0);
            }
        }
        __syncthreads();
        const int nb = (int)min((uint32_t)BATCH, rg.y - start);
        for (int q = 0; q < nb; ++q) {
            const uint32_t krel = start + q - rg.x;
            if (!wave_ballot(krel < npmax)) break;
            const uint32_t m = __builtin_amdgcn_readfirstlane((uint32_t)s_mask[q]);
            if (!((m >> w) & 1u)) continue;
            const float4 r0 = s_r0[q], r1 = s_r1[q], r2 = s_r2[q];
            const ExpRow er = exp_row(r1, pxc - r0.x);
            float ds = 0.f, dr = 0.f, dg = 0.f, db = 0.f;
            bool any = false;
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                if (krel >= np[j]) continue;
                const float e = exp_at(er, r1, pyc[j] - r0.y);
                if (e < kLog2AlphaMin) continue;
                const float araw = __builtin_amdgcn_exp2f(e);
                const float a = fminf(kAlphaMax, araw);
                const float wgt = a * T[j];
                const float c0 = r2.x * wgt, c1 = r2.y * wgt, c2 = r2.z * wgt;
                const float R0 = y0[j] - A0[j] - c0, R1 = y1[j] - A1[j] - c1, R2 = y2[j] - A2[j] - c2;
                const float inv1ma = 1.f / (1.f - a);
                const float dal = g0[j] * (r2.x * T[j] - R0 * inv1ma) + g1[j] * (r2.y * T[j] - R1 * inv1ma) +
                                  g2[j] * (r2.z * T[j] - R2 * inv1ma);
                dr += wgt * g0[j];
                dg += wgt * g1[j];
                db += wgt * g2[j];
                if (araw < kAlphaMax) ds += dal * (araw / r2.w);
                A0[j] += c0; A1[j] += c1; A2[j] += c2;
                T[j] = T[j] * (1.f - a);
                any = true;
            }
            if (wave_ballot(any)) {
                ds = wave_sum(ds); dr = wave_sum(dr); dg = wave_sum(dg); db = wave_sum(db);
                if (lane_id() == 0) {
                    float *pa = (float *)&acc[s_gid[q]];
                    atomicAdd(pa + 0, ds);
                    atomicAdd(pa + 1, dr);
                    atomicAdd(pa + 2, dg);
                    atomicAdd(pa + 3, db);
                }
            }
        }
    }
}

// Per Gaussian: dL/dsigma, and the chain through the clamp, the fused recolour and
// the DC term: gh = dL/drgb where the pre-clamp colour > 0;
//   selected:   dL/dC0 = Y00 M^T gh, dL/dM += gh (f + 1/2)^T;  unselected: dL/dC0 = Y00 gh.
__global__ __launch_bounds__(256) void k_grad_finish(const float4 *__restrict__ acc, const float4 *__restrict__ bwd,
                                                     const uint32_t *__restrict__ count, int64_t n,
                                                     const float *__restrict__ M, float *__restrict__ dop,
                                                     float *__restrict__ ddc, float *__restrict__ dM) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float m[9];
    bool sel = false;
    float gh[3] = {0.f, 0.f, 0.f}, f[3] = {0.f, 0.f, 0.f};
    if (i < n) {
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        uint32_t flags = 0;
        if (count[i] > 0) {
            a = acc[i];
            const float4 b = bwd[i];
            flags = __float_as_uint(b.w);
            f[0] = b.x; f[1] = b.y; f[2] = b.z;
        }
        gh[0] = (flags & 1u) ? a.y : 0.f;
        gh[1] = (flags & 2u) ? a.z : 0.f;
        gh[2] = (flags & 4u) ? a.w : 0.f;
        sel = (flags & 8u) != 0;
        dop[i] = a.x;
        if (sel) {
#pragma unroll
            for (int k = 0; k < 9; ++k) m[k] = M[k];
#pragma unroll
            for (int c = 0; c < 3; ++c) ddc[c * n + i] = kSH0 * (m[c] * gh[0] + m[3 + c] * gh[1] + m[6 + c] * gh[2]);
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) ddc[c * n + i] = kSH0 * gh[c];
        }
    }
    if (M && wave_ballot(sel)) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float v = wave_sum(sel ? gh[r] * f[c] : 0.f);
                if (lane_id() == 0) atomicAdd(&dM[r * 3 + c], v);
            }
    }
}

// L2 loss: loss += scale sum (y - t)^2, dL/dy = 2 scale (y - t)
__global__ __launch_bounds__(256) void k_loss_l2(const float *__restrict__ y, const float *__restrict__ tg, int64_t count,
                                                 float scale, float *__restrict__ dldy, float *__restrict__ loss) {
    __shared__ float s_w[4];
    float sum = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = y[i] - tg[i];
        dldy[i] = 2.f * scale * d;
        sum += d * d;
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, scale * (s_w[0] + s_w[1] + s_w[2] + s_w[3]));
}

// ---------------------------------------------------------------------------
template <int TW, int TH, int PPT>
static void bwd_one(int ntiles, hipStream_t st, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec, int W, int H,
                    int tiles_x, const float *image, const float *dldy, const uint32_t *nproc, float4 *acc) {
    hipLaunchKernelGGL((k_blend_bwd<TW, TH, PPT>), dim3(ntiles), dim3(TW * TH / PPT), 0, st, ranges, vals, rec, W, H, tiles_x,
                       image, dldy, nproc, acc);
}

bool launch_blend_bwd(int tw, int th, int ppt, int ntiles, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec,
                      int W, int H, int tiles_x, const float *image, const float *dldy, const uint32_t *nproc, float4 *acc,
                      hipStream_t st) {
#define RECOGS_BWD_CASE(A, B, P)                                                                     \
    if (tw == A && th == B && ppt == P) {                                                            \
        bwd_one<A, B, P>(ntiles, st, ranges, vals, rec, W, H, tiles_x, image, dldy, nproc, acc);     \
        return true;                                                                                 \
    }
    RECOGS_BWD_CASE(16, 16, 1) RECOGS_BWD_CASE(16, 16, 2) RECOGS_BWD_CASE(16, 16, 4)
    RECOGS_BWD_CASE(8, 8, 1) RECOGS_BWD_CASE(8, 8, 2) RECOGS_BWD_CASE(8, 8, 4)
    RECOGS_BWD_CASE(32, 8, 1) RECOGS_BWD_CASE(32, 8, 2) RECOGS_BWD_CASE(32, 8, 4)
#undef RECOGS_BWD_CASE
    return false;
}

void launch_grad_finish(const float4 *acc, const float4 *bwd, const uint32_t *count, int64_t n, const float *M, float *dop,
                        float *ddc, float *dM, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc, bwd, count, n, M, dop, ddc, dM);
}

void launch_loss_l2(const float *y, const float *tg, int64_t count, float scale, float *dldy, float *loss, hipStream_t st) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_loss_l2, dim3((unsigned)blocks), dim3(256), 0, st, y, tg, count, scale, dldy, loss);
}

}  // namespace recogs
