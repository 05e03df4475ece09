// Pieces of the background optimiser (Sec. 3.3 / 4.1): the L1 and SSIM terms of the
// loss of eq. 4 with their gradients (eq. 7), and the Adam step that moves the SH coefficients.
#include <cmath>
#include <cstring>

#include "optim_device.hpp"

namespace recogs {

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st);

// loss = scale sum |y - t| (overwritten by the caller's fill), dL/dy = scale sign(y - t)
// with sign(0) = 0. With vec (all three arrays 16-byte aligned) 4 elements per step.
__device__ __forceinline__ float sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(1024) void k_loss_l1(const float *__restrict__ y, const float *__restrict__ tg, int64_t count,
                                                 float scale, float *__restrict__ dldy, float *__restrict__ loss, int vec) {
    __shared__ float s_w[16];
    float sum = 0.f;
    const int64_t n4 = vec ? count / 4 : 0;
    const float4 *y4 = reinterpret_cast<const float4 *>(y), *t4 = reinterpret_cast<const float4 *>(tg);
    float4 *d4 = reinterpret_cast<float4 *>(dldy);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto one = [&](const float4 a, const float4 b, int64_t i) {
        const float4 d = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
        d4[i] = make_float4(scale * sgn(d.x), scale * sgn(d.y), scale * sgn(d.z), scale * sgn(d.w));
        sum += fabsf(d.x) + fabsf(d.y) + fabsf(d.z) + fabsf(d.w);
    };
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {   // four groups' loads in flight
        float4 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { a[u] = y4[i + u * stride]; b[u] = t4[i + u * stride]; }
#pragma unroll
        for (int u = 0; u < 4; ++u) one(a[u], b[u], i + u * stride);
    }
    for (; i < n4; i += stride) one(y4[i], t4[i], i);
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const float d = y[i] - tg[i];
        dldy[i] = scale * sgn(d);
        sum += fabsf(d);
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float w = 0.f;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) w += s_w[k];   // the waves' sums in order
        atomicAdd(loss, scale * w);
    }
}

void launch_loss_l1(const float *y, const float *tg, int64_t count, float scale, float *dldy, float *loss, hipStream_t st) {
    if (count <= 0) return;
    // few workgroups (of 16 waves): each adds its partial sum with one same-address atomic
    int64_t blocks = (count + 1023) / 1024;
    if (blocks > 128) blocks = 128;
    const int vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(tg) | reinterpret_cast<uintptr_t>(dldy)) &
                     15u) == 0;
    hipLaunchKernelGGL(k_loss_l1, dim3((unsigned)blocks), dim3(1024), 0, st, y, tg, count, scale, dldy, loss, vec);
}

// Adam, element-wise: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - lr (m / c1) / (sqrt(v / c2) + eps) with the bias corrections c1 = 1 - b1^step,
// c2 = 1 - b2^step (their reciprocals computed by the host in double precision).
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, int64_t count, AdamArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        float pi = ld_stream(p + i), mi = ld_stream(m + i), vi = ld_stream(v + i);
        adam_update(pi, ld_stream(g + i), mi, vi, a);
        st_stream(m + i, mi);
        st_stream(v + i, vi);
        st_stream(p + i, pi);
    }
}

// The same update on four consecutive values per thread (16-byte loads and stores: the
// step moves 28 bytes per coefficient and is bound by HBM).
__global__ __launch_bounds__(256) void k_adam4(float4 *__restrict__ p, const float4 *__restrict__ g,
                                               float4 *__restrict__ m, float4 *__restrict__ v, int64_t count4,
                                               AdamArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count4; i += stride) {
        const float4 gi = ld_stream(g + i);
        float4 mi = ld_stream(m + i), vi = ld_stream(v + i), pi = ld_stream(p + i);
        adam_update(pi.x, gi.x, mi.x, vi.x, a);
        adam_update(pi.y, gi.y, mi.y, vi.y, a);
        adam_update(pi.z, gi.z, mi.z, vi.z, a);
        adam_update(pi.w, gi.w, mi.w, vi.w, a);
        st_stream(m + i, mi);
        st_stream(v + i, vi);
        st_stream(p + i, pi);
    }
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr, float b1, float b2, float eps,
                 float ic1, float ic2, hipStream_t st) {
    if (count <= 0) return;
    const AdamArgs a{lr, b1, b2, eps, ic1, ic2};
    const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(g) | reinterpret_cast<uintptr_t>(m) |
                       reinterpret_cast<uintptr_t>(v)) & 15u) == 0;
    int64_t done = 0;
    if (vec && count >= 4) {
        const int64_t c4 = count / 4;
        int64_t blocks = (c4 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_adam4, dim3((unsigned)blocks), dim3(256), 0, st, (float4 *)p, (const float4 *)g, (float4 *)m,
                           (float4 *)v, c4, a);
        done = 4 * c4;
    }
    const int64_t rest = count - done;
    if (rest <= 0) return;
    int64_t blocks = (rest + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, p + done, g + done, m + done, v + done, rest, a);
}

// ---------------------------------------------------------------------------
// SSIM term of eq. 4 over HWC float images, per channel, with the 11 x 11 Gaussian
// window (sigma 1.5, zero outside the image): local means, variances and covariance
// are separable blurs; S = (2 mu_y mu_t + C1)(2 s_yt + C2) / ((mu_y^2 + mu_t^2 + C1)
// (s_y^2 + s_t^2 + C2)). Its gradient: S depends on y through mu_y = G*y, E_yy = G*(y^2)
// and E_yt = G*(y t), so dS/dy = G*a + 2 y (G*b) + t (G*c) with a, b, c the partial
// derivatives of S in those maps. Two passes over 16 x 16 output tiles, each with its
// 26 x 26 input halo in LDS, blurred along x then along y:
//   k_ssim_fwd: a workgroup per (tile, channel): the three maps a, b, c per pixel and
//               the tile's sum of S;
//   k_ssim_bwd: a workgroup per tile, the channels in turn: the blurs of a, b, c and the
//               gradient; its first workgroup first adds the tiles' sums in a fixed
//               order (the loss).
// ---------------------------------------------------------------------------
namespace {
constexpr int kSsimR = 5;                     // window radius (11 taps)
constexpr int kSsimT = 16;                    // output tile edge
constexpr int kSsimH = kSsimT + 2 * kSsimR;   // halo tile edge (26)
constexpr float kSsimC1 = 0.01f * 0.01f, kSsimC2 = 0.03f * 0.03f;
}  // namespace

struct SsimWindow { float g[2 * kSsimR + 1]; };

// part_l1 (optional): also the tile's sum of |y - t| for the channel (the L1 term)
__global__ __launch_bounds__(256) void k_ssim_fwd(const float *__restrict__ y, const float *__restrict__ t, int W, int H,
                                                  SsimWindow win, float *__restrict__ maps, float *__restrict__ part,
                                                  float *__restrict__ part_l1) {
    __shared__ float s_y[kSsimH * kSsimH], s_t[kSsimH * kSsimH];
    __shared__ float s_h[5][kSsimH][kSsimT];   // x-blurred y, t, y^2, t^2, y t
    __shared__ float s_w[4], s_w1[4];
    const int c = blockIdx.z;   // the channel: one workgroup per (tile, channel)
    const int ox = blockIdx.x * kSsimT, oy = blockIdx.y * kSsimT;
    const int tx = threadIdx.x % kSsimT, ty = threadIdx.x / kSsimT;
    const int px = ox + tx, py = oy + ty;
    const int64_t HW = (int64_t)W * H;
    // the channel's halo tiles of both images (zero outside the image); every load of the
    // thread is issued before the first LDS store, so the tile costs one memory round trip
    constexpr int NL = (kSsimH * kSsimH + 255) / 256;
    float ly[NL], lt[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int k = (int)threadIdx.x + 256 * i;
        const int x = ox + k % kSsimH - kSsimR, yy = oy + k / kSsimH - kSsimR;
        const bool in = k < kSsimH * kSsimH && x >= 0 && x < W && yy >= 0 && yy < H;
        const int64_t q = in ? ((int64_t)yy * W + x) * 3 + c : 0;
        ly[i] = in ? y[q] : 0.f;
        lt[i] = in ? t[q] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int k = (int)threadIdx.x + 256 * i;
        if (k < kSsimH * kSsimH) {
            s_y[k] = ly[i];
            s_t[k] = lt[i];
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kSsimH * kSsimT; k += 256) {
        const int r = k / kSsimT, cx = k % kSsimT;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int j = 0; j <= 2 * kSsimR; ++j) {
            const float u = s_y[r * kSsimH + cx + j], v = s_t[r * kSsimH + cx + j], g = win.g[j];
            a0 += g * u; a1 += g * v; a2 += g * (u * u); a3 += g * (v * v); a4 += g * (u * v);
        }
        s_h[0][r][cx] = a0; s_h[1][r][cx] = a1; s_h[2][r][cx] = a2; s_h[3][r][cx] = a3; s_h[4][r][cx] = a4;
    }
    __syncthreads();
    float my = 0.f, mt = 0.f, eyy = 0.f, ett = 0.f, eyt = 0.f;
#pragma unroll
    for (int j = 0; j <= 2 * kSsimR; ++j) {
        const float g = win.g[j];
        my += g * s_h[0][ty + j][tx]; mt += g * s_h[1][ty + j][tx];
        eyy += g * s_h[2][ty + j][tx]; ett += g * s_h[3][ty + j][tx]; eyt += g * s_h[4][ty + j][tx];
    }
    float ssum = 0.f, asum = 0.f;
    if (part_l1 && px < W && py < H) {
        const int k = (ty + kSsimR) * kSsimH + tx + kSsimR;
        asum = fabsf(s_y[k] - s_t[k]);
    }
    if (px < W && py < H) {
        const float syy = eyy - my * my, stt = ett - mt * mt, syt = eyt - my * mt;
        const float l1 = 2.f * my * mt + kSsimC1, l2 = my * my + mt * mt + kSsimC1;
        const float c1 = 2.f * syt + kSsimC2, c2 = syy + stt + kSsimC2;
        const float il2c2 = 1.f / (l2 * c2);
        const float S = l1 * c1 * il2c2;
        const float dS_dsyt = 2.f * l1 * il2c2;
        const float dS_dsyy = -S / c2;
        const float dS_dmy = 2.f * mt * c1 * il2c2 - S * 2.f * my / l2;
        const int64_t p = (int64_t)py * W + px;
        maps[(3 * c + 0) * HW + p] = dS_dmy - 2.f * my * dS_dsyy - mt * dS_dsyt;   // a
        maps[(3 * c + 1) * HW + p] = dS_dsyy;                                    // b
        maps[(3 * c + 2) * HW + p] = dS_dsyt;                                    // c
        ssum = S;
    }
    ssum = wave_sum(ssum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = ssum;
    if (part_l1) {
        asum = wave_sum(asum);
        if (lane_id() == 0) s_w1[threadIdx.x >> 6] = asum;
    }
    __syncthreads();
    // the workgroup's sums, added to the others in a fixed order by the backward
    const size_t at = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0) part[at] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
    if (part_l1 && threadIdx.x == 0) part_l1[at] = ((s_w1[0] + s_w1[1]) + s_w1[2]) + s_w1[3];
}

// The n partial sums added in a fixed order by one workgroup (thread t: entries t,
// t + 256, ... in turn, then the waves' sums in order): the same bits on every run.
// Eight loads in flight per thread. The total is returned to thread 0.
__device__ __forceinline__ float fixed_order_sum(const float *__restrict__ part, uint32_t n, float *s_w /* [4] */) {
    float acc = 0.f;
    for (uint32_t k0 = threadIdx.x; k0 < n; k0 += 256u * 8u) {
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = k0 + 256u * i < n ? part[k0 + 256u * i] : 0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (k0 + 256u * i < n) acc += v[i];
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    return ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

// part / nparts / weight / loss: the loss weight + gscale (sum of S), plus l1_scale (sum
// of |y - t|) with part_l1, summed by workgroup (0, 0) before its tile. With part_l1 the
// gradient also takes l1_scale sign(y - t), added before the SSIM term is (the bits of
// the L1 gradient written first and the SSIM gradient added to it).
__global__ __launch_bounds__(256) void k_ssim_bwd(const float *__restrict__ y, const float *__restrict__ t, int W, int H,
                                                  SsimWindow win, const float *__restrict__ maps, float gscale,
                                                  int accumulate, float *__restrict__ dldy, const float *__restrict__ part,
                                                  uint32_t nparts, float weight, float *__restrict__ loss,
                                                  const float *__restrict__ part_l1, float l1_scale) {
    __shared__ float s_m[3][kSsimH * kSsimH];
    __shared__ float s_h[3][kSsimH][kSsimT];
    __shared__ float s_lw[4], s_lw1[4];
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        const float ss = fixed_order_sum(part, nparts, s_lw);
        if (part_l1) {
            const float sa = fixed_order_sum(part_l1, nparts, s_lw1);
            if (threadIdx.x == 0) *loss = (weight + gscale * ss) + l1_scale * sa;
        } else if (threadIdx.x == 0) {
            *loss = weight + gscale * ss;
        }
    }
    const int ox = blockIdx.x * kSsimT, oy = blockIdx.y * kSsimT;
    const int tx = threadIdx.x % kSsimT, ty = threadIdx.x / kSsimT;
    const int px = ox + tx, py = oy + ty;
    const int64_t HW = (int64_t)W * H;
    // The three channels in turn (a pixel's three gradient values are then written by one
    // workgroup); the three maps of channel c + 1 are loaded into registers while channel
    // c is blurred, so the loads after the first channel's are off the critical path.
    constexpr int NL = (kSsimH * kSsimH + 255) / 256;
    float lm[3][NL];
    int64_t lp[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int k = (int)threadIdx.x + 256 * i;
        const int x = ox + k % kSsimH - kSsimR, yy = oy + k / kSsimH - kSsimR;
        lp[i] = (k < kSsimH * kSsimH && x >= 0 && x < W && yy >= 0 && yy < H) ? (int64_t)yy * W + x : -1;
    }
    auto load_maps = [&](int c) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int i = 0; i < NL; ++i) lm[q][i] = lp[i] >= 0 ? maps[(3 * c + q) * HW + lp[i]] : 0.f;
    };
    load_maps(0);
    for (int c = 0; c < 3; ++c) {
        __syncthreads();   // the previous channel's reads of s_m and s_h done
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int k = (int)threadIdx.x + 256 * i;
                if (k < kSsimH * kSsimH) s_m[q][k] = lm[q][i];
            }
        __syncthreads();
        if (c < 2) load_maps(c + 1);
        for (int k = threadIdx.x; k < kSsimH * kSsimT; k += 256) {
            const int r = k / kSsimT, cx = k % kSsimT;
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
            for (int j = 0; j <= 2 * kSsimR; ++j) {
                const float g = win.g[j];
                a0 += g * s_m[0][r * kSsimH + cx + j]; a1 += g * s_m[1][r * kSsimH + cx + j]; a2 += g * s_m[2][r * kSsimH + cx + j];
            }
            s_h[0][r][cx] = a0; s_h[1][r][cx] = a1; s_h[2][r][cx] = a2;
        }
        __syncthreads();
        float ga = 0.f, gb = 0.f, gc = 0.f;
#pragma unroll
        for (int j = 0; j <= 2 * kSsimR; ++j) {
            const float g = win.g[j];
            ga += g * s_h[0][ty + j][tx]; gb += g * s_h[1][ty + j][tx]; gc += g * s_h[2][ty + j][tx];
        }
        if (px < W && py < H) {
            const int64_t p = ((int64_t)py * W + px) * 3 + c;
            const float yp = y[p], tp = t[p];
            float d = gscale * (ga + 2.f * yp * gb + tp * gc);
            if (part_l1) d = l1_scale * sgn(yp - tp) + d;
            dldy[p] = accumulate ? dldy[p] + d : d;
        }
    }
}

// Scratch floats of the SSIM term: 9 per pixel (the maps), then two per (16 x 16 tile,
// channel) (the partial sums of S, then those of |y - t|).
size_t dssim_scratch_floats(int W, int H) {
    if (W <= 0 || H <= 0) return 0;
    const size_t tiles = (size_t)((W + kSsimT - 1) / kSsimT) * (size_t)((H + kSsimT - 1) / kSsimT);
    return (size_t)9 * (size_t)W * (size_t)H + 6 * tiles;
}

// maps: dssim_scratch_floats(W, H) floats of scratch. loss <- weight (1 - mean S); dL/dy
// (=, or += with accumulate) -weight dS/dy averaged over 3 H W values.
// with_l1: also the L1 term, l1_scale sum |y - t| and its gradient (eq. 4 and eq. 7 in one pass)
void launch_dssim(const float *y, const float *t, int W, int H, float weight, float *dldy, int accumulate, float *loss,
                  float *maps, hipStream_t st, int with_l1, float l1_scale) {
    SsimWindow win;
    double g[2 * kSsimR + 1], sum = 0.0;
    for (int j = 0; j <= 2 * kSsimR; ++j) {
        const double r = j - kSsimR;
        g[j] = std::exp(-(r * r) / (2.0 * 1.5 * 1.5));
        sum += g[j];
    }
    for (int j = 0; j <= 2 * kSsimR; ++j) win.g[j] = (float)(g[j] / sum);
    if (W <= 0 || H <= 0) {   // no pixels: weight (1 - SSIM) with SSIM taken as 0
        uint32_t wbits;
        std::memcpy(&wbits, &weight, 4);
        launch_fill_u32(reinterpret_cast<uint32_t *>(loss), wbits, 1, st);
        return;
    }
    const double N = 3.0 * (double)W * (double)H;
    const dim3 grid((unsigned)((W + kSsimT - 1) / kSsimT), (unsigned)((H + kSsimT - 1) / kSsimT), 3u);
    const uint32_t nparts = grid.x * grid.y * grid.z;
    float *part = maps + (size_t)9 * (size_t)W * (size_t)H;
    float *part_l1 = with_l1 ? part + nparts : nullptr;
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, st, y, t, W, H, win, maps, part, part_l1);
    hipLaunchKernelGGL(k_ssim_bwd, dim3(grid.x, grid.y), dim3(256), 0, st, y, t, W, H, win, maps, (float)(-weight / N),
                       accumulate, dldy, part, nparts, weight, loss, part_l1, l1_scale);
}

}  // namespace recogs
