// Render path kernels: preprocess (EWA projection, SH colour, tile rectangle),
// exclusive scan of tile counts, key emission, tile ranges, front-to-back blend.
#include "recogs_internal.hpp"

namespace recogs {

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

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

// ---------------------------------------------------------------------------
// Preprocess: one thread per Gaussian.
//   m = R mu + t (compensated); cull depth <= znear.
//   EWA: J at the 1.3x-frustum-clamped position, Sigma2D = J R Sigma R^T J^T + 0.3 I.
//   Cull det <= 0 and 255 sigma < 1. Box of q <= 2 ln(255 sigma) + 1/64 -> pixel range
//   [ceil(u - ex - 1/2), floor(u + ex - 1/2)] clipped -> tile rectangle and count.
//   Colour max(0, f + 1/2) or, for selected Gaussians of a fused recolour,
//   max(0, M (f + 1/2) + b).
// Writes the splat record, depth bits, packed tile rectangle and count; folds the
// depth range of Gaussians with keys into the workspace header.
// ---------------------------------------------------------------------------
template <int DT, int DEG>
__global__ __launch_bounds__(256) void k_preprocess(SceneDev sc, CamDev cam, RecolorDev rc, int keep_bwd,
                                                    SplatRec *__restrict__ rec, float4 *__restrict__ bwd,
                                                    uint32_t *__restrict__ zbits, uint2 *__restrict__ rect,
                                                    uint32_t *__restrict__ count, uint32_t *__restrict__ header) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t cnt = 0, zb = 0;
    uint2 rr = make_uint2(0u, 0u);
    if (i < sc.n) {
        const int64_t S = sc.stride;
        const float mx = sc.means[i], my = sc.means[S + i], mz = sc.means[2 * S + i];
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
                    const float fx0 = fmaxf(ceilf(u - ex - 0.5f), 0.f), fx1 = fminf(floorf(u + ex - 0.5f), (float)(cam.W - 1));
                    const float fy0 = fmaxf(ceilf(v - ey - 0.5f), 0.f), fy1 = fminf(floorf(v + ey - 0.5f), (float)(cam.H - 1));
                    if (fx0 <= fx1 && fy0 <= fy1) {
                        const uint32_t tx0 = (uint32_t)fx0 / cam.tw, tx1 = (uint32_t)fx1 / cam.tw;
                        const uint32_t ty0 = (uint32_t)fy0 / cam.th, ty1 = (uint32_t)fy1 / cam.th;
                        cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                        rr = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
                        // colour (eq. 2) at the view direction of the centre
                        float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
                        const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
                        dx *= inv; dy *= inv; dz *= inv;
                        constexpr int NC = (DEG + 1) * (DEG + 1);
                        float Y[16];
                        sh_basis<DEG>(dx, dy, dz, Y);
                        float f[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            float acc = 0.f;
#pragma unroll
                            for (int k = 0; k < NC; ++k) acc += Store<DT>::ld(sc.sh, (int64_t)(k * 3 + c) * S + i) * Y[k];
                            f[c] = acc + 0.5f;
                        }
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
                        rec[i] = s;
                        if (keep_bwd) bwd[i] = make_float4(f[0], f[1], f[2], __uint_as_float(flags));
                    }
                }
            }
        }
        count[i] = cnt;
        rect[i] = rr;
        zbits[i] = zb;
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of the tile counts, reduce-then-scan (no waiting between
// workgroups). Besides the key offsets it produces
//   - the compaction of the Gaussians with keys (index order kept) into
//     (depth bits, index) pairs, the input of the depth sort;
//   - the depth range (min / max depth bits of Gaussians with keys).
// reduce: per chunk of 4,096 Gaussians the key count, the count of Gaussians with
// keys and the depth range; top: one workgroup scans the chunk partials and writes
// the totals K, V and the depth range to the header; down: per chunk, offsets and
// compaction from the chunk's prefixes.
// ---------------------------------------------------------------------------
template <typename T, int NW>
__device__ __forceinline__ T block_excl_scan(T v, T *s_w, T &total) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const T inc = wave_incl_scan(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    T pre = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const T x = s_w[k];
        if (k < (int)w) pre += x;
        total += x;
    }
    __syncthreads();
    return pre + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ zbits,
                                                     int64_t n, uint64_t *__restrict__ pk, uint32_t *__restrict__ pv,
                                                     uint32_t *__restrict__ pzmn, uint32_t *__restrict__ pzmx) {
    __shared__ uint64_t s_k[4];
    __shared__ uint32_t s_v[4], s_zmn[4], s_zmx[4];
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint64_t tsum = 0;
    uint32_t vsum = 0, zmn = 0xffffffffu, zmx = 0u;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t v = (base + k < n) ? cnt[base + k] : 0u;
        tsum += v;
        if (v) {
            const uint32_t z = zbits[base + k];
            zmn = min(zmn, z);
            zmx = max(zmx, z);
            ++vsum;
        }
    }
    tsum = wave_sum(tsum);
    vsum = wave_sum(vsum);
    zmn = wave_min(zmn);
    zmx = wave_max(zmx);
    if (lane == 0) { s_k[w] = tsum; s_v[w] = vsum; s_zmn[w] = zmn; s_zmx[w] = zmx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        pk[blockIdx.x] = s_k[0] + s_k[1] + s_k[2] + s_k[3];
        pv[blockIdx.x] = s_v[0] + s_v[1] + s_v[2] + s_v[3];
        pzmn[blockIdx.x] = min(min(s_zmn[0], s_zmn[1]), min(s_zmn[2], s_zmn[3]));
        pzmx[blockIdx.x] = max(max(s_zmx[0], s_zmx[1]), max(s_zmx[2], s_zmx[3]));
    }
}

// One workgroup: exclusive scans of the chunk partials in place; header gets K, V and
// the depth range (minimum stored as its complement).
__global__ __launch_bounds__(1024) void k_scan_top(uint64_t *__restrict__ pk, uint32_t *__restrict__ pv,
                                                   const uint32_t *__restrict__ pzmn, const uint32_t *__restrict__ pzmx,
                                                   uint32_t nchunks, uint32_t *__restrict__ header) {
    __shared__ uint64_t s_wk[16];
    __shared__ uint32_t s_wv[16], s_zmn[16], s_zmx[16];
    const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
    uint64_t runk = 0;
    uint32_t runv = 0, zmn = 0xffffffffu, zmx = 0u;
    for (uint32_t c0 = 0; c0 < nchunks; c0 += 1024) {
        const uint32_t c = c0 + t;
        const uint64_t k = c < nchunks ? pk[c] : 0ull;
        const uint32_t v = c < nchunks ? pv[c] : 0u;
        if (c < nchunks) { zmn = min(zmn, pzmn[c]); zmx = max(zmx, pzmx[c]); }
        uint64_t ktot;
        uint32_t vtot;
        const uint64_t ek = block_excl_scan<uint64_t, 16>(k, s_wk, ktot);
        const uint32_t ev = block_excl_scan<uint32_t, 16>(v, s_wv, vtot);
        if (c < nchunks) { pk[c] = runk + ek; pv[c] = runv + ev; }
        runk += ktot;
        runv += vtot;
    }
    zmn = wave_min(zmn);
    zmx = wave_max(zmx);
    if (lane == 0) { s_zmn[w] = zmn; s_zmx[w] = zmx; }
    __syncthreads();
    if (t == 0) {
        for (int k = 1; k < 16; ++k) { zmn = min(zmn, s_zmn[k]); zmx = max(zmx, s_zmx[k]); }
        zmn = min(zmn, s_zmn[0]);
        zmx = max(zmx, s_zmx[0]);
        header[H_K_LO] = (uint32_t)runk;
        header[H_K_HI] = (uint32_t)(runk >> 32);
        header[H_V] = runv;
        header[H_ZMIN] = runv ? ~zmn : 0u;
        header[H_ZMAX] = runv ? zmx : 0u;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ zbits,
                                                   uint32_t *__restrict__ off, int64_t n, const uint64_t *__restrict__ pk,
                                                   const uint32_t *__restrict__ pv, uint32_t *__restrict__ dkeys,
                                                   uint32_t *__restrict__ dvals) {
    __shared__ uint64_t s_wk[4];
    __shared__ uint32_t s_wv[4];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint64_t tsum = 0;
    uint32_t vsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? cnt[base + k] : 0u;
        tsum += v[k];
        vsum += v[k] ? 1u : 0u;
    }
    uint64_t ktot;
    uint32_t vtot;
    uint64_t run = pk[blockIdx.x] + block_excl_scan<uint64_t, 4>(tsum, s_wk, ktot);
    uint32_t vrun = pv[blockIdx.x] + block_excl_scan<uint32_t, 4>(vsum, s_wv, vtot);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) off[base + k] = (uint32_t)run;
        run += v[k];
        if (v[k]) {
            dkeys[vrun] = zbits[base + k];
            dvals[vrun] = (uint32_t)(base + k);
            ++vrun;
        }
    }
}

// One workgroup: exclusive scan in place of a u32 array of chunk partials.
__global__ __launch_bounds__(1024) void k_scan_top_u32(uint32_t *__restrict__ a, uint32_t count) {
    __shared__ uint32_t s_w[16];
    uint32_t run = 0;
    for (uint32_t c0 = 0; c0 < count; c0 += 1024) {
        const uint32_t c = c0 + threadIdx.x;
        const uint32_t v = c < count ? a[c] : 0u;
        uint32_t tot;
        const uint32_t e = block_excl_scan<uint32_t, 16>(v, s_w, tot);
        if (c < count) a[c] = run + e;
        run += tot;
    }
}

// ---------------------------------------------------------------------------
// Key emission, wave-cooperative: a wave owns 64 consecutive Gaussians, whose keys
// occupy one contiguous range (the scan is exclusive). Lane j writes keys j, j+64, ...
// of that range, finding the owning Gaussian by binary search over the wave's
// prefix sums, so stores are coalesced however uneven the tile counts are.
// key = (tile << 32) | float32 depth bits, value = Gaussian index; within a
// Gaussian tiles go in row-major order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_emit(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ off,
                                              const uint2 *__restrict__ rect, const uint32_t *__restrict__ zbits,
                                              int64_t n, int tiles_x, uint64_t *__restrict__ keys,
                                              uint32_t *__restrict__ vals) {
    __shared__ uint32_t s_ex[4][64];
    __shared__ uint2 s_rect[4][64];
    __shared__ uint32_t s_zb[4][64];
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const int64_t g0 = ((int64_t)blockIdx.x * 4 + w) * 64;
    const int64_t g = g0 + lane;
    uint32_t c = 0, o = 0, zb = 0;
    uint2 r = make_uint2(0u, 0u);
    if (g < n) {
        c = cnt[g];
        o = off[g];
        if (c) { r = rect[g]; zb = zbits[g]; }
    }
    const uint32_t inc = wave_incl_scan(c);
    const uint32_t total = __shfl(inc, 63, 64);
    const uint32_t base = __shfl(o, 0, 64);
    s_ex[w][lane] = inc - c;
    s_rect[w][lane] = r;
    s_zb[w][lane] = zb;
    __syncthreads();
    for (uint32_t j = lane; j < total; j += 64) {
        int lo = 0, hi = 63;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_ex[w][mid] <= j) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t k = j - s_ex[w][lo];
        const uint2 rr = s_rect[w][lo];
        const uint32_t tx0 = rr.x & 0xffffu, tx1 = rr.x >> 16, ty0 = rr.y & 0xffffu;
        const uint32_t wd = tx1 - tx0 + 1;
        const uint32_t ty = ty0 + k / wd, tx = tx0 + k % wd;
        keys[base + j] = ((uint64_t)(ty * (uint32_t)tiles_x + tx) << 32) | s_zb[w][lo];
        vals[base + j] = (uint32_t)(g0 + lo);
    }
}

// ---------------------------------------------------------------------------
// Key emission in depth order: the Gaussians with keys, already sorted by (depth,
// index), emit (tile id, index) pairs; a stable sort on the tile id then yields the
// (tile, depth, index) order. Reduce-then-scan over chunks of 1,024 depth-ordered
// Gaussians: k_emit_reduce sums each chunk's tile counts, k_scan_top_u32 turns the
// sums into chunk offsets, k_emit_down writes. In k_emit_down wave w handles groups
// r of 64 consecutive Gaussians; a group's keys form one contiguous range, written
// cooperatively (coalesced stores, owner found by binary search over the group's
// prefix sums).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t rect_count(uint2 r) {
    return ((r.x >> 16) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.y & 0xffffu) + 1u);
}

// also gathers each depth-ordered Gaussian's tile rectangle once (srect, coalesced
// for k_emit_down); every Gaussian in the order has at least one key
__global__ __launch_bounds__(256) void k_emit_reduce(const uint32_t *__restrict__ order, uint32_t V,
                                                     const uint2 *__restrict__ rect, uint2 *__restrict__ srect,
                                                     uint32_t *__restrict__ esum) {
    __shared__ uint32_t s_w[4];
    const uint32_t base = blockIdx.x * (uint32_t)kEmitChunk + threadIdx.x;
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kEmitItems; ++r) {
        const uint32_t j = base + r * 256;
        if (j < V) {
            const uint2 rc = rect[order[j]];
            srect[j] = rc;
            sum += rect_count(rc);
        }
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) esum[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ __launch_bounds__(256) void k_emit_down(const uint32_t *__restrict__ order, uint32_t V,
                                                   const uint2 *__restrict__ srect, int tiles_x,
                                                   const uint32_t *__restrict__ epre, uint32_t *__restrict__ tkeys,
                                                   uint32_t *__restrict__ tvals) {
    constexpr int R = kEmitItems;
    __shared__ uint32_t s_gsum[4 * R];     // per-group totals, then per-group exclusive prefix
    __shared__ uint32_t s_ex[4][64];
    __shared__ uint2 s_rect[4][64];
    __shared__ uint32_t s_g[4][64];
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const uint32_t j0 = blockIdx.x * (uint32_t)kEmitChunk + w * (64 * R) + lane;
    uint32_t c[R], inc[R], g[R];
    uint2 rr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t j = j0 + r * 64;
        g[r] = j < V ? order[j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t j = j0 + r * 64;
        rr[r] = j < V ? srect[j] : make_uint2(0u, 0u);
        c[r] = j < V ? rect_count(rr[r]) : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        inc[r] = wave_incl_scan(c[r]);
        if (lane == 63) s_gsum[w * R + r] = inc[r];
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive scan of the 4R group totals (one wave)
        const uint32_t v = threadIdx.x < 4 * R ? s_gsum[threadIdx.x] : 0u;
        const uint32_t x = wave_incl_scan(v);
        if (threadIdx.x < 4 * R) s_gsum[threadIdx.x] = x - v;
    }
    __syncthreads();
    const uint32_t cbase = epre[blockIdx.x];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        s_ex[w][lane] = inc[r] - c[r];
        s_rect[w][lane] = rr[r];
        s_g[w][lane] = g[r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t base = cbase + s_gsum[w * R + r];
        const uint32_t gtotal = __shfl(inc[r], 63, 64);
        for (uint32_t q = lane; q < gtotal; q += 64) {
            int lo = 0, hi = 63;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_ex[w][mid] <= q) lo = mid;
                else hi = mid - 1;
            }
            const uint32_t k = q - s_ex[w][lo];
            const uint2 rc = s_rect[w][lo];
            const uint32_t tx0 = rc.x & 0xffffu, tx1 = rc.x >> 16, ty0 = rc.y & 0xffffu;
            const uint32_t wd = tx1 - tx0 + 1;
            const uint32_t ty = ty0 + k / wd, tx = tx0 + k % wd;
            tkeys[base + q] = ty * (uint32_t)tiles_x + tx;
            tvals[base + q] = s_g[w][lo];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// [first, last+1) of each tile in tile-sorted 32-bit tile ids (ranges zeroed beforehand).
__global__ __launch_bounds__(256) void k_ranges32(const uint32_t *__restrict__ tiles, uint32_t K, uint2 *__restrict__ ranges) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const uint32_t t = tiles[k];
    if (k == 0 || tiles[k - 1] != t) ranges[t].x = k;
    if (k == K - 1 || tiles[k + 1] != t) ranges[t].y = k + 1;
}

// [first, last+1) of each tile in the sorted keys (ranges zeroed beforehand).
__global__ __launch_bounds__(256) void k_ranges(const uint64_t *__restrict__ keys, uint32_t K, uint2 *__restrict__ ranges) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const uint32_t t = (uint32_t)(keys[k] >> 32);
    if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[t].x = k;
    if (k == K - 1 || (uint32_t)(keys[k + 1] >> 32) != t) ranges[t].y = k + 1;
}

// ---------------------------------------------------------------------------
// Blend (eq. 3), one workgroup per tile (see TileMap for the thread -> pixel map).
// Splat records of the tile's sorted list are staged through LDS in batches; while
// staging, each record gets a bit mask of the wave regions its alpha >= 1/255 box
// meets, so a wave skips a splat with one scalar test. Per pixel: alpha =
// min(0.99, 2^e) with e from exp_row/exp_at, skipped below 1/255; the pixel stops
// when blending would drop transmittance below 1e-4; the workgroup stops when all
// its pixels have. Output HWC image, final transmittance and, per pixel, the count
// of tile-list entries up to and including the last blended one.
// ---------------------------------------------------------------------------
template <int TW, int TH, int PPT>
__global__ __launch_bounds__(TW *TH / PPT) void k_blend(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                                       const SplatRec *__restrict__ rec, int W, int H, int tiles_x,
                                                       float bg0, float bg1, float bg2, float *__restrict__ image,
                                                       float *__restrict__ finalT, uint32_t *__restrict__ nproc) {
#pragma clang fp contract(off)
    using Map = TileMap<TW, TH, PPT>;
    constexpr int NT = Map::NT;
    constexpr int BATCH = 256;
    __shared__ float4 s_r0[BATCH], s_r1[BATCH], s_r2[BATCH];
    __shared__ uint8_t s_mask[BATCH];
    const int tile = blockIdx.x;
    const int tx0 = (tile % tiles_x) * TW, ty0 = (tile / tiles_x) * TH;
    const int t = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(Map::wave(t));
    int lx, lrow;
    Map::pixel(t, lx, lrow);
    const int px = tx0 + lx;
    const float pxc = (float)px + 0.5f;
    float pyc[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
    uint32_t last[PPT];
    bool done[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = ty0 + lrow * PPT + j;
        pyc[j] = (float)py + 0.5f;
        T[j] = 1.f; C0[j] = C1[j] = C2[j] = 0.f; last[j] = 0;
        done[j] = !(px < W && py < H);
    }

    const uint2 rg = ranges[tile];
    for (uint32_t start = rg.x; start < rg.y; start += BATCH) {
        bool mine = true;
#pragma unroll
        for (int j = 0; j < PPT; ++j) mine = mine && done[j];
        if (__syncthreads_and(mine)) break;
        for (int q = t; q < BATCH; q += NT) {
            const uint32_t k = start + q;
            if (k < rg.y) {
                const SplatRec s = rec[vals[k]];
                s_r0[q] = s.r0; s_r1[q] = s.r1; s_r2[q] = s.r2;
                s_mask[q] = (uint8_t)Map::wave_mask(s.r0, (float)tx0, (float)ty0);
            }
        }
        __syncthreads();
        const int nb = (int)min((uint32_t)BATCH, rg.y - start);
        const uint32_t krel0 = start + 1 - rg.x;
        for (int q = 0; q < nb; ++q) {
            bool alive = false;
#pragma unroll
            for (int j = 0; j < PPT; ++j) alive = alive || !done[j];
            if (!wave_ballot(alive)) break;
            const uint32_t m = __builtin_amdgcn_readfirstlane((uint32_t)s_mask[q]);
            if (!((m >> w) & 1u)) continue;
            const float4 r0 = s_r0[q], r1 = s_r1[q], r2 = s_r2[q];
            const ExpRow er = exp_row(r1, pxc - r0.x);
            const uint32_t kq = krel0 + (uint32_t)q;
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                if (done[j]) continue;
                const float e = exp_at(er, r1, pyc[j] - r0.y);
                if (e < kLog2AlphaMin) continue;
                const float a = fminf(kAlphaMax, __builtin_amdgcn_exp2f(e));
                const float Tn = T[j] * (1.f - a);
                if (Tn < kTMin) { done[j] = true; continue; }
                const float wgt = a * T[j];
                C0[j] = __builtin_fmaf(r2.x, wgt, C0[j]);
                C1[j] = __builtin_fmaf(r2.y, wgt, C1[j]);
                C2[j] = __builtin_fmaf(r2.z, wgt, C2[j]);
                T[j] = Tn;
                last[j] = kq;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = ty0 + lrow * PPT + j;
        if (px < W && py < H) {
            const int64_t p = (int64_t)py * W + px;
            image[p * 3 + 0] = __builtin_fmaf(T[j], bg0, C0[j]);
            image[p * 3 + 1] = __builtin_fmaf(T[j], bg1, C1[j]);
            image[p * 3 + 2] = __builtin_fmaf(T[j], bg2, C2[j]);
            finalT[p] = T[j];
            nproc[p] = last[j];
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
}

template <int DT>
static void preprocess_dt(int deg, dim3 g, hipStream_t st, const SceneDev &sc, const CamDev &cam, const RecolorDev &rc,
                          int keep, SplatRec *rec, float4 *bwd, uint32_t *zb, uint2 *rect, uint32_t *cnt, uint32_t *hdr) {
    switch (deg) {
    case 0: hipLaunchKernelGGL((k_preprocess<DT, 0>), g, dim3(256), 0, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr); break;
    case 1: hipLaunchKernelGGL((k_preprocess<DT, 1>), g, dim3(256), 0, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr); break;
    case 2: hipLaunchKernelGGL((k_preprocess<DT, 2>), g, dim3(256), 0, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr); break;
    default: hipLaunchKernelGGL((k_preprocess<DT, 3>), g, dim3(256), 0, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr); break;
    }
}

void launch_preprocess(int dt, int deg, const SceneDev &sc, const CamDev &cam, const RecolorDev &rc, int keep,
                       SplatRec *rec, float4 *bwd, uint32_t *zb, uint2 *rect, uint32_t *cnt, uint32_t *hdr,
                       hipStream_t st) {
    if (sc.n <= 0) return;
    const dim3 g((unsigned)((sc.n + 255) / 256));
    if (dt == RECOGS_F32) preprocess_dt<RECOGS_F32>(deg, g, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr);
    else if (dt == RECOGS_F16) preprocess_dt<RECOGS_F16>(deg, g, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr);
    else preprocess_dt<RECOGS_BF16>(deg, g, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, hdr);
}

void launch_scan(const uint32_t *cnt, const uint32_t *zbits, uint32_t *off, int64_t n, uint64_t *pk, uint32_t *pv,
                 uint32_t *pzmn, uint32_t *pzmx, uint32_t *dkeys, uint32_t *dvals, uint32_t *hdr, hipStream_t st) {
    if (n <= 0) return;
    const uint32_t nchunks = (uint32_t)((n + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nchunks), dim3(256), 0, st, cnt, zbits, n, pk, pv, pzmn, pzmx);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, pk, pv, pzmn, pzmx, nchunks, hdr);
    hipLaunchKernelGGL(k_scan_down, dim3(nchunks), dim3(256), 0, st, cnt, zbits, off, n, pk, pv, dkeys, dvals);
}

void launch_emit_sorted(const uint32_t *order, uint32_t V, const uint2 *rect, uint2 *srect, int tiles_x,
                        uint32_t *esum, uint32_t *tkeys, uint32_t *tvals, hipStream_t st) {
    if (V == 0) return;
    const uint32_t chunks = (V + kEmitChunk - 1) / kEmitChunk;
    hipLaunchKernelGGL(k_emit_reduce, dim3(chunks), dim3(256), 0, st, order, V, rect, srect, esum);
    hipLaunchKernelGGL(k_scan_top_u32, dim3(1), dim3(1024), 0, st, esum, chunks);
    hipLaunchKernelGGL(k_emit_down, dim3(chunks), dim3(256), 0, st, order, V, srect, tiles_x, esum, tkeys, tvals);
}

void launch_ranges32(const uint32_t *tiles, uint32_t K, uint2 *ranges, hipStream_t st) {
    if (K == 0) return;
    hipLaunchKernelGGL(k_ranges32, dim3((K + 255) / 256), dim3(256), 0, st, tiles, K, ranges);
}

void launch_emit(const uint32_t *cnt, const uint32_t *off, const uint2 *rect, const uint32_t *zb, int64_t n, int tiles_x,
                 uint64_t *keys, uint32_t *vals, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cnt, off, rect, zb, n, tiles_x, keys, vals);
}

void launch_ranges(const uint64_t *keys, uint32_t K, uint2 *ranges, hipStream_t st) {
    if (K == 0) return;
    hipLaunchKernelGGL(k_ranges, dim3((K + 255) / 256), dim3(256), 0, st, keys, K, ranges);
}

template <int TW, int TH, int PPT>
static void blend_one(int ntiles, hipStream_t st, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec, int W,
                      int H, int tiles_x, const float *bg, float *image, float *finalT, uint32_t *nproc) {
    hipLaunchKernelGGL((k_blend<TW, TH, PPT>), dim3(ntiles), dim3(TW * TH / PPT), 0, st, ranges, vals, rec, W, H, tiles_x,
                       bg[0], bg[1], bg[2], image, finalT, nproc);
}

bool launch_blend(int tw, int th, int ppt, int ntiles, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec,
                  int W, int H, int tiles_x, const float *bg, float *image, float *finalT, uint32_t *nproc,
                  hipStream_t st) {
#define RECOGS_BLEND_CASE(A, B, P)                                                                         \
    if (tw == A && th == B && ppt == P) {                                                                  \
        blend_one<A, B, P>(ntiles, st, ranges, vals, rec, W, H, tiles_x, bg, image, finalT, nproc);        \
        return true;                                                                                       \
    }
    RECOGS_BLEND_CASE(16, 16, 1) RECOGS_BLEND_CASE(16, 16, 2) RECOGS_BLEND_CASE(16, 16, 4)
    RECOGS_BLEND_CASE(8, 8, 1) RECOGS_BLEND_CASE(8, 8, 2) RECOGS_BLEND_CASE(8, 8, 4)
    RECOGS_BLEND_CASE(32, 8, 1) RECOGS_BLEND_CASE(32, 8, 2) RECOGS_BLEND_CASE(32, 8, 4)
#undef RECOGS_BLEND_CASE
    return false;
}

}  // namespace recogs
