// Per-Gaussian streaming kernels: covariance (eq. 1), selection, recolour (eq. 6).
// One thread per Gaussian, planar (SoA) loads: consecutive lanes read consecutive
// elements of each plane.
#include "recogs_internal.hpp"

namespace recogs {

// eq. (1): Sigma = R S S^T R^T, S = diag(exp(log_scale)), R from the normalised
// quaternion (w, x, y, z).
__global__ __launch_bounds__(256) void k_covariance(const float *__restrict__ ls, const float *__restrict__ q,
                                                    float *__restrict__ cov, int64_t n, int64_t stride) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float w = q[i], x = q[stride + i], y = q[2 * stride + i], z = q[3 * stride + i];
    const float inv = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    const float R00 = 1.f - 2.f * (y * y + z * z), R01 = 2.f * (x * y - w * z), R02 = 2.f * (x * z + w * y);
    const float R10 = 2.f * (x * y + w * z), R11 = 1.f - 2.f * (x * x + z * z), R12 = 2.f * (y * z - w * x);
    const float R20 = 2.f * (x * z - w * y), R21 = 2.f * (y * z + w * x), R22 = 1.f - 2.f * (x * x + y * y);
    const float s0 = expf(ls[i]), s1 = expf(ls[stride + i]), s2 = expf(ls[2 * stride + i]);
    const float M00 = R00 * s0, M01 = R01 * s1, M02 = R02 * s2;
    const float M10 = R10 * s0, M11 = R11 * s1, M12 = R12 * s2;
    const float M20 = R20 * s0, M21 = R21 * s1, M22 = R22 * s2;
    cov[i] = M00 * M00 + M01 * M01 + M02 * M02;
    cov[stride + i] = M00 * M10 + M01 * M11 + M02 * M12;
    cov[2 * stride + i] = M00 * M20 + M01 * M21 + M02 * M22;
    cov[3 * stride + i] = M10 * M10 + M11 * M11 + M12 * M12;
    cov[4 * stride + i] = M10 * M20 + M11 * M21 + M12 * M22;
    cov[5 * stride + i] = M20 * M20 + M21 * M21 + M22 * M22;
}

// Selection: depth > znear, projected centre in the closed disk, DC colour in the
// closed ball. The count is reduced per workgroup (wave ballots, then LDS) and added
// with one atomic per workgroup: same-address device atomics are serialised far
// from the CU, so a grid-stride loop over at most kSelectBlocks workgroups bounds them.
constexpr unsigned kSelectBlocks = 1024;

template <int DT>
__global__ __launch_bounds__(256) void k_select(SceneDev sc, CamDev cam, float scx, float scy, float r2,
                                                float ref0, float ref1, float ref2, float rho2,
                                                uint8_t *__restrict__ mask, int32_t *__restrict__ count) {
    __shared__ uint32_t s_cnt[4];
    uint32_t wave_cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i - threadIdx.x < sc.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool sel = false;
        if (i < sc.n) {
            const float mx = sc.means[i], my = sc.means[sc.stride + i], mz = sc.means[2 * sc.stride + i];
            const float z = dot3c(cam.R[6], mx, cam.R[7], my, cam.R[8], mz, cam.t[2]);
            if (z > cam.znear) {
                const float x = dot3c(cam.R[0], mx, cam.R[1], my, cam.R[2], mz, cam.t[0]);
                const float y = dot3c(cam.R[3], mx, cam.R[4], my, cam.R[5], mz, cam.t[1]);
                const float u = cam.fx * (x / z) + cam.cx, v = cam.fy * (y / z) + cam.cy;
                const float du = u - scx, dv = v - scy;
                const float d2 = du * du + dv * dv;
                const float c0 = kSH0 * Store<DT>::ldc(sc.sh, i) + 0.5f - ref0;
                const float c1 = kSH0 * Store<DT>::ldc(sc.sh, sc.stride + i) + 0.5f - ref1;
                const float c2 = kSH0 * Store<DT>::ldc(sc.sh, 2 * sc.stride + i) + 0.5f - ref2;
                sel = (d2 <= r2) && (c0 * c0 + c1 * c1 + c2 * c2 <= rho2);
            }
            mask[i] = sel ? 1 : 0;
        }
        wave_cnt += (uint32_t)__popcll(wave_ballot(sel));
    }
    if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = wave_cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t c = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        if (c) atomicAdd(count, (int32_t)c);
    }
}

// Recolour on coefficients: C'_k = M C_k (k >= 1), C'_0 = M C_0 + ((M - I) 1/2 + b)/Y00.
// A thread reads the mask bytes of four consecutive Gaussians with one load.
constexpr int kRecolorPer = 4;
template <int DT>
__global__ __launch_bounds__(256) void k_recolor(SceneDev sc, int ncoef, void *__restrict__ dst,
                                                 const uint8_t *__restrict__ mask, const float *__restrict__ Mp,
                                                 const float *__restrict__ bp, int copy_unselected) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRecolorPer;
    // the matrix and offset (uniform) are loaded with the mask, not after it
    float M[9], bb[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = Mp[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) bb[r] = bp[r];
    uint32_t sel = 0;   // byte k: Gaussian i0 + k selected
    if (i0 + kRecolorPer <= sc.n && ((uintptr_t)mask & 3u) == 0) {
        sel = *reinterpret_cast<const uint32_t *>(mask + i0);
    } else {
        for (int k = 0; k < kRecolorPer; ++k)
            if (i0 + k < sc.n && mask[i0 + k]) sel |= 1u << (8 * k);
    }
    if (copy_unselected && dst != sc.sh)
        for (int k = 0; k < kRecolorPer; ++k)
            if (i0 + k < sc.n && !((sel >> (8 * k)) & 0xffu))
                for (int p = 0; p < ncoef * 3; ++p)
                    Store<DT>::st(dst, p * sc.stride + i0 + k, Store<DT>::ldc(sc.sh, p * sc.stride + i0 + k));
    // The selected Gaussians of the wave (a sparse selection leaves one or two per wave)
    // are listed in index order in LDS; then each group of 16 lanes recolours one of them,
    // four at a time: lane k of a group takes coefficient k's three planes, so a Gaussian
    // costs three loads and three stores of up to 16 lanes each, and a wave's Gaussians
    // cost one memory round trip per four instead of one each. A lane loads its planes
    // before it stores them, so the destination may alias the source.
    __shared__ uint16_t s_list[4][64 * kRecolorPer];
    const uint64_t m = wave_ballot(sel != 0u);
    if (!m) return;
    const int l = (int)lane_id(), w = (int)(threadIdx.x >> 6);
    const uint32_t nsel_l = ((sel & 0xffu) ? 1u : 0u) + ((sel >> 8 & 0xffu) ? 1u : 0u) +
                            ((sel >> 16 & 0xffu) ? 1u : 0u) + ((sel >> 24) ? 1u : 0u);   // selected of the lane
    const uint32_t incl = wave_incl_scan(nsel_l);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    {
        uint32_t pos = incl - nsel_l;
#pragma unroll
        for (int k = 0; k < kRecolorPer; ++k)
            if ((sel >> (8 * k)) & 0xffu) s_list[w][pos++] = (uint16_t)(l * kRecolorPer + k);
    }
    wave_sync();   // the list written before any lane reads it
    float off[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) off[r] = ((M[r * 3] + M[r * 3 + 1] + M[r * 3 + 2] - 1.0f) * 0.5f + bb[r]) / kSH0;
    const int64_t wbase = i0 - (int64_t)l * kRecolorPer;   // the first Gaussian of lane 0
    const int grp = l >> 4, co = l & 15;
    for (uint32_t j0 = 0; j0 < total; j0 += 4) {
        const uint32_t j = j0 + (uint32_t)grp;
        if (j < total && co < ncoef) {
            const int64_t g = wbase + (int64_t)s_list[w][j];
            const float c0 = Store<DT>::ldc(sc.sh, (int64_t)(3 * co) * sc.stride + g);
            const float c1 = Store<DT>::ldc(sc.sh, (int64_t)(3 * co + 1) * sc.stride + g);
            const float c2 = Store<DT>::ldc(sc.sh, (int64_t)(3 * co + 2) * sc.stride + g);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                float v = M[r * 3] * c0 + M[r * 3 + 1] * c1 + M[r * 3 + 2] * c2;
                if (co == 0) v += off[r];
                Store<DT>::st(dst, (int64_t)(3 * co + r) * sc.stride + g, v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void launch_covariance(const float *ls, const float *q, float *cov, int64_t n, int64_t stride, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_covariance, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ls, q, cov, n, stride);
}

void launch_select(int dt, const SceneDev &sc, const CamDev &cam, const recogs_select_params &p, uint8_t *mask,
                   int32_t *count, hipStream_t st) {
    if (sc.n <= 0) return;
    const int64_t need = (sc.n + 255) / 256;
    const dim3 g((unsigned)(need < kSelectBlocks ? need : kSelectBlocks)), b(256);
    const float r2 = p.radius * p.radius, rho2 = p.color_radius * p.color_radius;
    if (dt == RECOGS_F32) hipLaunchKernelGGL(k_select<RECOGS_F32>, g, b, 0, st, sc, cam, p.cx, p.cy, r2, p.ref[0], p.ref[1], p.ref[2], rho2, mask, count);
    else if (dt == RECOGS_F16) hipLaunchKernelGGL(k_select<RECOGS_F16>, g, b, 0, st, sc, cam, p.cx, p.cy, r2, p.ref[0], p.ref[1], p.ref[2], rho2, mask, count);
    else hipLaunchKernelGGL(k_select<RECOGS_BF16>, g, b, 0, st, sc, cam, p.cx, p.cy, r2, p.ref[0], p.ref[1], p.ref[2], rho2, mask, count);
}

void launch_recolor(int dt, const SceneDev &sc, int ncoef, void *dst, const uint8_t *mask, const float *M,
                    const float *b, int copy_unselected, hipStream_t st) {
    if (sc.n <= 0) return;
    const int64_t threads = (sc.n + kRecolorPer - 1) / kRecolorPer;
    const dim3 g((unsigned)((threads + 255) / 256)), bl(256);
    if (dt == RECOGS_F32) hipLaunchKernelGGL(k_recolor<RECOGS_F32>, g, bl, 0, st, sc, ncoef, dst, mask, M, b, copy_unselected);
    else if (dt == RECOGS_F16) hipLaunchKernelGGL(k_recolor<RECOGS_F16>, g, bl, 0, st, sc, ncoef, dst, mask, M, b, copy_unselected);
    else hipLaunchKernelGGL(k_recolor<RECOGS_BF16>, g, bl, 0, st, sc, ncoef, dst, mask, M, b, copy_unselected);
}

}  // namespace recogs
