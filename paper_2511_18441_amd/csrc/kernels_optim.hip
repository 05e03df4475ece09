// Pieces of the background optimiser (Sec. 3.3 / 4.1): the L1 term of the loss of
// eq. 7 with its gradient, and the Adam step that moves the SH coefficients.
#include "recogs_internal.hpp"

namespace recogs {

// loss = scale sum |y - t| (overwritten by the caller's fill), dL/dy = scale sign(y - t)
// with sign(0) = 0. With vec (all three arrays 16-byte aligned) 4 elements per step.
__device__ __forceinline__ float sgn(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__global__ __launch_bounds__(256) void k_loss_l1(const float *__restrict__ y, const float *__restrict__ tg, int64_t count,
                                                 float scale, float *__restrict__ dldy, float *__restrict__ loss, int vec) {
    __shared__ float s_w[4];
    float sum = 0.f;
    const int64_t n4 = vec ? count / 4 : 0;
    const float4 *y4 = reinterpret_cast<const float4 *>(y), *t4 = reinterpret_cast<const float4 *>(tg);
    float4 *d4 = reinterpret_cast<float4 *>(dldy);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 a = y4[i], b = t4[i];
        const float4 d = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
        d4[i] = make_float4(scale * sgn(d.x), scale * sgn(d.y), scale * sgn(d.z), scale * sgn(d.w));
        sum += fabsf(d.x) + fabsf(d.y) + fabsf(d.z) + fabsf(d.w);
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const float d = y[i] - tg[i];
        dldy[i] = scale * sgn(d);
        sum += fabsf(d);
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, scale * (s_w[0] + s_w[1] + s_w[2] + s_w[3]));
}

void launch_loss_l1(const float *y, const float *tg, int64_t count, float scale, float *dldy, float *loss, hipStream_t st) {
    if (count <= 0) return;
    // few workgroups: each adds its partial sum with one same-address atomic
    int64_t blocks = (count + 255) / 256;
    if (blocks > 512) blocks = 512;
    const int vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(tg) | reinterpret_cast<uintptr_t>(dldy)) &
                     15u) == 0;
    hipLaunchKernelGGL(k_loss_l1, dim3((unsigned)blocks), dim3(256), 0, st, y, tg, count, scale, dldy, loss, vec);
}

// Adam, element-wise: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - lr (m / c1) / (sqrt(v / c2) + eps) with the bias corrections c1 = 1 - b1^step,
// c2 = 1 - b2^step (computed by the host in double precision).
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, int64_t count, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * (gi * gi);
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, p, g, m, v, count, lr, b1, b2, eps, c1, c2);
}

}  // namespace recogs
