// Pixel selection around the renderer (Sec. 3.2, 3.3):
//   - unprojection of a 2D selection, thinned by a sampling mask, to world points
//     with a per-pixel depth (the rough depth map) and the camera;
//   - reprojection of a point cloud into a view as screen-space squares of one size,
//     depth-tested against the view's depth map: the view's selection mask;
//   - the tint c* = t c on the pixels a mask marks.
// All three are streaming per-pixel / per-point work (HBM and launch bound): no LDS
// tiling beyond the workgroup scan of the unprojection's compaction.
#include <atomic>
#include <mutex>

#include "recogs_internal.hpp"

namespace recogs {

constexpr int kUnpItems = 4;                      // pixels per thread (in 4 rounds of 256)
constexpr int kUnpBlock = 256 * kUnpItems;        // pixels per workgroup

__device__ __forceinline__ bool unp_take(const uint8_t *__restrict__ mask, const uint8_t *__restrict__ keep,
                                         const float *__restrict__ depth, int64_t p) {
    return mask[p] != 0 && (!keep || keep[p] != 0) && depth[p] > 0.f;
}

// Selected pixels per workgroup of kUnpBlock consecutive pixels.
__global__ __launch_bounds__(256) void k_unp_count(const uint8_t *__restrict__ mask, const uint8_t *__restrict__ keep,
                                                   const float *__restrict__ depth, int64_t P,
                                                   uint32_t *__restrict__ part) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kUnpBlock;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kUnpItems; ++k) {
        const int64_t p = base + k * 256 + threadIdx.x;
        c += (p < P && unp_take(mask, keep, depth, p)) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Exclusive scan of the nblk workgroup counts in place (one workgroup, chunks of
// 1024 with a running carry); the total goes to *count.
__global__ __launch_bounds__(1024) void k_unp_scan(uint32_t *__restrict__ part, uint32_t nblk,
                                                   uint32_t *__restrict__ count) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int l = (int)lane_id(), w = (int)(threadIdx.x >> 6);
    for (uint32_t c0 = 0; c0 < nblk; c0 += 1024) {
        const uint32_t i = c0 + threadIdx.x;
        const uint32_t v = i < nblk ? part[i] : 0u;
        uint32_t x = v;   // inclusive scan within the wave
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (l >= o) x += y;
        }
        if (l == 63) s_w[w] = x;
        __syncthreads();
        uint32_t before = s_carry;
        for (int k = 0; k < w; ++k) before += s_w[k];
        if (i < nblk) part[i] = before + x - v;
        __syncthreads();   // every read of s_w and s_carry before they change
        if (threadIdx.x == 1023) s_carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = s_carry;
}

// Writes the selected pixels' world points in pixel order: X = R^T (m - t) with the
// camera-space point m = d ((x + 1/2 - cx) / fx, (y + 1/2 - cy) / fy, 1). Points at
// output positions >= cap are not written (the count still includes them).
__global__ __launch_bounds__(256) void k_unp_write(const uint8_t *__restrict__ mask, const uint8_t *__restrict__ keep,
                                                   const float *__restrict__ depth, int64_t P, int W,
                                                   const uint32_t *__restrict__ part, CamDev cam,
                                                   float *__restrict__ pts, int64_t cap) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kUnpBlock;
    const int l = (int)lane_id(), w = (int)(threadIdx.x >> 6);
    uint32_t run = part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kUnpItems; ++k) {
        const int64_t p = base + k * 256 + threadIdx.x;
        const bool take = p < P && unp_take(mask, keep, depth, p);
        const uint64_t bal = __ballot(take);
        const uint32_t below = (uint32_t)__popcll(bal & ((1ull << l) - 1ull));
        if (l == 0) s_w[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = run;
        for (int q = 0; q < w; ++q) before += s_w[q];
        const uint32_t total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();   // s_w is rewritten in the next iteration
        if (take) {
            const int64_t o = (int64_t)before + below;
            if (o < cap) {
                const int x = (int)(p % W), y = (int)(p / W);
                const float d = depth[p];
                const float xc = ((float)x + 0.5f - cam.cx) / cam.fx;
                const float yc = ((float)y + 0.5f - cam.cy) / cam.fy;
                const float m0 = d * xc - cam.t[0], m1 = d * yc - cam.t[1], m2 = d - cam.t[2];
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    pts[j * cap + o] = __builtin_fmaf(cam.R[6 + j], m2, __builtin_fmaf(cam.R[3 + j], m1, cam.R[j] * m0));
            }
        }
        run += total;
    }
}

__global__ __launch_bounds__(256) void k_zero_u8(uint8_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// One thread per point: m = R X + t; points with z <= znear are not drawn. The square
// of half side h around (u, v) covers pixels x in [ceil(u - h - 1/2), ceil(u + h - 1/2))
// (centres in [u - h, u + h)), likewise y; a covered pixel is marked where the depth map
// is 0 or z <= d (1 + eps). Every thread writes the same value, so overlaps are benign.
__global__ __launch_bounds__(256) void k_reproject(const float *__restrict__ pts, int64_t n, int64_t stride, CamDev cam,
                                                   float h, const float *__restrict__ depth, float eps,
                                                   uint8_t *__restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float X0 = pts[i], X1 = pts[stride + i], X2 = pts[2 * stride + i];
    const float mx = __builtin_fmaf(cam.R[2], X2, __builtin_fmaf(cam.R[1], X1, __builtin_fmaf(cam.R[0], X0, cam.t[0])));
    const float my = __builtin_fmaf(cam.R[5], X2, __builtin_fmaf(cam.R[4], X1, __builtin_fmaf(cam.R[3], X0, cam.t[1])));
    const float z = __builtin_fmaf(cam.R[8], X2, __builtin_fmaf(cam.R[7], X1, __builtin_fmaf(cam.R[6], X0, cam.t[2])));
    if (!(z > cam.znear)) return;
    const float u = cam.fx * (mx / z) + cam.cx, v = cam.fy * (my / z) + cam.cy;
    // off-screen (or not finite): nothing to draw; keeps the conversions below in range
    if (!(u + h > -1.f && u - h < (float)cam.W + 1.f && v + h > -1.f && v - h < (float)cam.H + 1.f)) return;
    const int x0 = max(0, (int)ceilf(u - h - 0.5f)), x1 = min(cam.W, (int)ceilf(u + h - 0.5f));
    const int y0 = max(0, (int)ceilf(v - h - 0.5f)), y1 = min(cam.H, (int)ceilf(v + h - 0.5f));
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            const int64_t p = (int64_t)y * cam.W + x;
            if (depth) {
                const float d = depth[p];
                if (d != 0.f && !(z <= __builtin_fmaf(d, eps, d))) continue;
            }
            mask[p] = 1;
        }
}

// c* = t c on the pixels the mask marks (HWC, one thread per value); in place allowed.
__global__ __launch_bounds__(256) void k_tint(const float *image, const uint8_t *__restrict__ mask, float t0, float t1,
                                              float t2, float *out, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const int64_t p = e / 3;
    const int c = (int)(e - 3 * p);
    const float t = c == 0 ? t0 : (c == 1 ? t1 : t2);
    const float v = image[e];
    out[e] = mask[p] ? v * t : v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
uint32_t unproject_blocks(int64_t pixels) { return (uint32_t)((pixels + kUnpBlock - 1) / kUnpBlock); }

void launch_unproject(const CamDev &cam, const uint8_t *mask, const uint8_t *keep, const float *depth, int64_t P,
                      uint32_t *part, uint32_t *count, float *pts, int64_t cap, hipStream_t st) {
    const uint32_t nblk = unproject_blocks(P);
    if (nblk) hipLaunchKernelGGL(k_unp_count, dim3(nblk), dim3(256), 0, st, mask, keep, depth, P, part);
    hipLaunchKernelGGL(k_unp_scan, dim3(1), dim3(1024), 0, st, part, nblk, count);
    if (nblk)
        hipLaunchKernelGGL(k_unp_write, dim3(nblk), dim3(256), 0, st, mask, keep, depth, P, (int)cam.W, part, cam, pts, cap);
}

// ---------------------------------------------------------------------------
// Unprojection without caller or library allocations: the per-workgroup counts live in
// a fixed device array (one per GPU, for the life of the process) instead of a workspace.
// ---------------------------------------------------------------------------
constexpr int64_t kUnpScratchMaxPixels = (int64_t)1 << 26;   // 67,108,864 pixels, e.g. 8192 x 8192
constexpr uint32_t kUnpScratchWords = (uint32_t)(kUnpScratchMaxPixels / kUnpBlock);   // 65,536 counts, 256 KB
static __device__ __align__(256) uint32_t scratch[kUnpScratchWords];

int64_t unproject_scratch_max_pixels() { return kUnpScratchMaxPixels; }

// Device address of `scratch` on the current device, looked up once per device (the
// host-side name of the array is not a device address). nullptr (with *err set) on failure.
uint32_t *unproject_scratch_ptr(hipError_t *err) {
    constexpr int kMaxDevices = 64;
    static std::atomic<uint32_t *> ptrs[kMaxDevices];
    static std::mutex lock;
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    uint32_t *p = ptrs[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> g(lock);
    p = ptrs[dev].load(std::memory_order_relaxed);
    if (!p) {
        void *a = nullptr;
        *err = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (*err != hipSuccess || !a) {
            if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
            return nullptr;
        }
        p = (uint32_t *)a;
        ptrs[dev].store(p, std::memory_order_release);
    }
    return p;
}

// exclusive scan of nblk counts in place, total to *count (the compaction step shared
// with the outlier filter)
void launch_excl_scan_u32(uint32_t *part, uint32_t nblk, uint32_t *count, hipStream_t st) {
    hipLaunchKernelGGL(k_unp_scan, dim3(1), dim3(1024), 0, st, part, nblk, count);
}

void launch_reproject(const CamDev &cam, const float *pts, int64_t n, int64_t stride, float quad_px, const float *depth,
                      float eps, uint8_t *mask, hipStream_t st) {
    const int64_t P = (int64_t)cam.W * cam.H;
    int64_t zb = (P + 255) / 256;
    if (zb > 4096) zb = 4096;
    hipLaunchKernelGGL(k_zero_u8, dim3((unsigned)zb), dim3(256), 0, st, mask, P);
    if (n > 0)
        hipLaunchKernelGGL(k_reproject, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pts, n, stride, cam,
                           0.5f * quad_px, depth, eps, mask);
}

void launch_tint(const float *image, const uint8_t *mask, const float *t, float *out, int64_t pixels, hipStream_t st) {
    const int64_t count = 3 * pixels;
    if (count <= 0) return;
    hipLaunchKernelGGL(k_tint, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, image, mask, t[0], t[1], t[2], out,
                       count);
}

}  // namespace recogs
