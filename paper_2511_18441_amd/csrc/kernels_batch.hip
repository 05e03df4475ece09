// Batched render: many (scene, view) renders in one launch sequence with no host
// synchronisation (capturable in a HIP graph).
//
// Every stage runs once over the whole batch. The (view, Gaussian) pairs of all views
// form one index space (view v owns pairs [pair_base_v, pair_base_v + n_v)) and the
// tiles of all views one global tile-id space (view v owns [tile_base_v, +ntiles_v)).
// Preprocess writes per-pair records; the count scan, the depth sort, the emission
// (global tile ids) and the tile-id sort are the single-view kernels run over pairs;
// the blend is persistent: workgroups take global tiles (or, in region form, one-wave
// workgroups take (tile, region) items from per-XCD queues) from atomic queues in
// largest-list-first order, so uneven views share the GPU without a tail of idle CUs.
#include "render_device.hpp"

namespace recogs {

// last view v with key(v) <= x (key = preprocess block base or tile base); uniform
__device__ __forceinline__ int view_of_block(const ViewDev *views, int nviews, uint32_t x) {
    int lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].blk_base <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int view_of_tile(const ViewDev *views, int nviews, uint32_t x) {
    int lo = 0, hi = nviews - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int DT, int DEG>
__global__ __launch_bounds__(256) void k_preprocess_batch(const ViewDev *__restrict__ views, int nviews,
                                                          SplatRec *__restrict__ rec, uint32_t *__restrict__ zbits,
                                                          uint2 *__restrict__ rect, uint32_t *__restrict__ count) {
    const int v = view_of_block(views, nviews, blockIdx.x);
    const ViewDev &vw = views[v];
    const int64_t i = (int64_t)(blockIdx.x - vw.blk_base) * 256 + threadIdx.x;
    if (i < vw.sc.n)
        preprocess_one<DT, DEG>(vw.sc, vw.cam, vw.rc, 0, i, (int64_t)vw.pair_base + i, rec, nullptr, zbits, rect, count);
}

// Largest-first order of the global tiles: length classes c = bit length of the list
// length (0 for empty), counted, turned into descending-class cursors, then scattered
// with wave-aggregated atomics (lanes of one class take one atomic).
__device__ __forceinline__ uint32_t len_class(uint2 rg) {
    const uint32_t len = rg.y - rg.x;
    return len ? min(31u, 32u - (uint32_t)__builtin_clz(len)) : 0u;
}

__global__ __launch_bounds__(256) void k_tile_order_hist(const uint2 *__restrict__ ranges, uint32_t ntiles,
                                                         uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[32];
    if (threadIdx.x < 32) h[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < ntiles; t += gridDim.x * 256) atomicAdd(&h[len_class(ranges[t])], 1u);
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(64) void k_tile_order_scan(const uint32_t *__restrict__ hist, uint32_t *__restrict__ cur) {
    const uint32_t c = threadIdx.x;
    uint32_t s = 0;
    for (uint32_t k = c + 1; k < 32; ++k) s += hist[k];
    if (c < 32) cur[c] = s;
}

__global__ __launch_bounds__(256) void k_tile_order_scatter(const uint2 *__restrict__ ranges, uint32_t ntiles,
                                                            uint32_t *__restrict__ cur, uint32_t *__restrict__ order) {
    const uint32_t w0 = (blockIdx.x * 256 + threadIdx.x) & ~63u;
    for (uint32_t base = w0; base < ntiles; base += gridDim.x * 256) {
        const uint32_t t = base + lane_id();
        const bool valid = t < ntiles;
        const uint32_t c = valid ? len_class(ranges[t]) : 0u;
        uint64_t m = wave_ballot(valid);
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const bool bit = (c >> b) & 1u;
            const uint64_t bb = wave_ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t r = rank_below(m);
        const uint32_t leader = (uint32_t)__builtin_ctzll(m | (1ull << 63));
        uint32_t pos = 0;
        if (valid && r == 0) pos = atomicAdd(&cur[c], (uint32_t)__popcll(m));
        pos = __shfl(pos, (int)leader, 64);
        if (valid) order[pos + r] = t;
    }
}

// Persistent blend: each workgroup loops taking the next global tile from the queue
// until the queue is exhausted (every workgroup reaches that exit).
template <int TW, int TH, int PPT>
__global__ __launch_bounds__(TW *TH / PPT) void k_blend_persistent(const ViewDev *__restrict__ views, int nviews,
                                                                  const uint2 *__restrict__ ranges,
                                                                  const uint32_t *__restrict__ vals,
                                                                  const SplatRec *__restrict__ rec,
                                                                  const uint32_t *__restrict__ order, uint32_t ntiles,
                                                                  uint32_t *__restrict__ queue) {
    __shared__ BlendStage sm;
    __shared__ uint32_t s_item;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= ntiles) break;
        const uint32_t gt = order[item];
        const int v = view_of_tile(views, nviews, gt);
        const ViewDev &vw = views[v];
        blend_tile<TW, TH, PPT, false>((int)(gt - vw.tile_base), ranges[gt], vals, rec, vw.cam.W, vw.cam.H, vw.cam.tiles_x,
                                vw.bg[0], vw.bg[1], vw.bg[2], vw.image, 0, nullptr, nullptr, sm);
    }
}

// Persistent region form: `grid` one-wave workgroups take (tile, region) items from
// per-XCD queues until theirs is exhausted (every wave reaches that exit). Tile j of
// the longest-first order belongs to queue j mod 8 and its regions are consecutive
// items of that queue, so its list is read through one L2; workgroup b takes items
// from queue b mod 8, the XCD it runs on when workgroups are dealt to the XCDs in turn
// (any other placement only costs locality).
template <int TW, int TH, int PPT>
__global__ __launch_bounds__(64) void k_blend_region_persistent(const ViewDev *__restrict__ views, int nviews,
                                                               const uint2 *__restrict__ ranges,
                                                               const uint32_t *__restrict__ vals,
                                                               const SplatRec *__restrict__ rec,
                                                               const uint32_t *__restrict__ order, uint32_t ntiles,
                                                               uint32_t *__restrict__ xqueue) {
    constexpr uint32_t NR = (TW / 8) * (TH / (8 * PPT));
    __shared__ BlendRec sm[64];
    const uint32_t x = blockIdx.x & 7u;
    const uint32_t nitems = (ntiles > x ? (ntiles - x + 7u) / 8u : 0u) * NR;
    uint32_t *q = xqueue + 32u * x;
    while (true) {
        uint32_t m = 0;
        if (lane_id() == 0) m = atomicAdd(q, 1u);
        m = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);
        if (m >= nitems) break;
        const uint32_t gt = order[(m / NR) * 8u + x];
        const int v = view_of_tile(views, nviews, gt);
        const ViewDev &vw = views[v];
        blend_region<TW, TH, PPT, false>((int)(gt - vw.tile_base), (int)(m % NR), ranges[gt], vals, rec, vw.cam.W,
                                         vw.cam.H, vw.cam.tiles_x, vw.bg[0], vw.bg[1], vw.bg[2], vw.image, 0,
                                         nullptr, nullptr, sm);
    }
}

// ---------------------------------------------------------------------------
template <int DT>
static void preprocess_batch_dt(int deg, uint32_t blocks, hipStream_t st, const ViewDev *views, int nviews, SplatRec *rec,
                                uint32_t *zb, uint2 *rect, uint32_t *cnt) {
    const dim3 g(blocks), b(256);
    switch (deg) {
    case 0: hipLaunchKernelGGL((k_preprocess_batch<DT, 0>), g, b, 0, st, views, nviews, rec, zb, rect, cnt); break;
    case 1: hipLaunchKernelGGL((k_preprocess_batch<DT, 1>), g, b, 0, st, views, nviews, rec, zb, rect, cnt); break;
    case 2: hipLaunchKernelGGL((k_preprocess_batch<DT, 2>), g, b, 0, st, views, nviews, rec, zb, rect, cnt); break;
    default: hipLaunchKernelGGL((k_preprocess_batch<DT, 3>), g, b, 0, st, views, nviews, rec, zb, rect, cnt); break;
    }
}

void launch_preprocess_batch(int dt, int deg, uint32_t blocks, const ViewDev *views, int nviews, SplatRec *rec, uint32_t *zb,
                             uint2 *rect, uint32_t *cnt, hipStream_t st) {
    if (blocks == 0) return;
    if (dt == RECOGS_F32) preprocess_batch_dt<RECOGS_F32>(deg, blocks, st, views, nviews, rec, zb, rect, cnt);
    else if (dt == RECOGS_F16) preprocess_batch_dt<RECOGS_F16>(deg, blocks, st, views, nviews, rec, zb, rect, cnt);
    else preprocess_batch_dt<RECOGS_BF16>(deg, blocks, st, views, nviews, rec, zb, rect, cnt);
}

void launch_tile_order(const uint2 *ranges, uint32_t ntiles, uint32_t *hist, uint32_t *cur, uint32_t *order, hipStream_t st) {
    if (ntiles == 0) return;
    uint32_t blocks = (ntiles + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_tile_order_hist, dim3(blocks), dim3(256), 0, st, ranges, ntiles, hist);
    hipLaunchKernelGGL(k_tile_order_scan, dim3(1), dim3(64), 0, st, hist, cur);
    hipLaunchKernelGGL(k_tile_order_scatter, dim3(blocks), dim3(256), 0, st, ranges, ntiles, cur, order);
}

template <int TW, int TH, int PPT>
static void persistent_one(uint32_t grid, hipStream_t st, const ViewDev *views, int nviews, const uint2 *ranges,
                           const uint32_t *vals, const SplatRec *rec, const uint32_t *order, uint32_t ntiles,
                           uint32_t *queue) {
    if constexpr (region_shape(TW, TH, PPT)) {
        // 32 one-wave workgroups per CU (grid = CUs x 8); `queue` is the header's H_QUEUE word
        hipLaunchKernelGGL((k_blend_region_persistent<TW, TH, PPT>), dim3(grid * 4), dim3(64), 0, st, views, nviews, ranges,
                           vals, rec, order, ntiles, queue + (H_XQUEUE - H_QUEUE));
    } else {
        hipLaunchKernelGGL((k_blend_persistent<TW, TH, PPT>), dim3(grid), dim3(TW * TH / PPT), 0, st, views, nviews, ranges,
                           vals, rec, order, ntiles, queue);
    }
}

bool launch_blend_persistent(int tw, int th, int ppt, uint32_t grid, const ViewDev *views, int nviews, const uint2 *ranges,
                             const uint32_t *vals, const SplatRec *rec, const uint32_t *order, uint32_t ntiles,
                             uint32_t *queue, hipStream_t st) {
#define RECOGS_PERS_CASE(A, B, P)                                                                     \
    if (tw == A && th == B && ppt == P) {                                                             \
        persistent_one<A, B, P>(grid, st, views, nviews, ranges, vals, rec, order, ntiles, queue);    \
        return true;                                                                                  \
    }
    RECOGS_PERS_CASE(16, 16, 1) RECOGS_PERS_CASE(16, 16, 2) RECOGS_PERS_CASE(16, 16, 4)
    RECOGS_PERS_CASE(8, 8, 1) RECOGS_PERS_CASE(8, 8, 2) RECOGS_PERS_CASE(8, 8, 4)
    RECOGS_PERS_CASE(32, 8, 1) RECOGS_PERS_CASE(32, 8, 2) RECOGS_PERS_CASE(32, 8, 4)
    RECOGS_PERS_CASE(32, 16, 1) RECOGS_PERS_CASE(32, 16, 2) RECOGS_PERS_CASE(32, 16, 4)
    RECOGS_PERS_CASE(32, 32, 1) RECOGS_PERS_CASE(32, 32, 2) RECOGS_PERS_CASE(32, 32, 4)
#undef RECOGS_PERS_CASE
    return false;
}

}  // namespace recogs
