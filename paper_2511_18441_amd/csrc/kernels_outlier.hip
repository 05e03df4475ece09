// Statistical outlier removal of a point cloud (Sec. 3.2, Fig. 2 caption: mean distance
// to 16 neighbours, standard-deviation scale 0.007):
//   D_i = mean distance from point i to its k nearest other points (all others when
//         there are fewer), mu / sigma = mean and population standard deviation of D,
//   keep i  iff  D_i <= mu + std_ratio sigma.
//
// Exact k-nearest neighbours through a hashed uniform grid:
//   1. bounding box (reduction), then per-axis 1024-bin histograms over it; the cell
//      size h is the largest 1%-99% quantile extent divided by ceil(2 n^(1/3)) (at most
//      128), so far-away stray points do not coarsen the grid for the rest;
//   2. each point's cell (floor((x - min) / h) per axis) goes to the slot made of its
//      coordinates modulo powers of two (2^b slots, b = log2 of about 2n, at least 4 bits
//      per axis); a radix sort by slot and a range pass give each slot its run of points
//      (slot order is also the query order: queries of one wave start in nearby cells);
//   3. per query, the cells of Chebyshev rings r = 0, 1, ... are scanned (no two cells of
//      one search share a slot; points of far cells that do are scanned too), keeping the k
//      smallest squared distances in registers (sorted insertion): rings 0-1 one thread
//      per query, further rings one wave per query (the lanes split a ring's cells, so a
//      few sparse neighbourhoods do not hold whole waves back); after ring r >= 1 the
//      search stops once the k-th distance is within (r - 1/16) h, the distance below
//      which no unscanned cell lies (the 1/16 absorbs float32 rounding of the cell
//      coordinates). A query whose rings reach kOlMaxRing without that bound (a far
//      stray point) is deferred to a second kernel that scans the whole cloud with one
//      workgroup per query (strided per-thread lists merged in LDS).
//   4. mu and sigma from compensated float32 sums (float-float, TwoSum) in a fixed order:
//      a pass for the sum of D, a pass for the sum of (D - mu)^2; the threshold, the keep
//      mask (float32 comparison) and the compaction of the kept points (input order)
//      follow. No double precision on the GPU.
#include "recogs_internal.hpp"

namespace recogs {

int radix_sort_u32(uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t, uint32_t, int, uint32_t *, uint32_t *,
                   hipStream_t, const EmitFold * = nullptr, bool = false);
void launch_ranges32(const uint32_t *, uint32_t, uint2 *, hipStream_t, const uint32_t *);
void launch_fill_u32(uint32_t *, uint32_t, int64_t, hipStream_t);
void launch_excl_scan_u32(uint32_t *, uint32_t, uint32_t *, hipStream_t);

constexpr int kOlBins = 1024;
constexpr int kOlMaxDim = 128;
constexpr int kOlThreadRing = 2;               // rings searched by the one-thread-per-query pass
constexpr int kOlMaxRing = 6;                  // rings searched by the wave-per-query pass
constexpr int kOlWaveBlocks = 2048;            // grid of the wave-per-query pass (4 waves each)
static_assert(2 * (kOlMaxRing - 1) + 1 <= 16, "one search's cells must fit in 16 slot residues per axis");
constexpr int kOlFarBlocks = 1024;             // grid of the whole-cloud scans (grid-stride over the queries)
constexpr int kOlFarThreads = 512;             // threads per whole-cloud scan (LDS: 512 k floats, 64 KB at k = 32)
constexpr int kOlRedBlocks = 512;              // grid of the reductions (grid-stride)
constexpr int kOlItems = 4;                    // points per thread of the keep/compaction passes
constexpr int kOlBlock = 256 * kOlItems;
constexpr float kOlClamp = 1048576.f;          // cell coordinates are clamped to +-2^20
// Ring-search guard: a float32 cell coordinate f = (v - min) / h is within 3 2^-24 |f|
// of its exact value, so for |f| <= 2^16 two coordinates are within 0.024 cells of the
// exact difference; the stop bound keeps kOlMargin = 1/16 cell of slack for it. Queries
// beyond 2^16 cells from the box corner scan the whole cloud.
constexpr float kOlQueryLimit = 65536.f;
constexpr float kOlMargin = 1.f / 16.f;

// Workspace header (device, written by the setup kernels).
struct OlHdr {
    float mn[3], mx[3];   // bounding box
    float h, inv_h;       // cell size and its reciprocal
    uint32_t bx, by, bz;  // slot bits per axis
    uint32_t ndefer;      // queries left to the whole-cloud scan
    uint32_t nslow;       // queries left to the wave-per-query search
    float thr;            // mu + std_ratio sigma
    float mu, sigma;
};

__device__ __forceinline__ void ol_load(const float *__restrict__ pts, int64_t stride, int64_t i, float &x, float &y,
                                        float &z) {
    x = pts[i];
    y = pts[stride + i];
    z = pts[2 * stride + i];
}

__device__ __forceinline__ int ol_coord(float v, float mn, float inv_h) {
    const float f = fminf(fmaxf(floorf((v - mn) * inv_h), -kOlClamp), kOlClamp);
    return (int)f;
}

// Slot of a cell: its coordinates modulo 2^bx, 2^by, 2^bz, packed (bx + by + bz = the
// slot bits, each at least 4). Cells that differ by less than 16 along every axis get
// different slots, so the cells of one search (at most 11 x 11 x 11) never share a slot
// and a slot's run can be scanned without checking each point's cell: the points of
// far cells that share it are real points of the cloud, and only add candidates.
__device__ __forceinline__ uint32_t ol_slot(int cx, int cy, int cz, uint32_t bx, uint32_t by, uint32_t bz) {
    return ((uint32_t)cx & ((1u << bx) - 1u)) | (((uint32_t)cy & ((1u << by) - 1u)) << bx) |
           (((uint32_t)cz & ((1u << bz) - 1u)) << (bx + by));
}

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// 1a. per-workgroup bounding boxes -> part[blk][6]
__global__ __launch_bounds__(256) void k_ol_bbox(const float *__restrict__ pts, int64_t n, int64_t stride,
                                                 float *__restrict__ part) {
    __shared__ float s[4][6];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float p[3];
        ol_load(pts, stride, i, p[0], p[1], p[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], p[a]);
            hi[a] = fmaxf(hi[a], p[a]);
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (lane_id() == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s[w][a] = lo[a];
            s[w][3 + a] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = s[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) v = threadIdx.x < 3 ? fminf(v, s[k][threadIdx.x]) : fmaxf(v, s[k][threadIdx.x]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

// 1b. final box: wave w (of 6) reduces bound w over the partials
__global__ __launch_bounds__(384) void k_ol_bbox_final(const float *__restrict__ part, int nblk, OlHdr *__restrict__ hdr) {
    const int a = threadIdx.x >> 6, l = (int)lane_id();
    const bool lo = a < 3;
    float v = lo ? INFINITY : -INFINITY;
    for (int b = l; b < nblk; b += 64) v = lo ? fminf(v, part[b * 6 + a]) : fmaxf(v, part[b * 6 + a]);
    v = lo ? wave_min(v) : wave_max(v);
    if (l == 0) {
        if (lo) hdr->mn[a] = v;
        else hdr->mx[a - 3] = v;
        if (a == 0) {
            hdr->ndefer = 0;
            hdr->nslow = 0;
        }
    }
}

// 1c. per-axis histograms over the box (LDS counts, then one atomic per bin and
// workgroup; integer counts, so the result is independent of the order)
__global__ __launch_bounds__(256) void k_ol_hist(const float *__restrict__ pts, int64_t n, int64_t stride,
                                                 const OlHdr *__restrict__ hdr, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[3 * kOlBins];
    for (int k = threadIdx.x; k < 3 * kOlBins; k += 256) s_h[k] = 0;
    __syncthreads();
    float mn[3], sc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn[a] = hdr->mn[a];
        const float e = hdr->mx[a] - mn[a];
        sc[a] = e > 0.f ? (float)kOlBins / e : 0.f;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float p[3];
        ol_load(pts, stride, i, p[0], p[1], p[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int b = (int)((p[a] - mn[a]) * sc[a]);
            b = b < 0 ? 0 : (b >= kOlBins ? kOlBins - 1 : b);
            atomicAdd(&s_h[a * kOlBins + b], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 3 * kOlBins; k += 256)
        if (s_h[k]) atomicAdd(&hist[k], s_h[k]);
}

// 1d. cell size from the 1%-99% quantile extents: wave a scans axis a's 1024 bins (16
// per lane, then a wave scan) and finds the first bins whose cumulative count passes 1%
// and 99% of the points; then thread 0 sets h.
__global__ __launch_bounds__(192) void k_ol_setup(const uint32_t *__restrict__ hist, int64_t n, uint32_t slot_bits,
                                                  OlHdr *__restrict__ hdr) {
    __shared__ float s_ext[3];
    constexpr int PER = kOlBins / 64;
    const int a = threadIdx.x >> 6, l = (int)lane_id();
    const uint64_t lo_need = (uint64_t)n / 100u, hi_need = (uint64_t)n * 99u / 100u;
    uint32_t c[PER];
    uint32_t mine = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        c[q] = hist[a * kOlBins + l * PER + q];
        mine += c[q];
    }
    const uint32_t incl = wave_incl_scan(mine);
    // first bin (in lane-major order) where the running count exceeds `need`
    auto first_over = [&](uint64_t need) -> int {
        int bin = kOlBins;
        uint64_t cum = incl - mine;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            cum += c[q];
            if (bin == kOlBins && cum > need) bin = l * PER + q;
        }
        int best = bin;
        for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o));
        return best;
    };
    int blo = first_over(lo_need);
    int bhi = first_over(hi_need < (uint64_t)n ? hi_need : (uint64_t)n - 1);
    blo = blo >= kOlBins ? 0 : blo;
    bhi = bhi >= kOlBins ? kOlBins - 1 : bhi;
    if (l == 0) {
        const float e = hdr->mx[a] - hdr->mn[a];
        s_ext[a] = (float)(bhi - blo + 1) * (e / (float)kOlBins);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float L = fmaxf(s_ext[0], fmaxf(s_ext[1], s_ext[2]));
        // D = ceil(2 n^(1/3)), the least D with D^3 >= 8 n, capped at kOlMaxDim
        int D = 1;
        while (D < kOlMaxDim && (uint64_t)D * D * D < 8u * (uint64_t)n) ++D;
        float h = L / (float)D;
        if (!(h > 0.f) || !isfinite(h)) h = 1.f;   // all points coincide (or a degenerate box)
        hdr->h = h;
        hdr->inv_h = 1.f / h;
        hdr->bz = slot_bits / 3;
        hdr->by = (slot_bits - slot_bits / 3) / 2;
        hdr->bx = slot_bits - hdr->bz - hdr->by;
    }
}

// 2. slot keys
__global__ __launch_bounds__(256) void k_ol_key(const float *__restrict__ pts, int64_t n, int64_t stride,
                                                const OlHdr *__restrict__ hdr, uint32_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float x, y, z;
    ol_load(pts, stride, i, x, y, z);
    const float ih = hdr->inv_h;
    keys[i] = ol_slot(ol_coord(x, hdr->mn[0], ih), ol_coord(y, hdr->mn[1], ih), ol_coord(z, hdr->mn[2], ih), hdr->bx,
                      hdr->by, hdr->bz);
    vals[i] = (uint32_t)i;
}

// 2b. the points in slot order as float4 (x, y, z, input index bits): one 16-byte load
// per candidate in the searches below
__global__ __launch_bounds__(256) void k_ol_gather(const float *__restrict__ pts, int64_t n, int64_t stride,
                                                   const uint32_t *__restrict__ svals, float4 *__restrict__ spts) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = svals[j];
    float x, y, z;
    ol_load(pts, stride, i, x, y, z);
    spts[j] = make_float4(x, y, z, __uint_as_float(i));
}

template <int K>
__device__ __forceinline__ void ol_insert(float (&best)[K], float d2) {
    if (!(d2 < best[K - 1])) return;
#pragma unroll
    for (int q = K - 1; q > 0; --q) best[q] = d2 < best[q - 1] ? best[q - 1] : (d2 < best[q] ? d2 : best[q]);
    best[0] = d2 < best[0] ? d2 : best[0];
}

// One slot's candidates [rg.x, rg.y) of the slot-ordered points against query i at
// (x, y, z); four loads in flight.
template <int K>
__device__ __forceinline__ void ol_scan_cell(const float4 *__restrict__ spts, uint2 rg, uint32_t i, float x, float y,
                                             float z, float (&best)[K]) {
    for (uint32_t j = rg.x; j < rg.y; j += 4) {
        float4 c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = j + u < rg.y ? spts[j + u] : make_float4(0.f, 0.f, 0.f, __uint_as_float(i));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (__float_as_uint(c[u].w) == i) continue;   // the query itself, or past the range
            const float ex = c[u].x - x, ey = c[u].y - y, ez = c[u].z - z;
            ol_insert<K>(best, __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)));
        }
    }
}

// 3. k nearest neighbours of every point (one thread per point, slot order), rings 0
// and 1 only: a query not settled by then goes to the wave-per-query search (slow list,
// slot positions), a query beyond the coordinate guard to the whole-cloud scan.
template <int K>
__global__ __launch_bounds__(256) void k_ol_knn(const float4 *__restrict__ spts, int64_t n, OlHdr *hdr,
                                                const uint2 *__restrict__ ranges, uint32_t *__restrict__ slow,
                                                uint32_t *__restrict__ defer, float *__restrict__ dmean) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const float4 me = spts[s];
    const uint32_t i = __float_as_uint(me.w);
    const float x = me.x, y = me.y, z = me.z;
    const float mnx = hdr->mn[0], mny = hdr->mn[1], mnz = hdr->mn[2], ih = hdr->inv_h, h = hdr->h;
    const uint32_t bx = hdr->bx, by = hdr->by, bz = hdr->bz;
    const int cx = ol_coord(x, mnx, ih), cy = ol_coord(y, mny, ih), cz = ol_coord(z, mnz, ih);
    const int want = n - 1 < (int64_t)K ? (int)(n - 1) : K;
    float best[K];
#pragma unroll
    for (int q = 0; q < K; ++q) best[q] = INFINITY;
    bool done = want == 0;
    const bool clamped = fabsf((x - mnx) * ih) > kOlQueryLimit || fabsf((y - mny) * ih) > kOlQueryLimit ||
                         fabsf((z - mnz) * ih) > kOlQueryLimit;
    static_assert(kOlThreadRing == 2, "the one-thread pass covers the 3 x 3 x 3 cells of rings 0 and 1");
    if (!done && !clamped) {
        // the 27 slot ranges first (independent loads), then the cells' candidates
        uint2 rg[27];
#pragma unroll
        for (int t = 0; t < 27; ++t)
            rg[t] = ranges[ol_slot(cx + t % 3 - 1, cy + (t / 3) % 3 - 1, cz + t / 9 - 1, bx, by, bz)];
#pragma unroll 1
        for (int t = 0; t < 27; ++t) ol_scan_cell<K>(spts, rg[t], i, x, y, z, best);
        float kth = best[0];
#pragma unroll
        for (int q = 1; q < K; ++q) kth = q == want - 1 ? best[q] : kth;
        const float bound = (1.f - kOlMargin) * h;
        done = kth <= bound * bound;
    }
    if (!done) {
        if (clamped) defer[atomicAdd(&hdr->ndefer, 1u)] = i;
        else slow[atomicAdd(&hdr->nslow, 1u)] = (uint32_t)s;
        return;
    }
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < K; ++q) sum += q < want ? sqrtf(best[q]) : 0.f;
    dmean[i] = want > 0 ? sum / (float)want : 0.f;
}

// 3b. the slow queries, one wave each (grid-stride over the list): the lanes split
// each ring's cells (cube index t -> offsets, ring cells only) and keep their own k
// smallest squared distances. The stop test after ring r counts, over the lanes, the
// entries of their lists within the bound: the k-th smallest of the union is within it
// iff at least k are (each of the k smallest overall is in its lane's k smallest). The
// 64 lists are then merged pairwise in LDS (6 rounds, wave-level ordering only).
// Queries not settled by ring kOlMaxRing - 1 go to the whole-cloud scan.
template <int K>
__global__ __launch_bounds__(256) void k_ol_knn_wave(const float4 *__restrict__ spts, int64_t n, OlHdr *hdr,
                                                     const uint2 *__restrict__ ranges, const uint32_t *__restrict__ slow,
                                                     uint32_t *__restrict__ defer, float *__restrict__ dmean) {
    __shared__ float s_l[4][64 * K];
    const int wv = (int)(threadIdx.x >> 6), l = (int)lane_id();
    float *Ls = s_l[wv];
    const uint32_t ns = hdr->nslow;
    const uint32_t waves = gridDim.x * 4u;
    const float mnx = hdr->mn[0], mny = hdr->mn[1], mnz = hdr->mn[2], ih = hdr->inv_h, h = hdr->h;
    const uint32_t bx = hdr->bx, by = hdr->by, bz = hdr->bz;
    const int want = n - 1 < (int64_t)K ? (int)(n - 1) : K;
    for (uint32_t q = blockIdx.x * 4u + (uint32_t)wv; q < ns; q += waves) {
        const float4 me = spts[slow[q]];
        const uint32_t i = __float_as_uint(me.w);
        const float x = me.x, y = me.y, z = me.z;
        const int cx = ol_coord(x, mnx, ih), cy = ol_coord(y, mny, ih), cz = ol_coord(z, mnz, ih);
        float best[K];
#pragma unroll
        for (int a = 0; a < K; ++a) best[a] = INFINITY;
        bool done = false;
        for (int r = 0; r < kOlMaxRing && !done; ++r) {
            const int side = 2 * r + 1, cube = side * side * side;
            for (int t = l; t < cube; t += 64) {
                const int dx = t % side - r, dy = (t / side) % side - r, dz = t / (side * side) - r;
                if (max(abs(dx), max(abs(dy), abs(dz))) != r) continue;   // inner cells: earlier rings
                const int qx = cx + dx, qy = cy + dy, qz = cz + dz;
                ol_scan_cell<K>(spts, ranges[ol_slot(qx, qy, qz, bx, by, bz)], i, x, y, z, best);
            }
            if (r >= 1) {
                const float bound = ((float)r - kOlMargin) * h, b2 = bound * bound;
                int c = 0;
#pragma unroll
                for (int a = 0; a < K; ++a) c += best[a] <= b2 ? 1 : 0;
                for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
                done = c >= want;
            }
        }
        if (!done) {
            if (l == 0) defer[atomicAdd(&hdr->ndefer, 1u)] = i;
            continue;
        }
#pragma unroll
        for (int a = 0; a < K; ++a) Ls[l * K + a] = best[a];
        wave_sync();
        for (int sp = 1; sp < 64; sp <<= 1) {
            if ((l & (2 * sp - 1)) == 0) {
                const float *A = Ls + l * K, *B = Ls + (l + sp) * K;
                float m[K];
                int ia = 0, ib = 0;
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const float va = A[ia], vb = B[ib];
                    const bool ta = va <= vb;
                    m[a] = ta ? va : vb;
                    ia += ta ? 1 : 0;
                    ib += ta ? 0 : 1;
                }
#pragma unroll
                for (int a = 0; a < K; ++a) Ls[l * K + a] = m[a];
            }
            wave_sync();
        }
        if (l == 0) {
            float sum = 0.f;
            for (int a = 0; a < want; ++a) sum += sqrtf(Ls[a]);
            dmean[i] = want > 0 ? sum / (float)want : 0.f;
        }
        wave_sync();   // the lists are rewritten by the next query
    }
}

// 3c. the deferred queries, one workgroup each (grid-stride over the list): every
// thread keeps the k smallest squared distances of a strided share of the cloud, then
// the kOlFarThreads sorted lists are merged pairwise in LDS (9 rounds).
template <int K>
__global__ __launch_bounds__(kOlFarThreads) void k_ol_knn_far(const float4 *__restrict__ spts, const float *__restrict__ pts,
                                                    int64_t n, int64_t stride, const OlHdr *__restrict__ hdr,
                                                    const uint32_t *__restrict__ defer, float *__restrict__ dmean) {
    __shared__ float s_l[kOlFarThreads * K];
    __shared__ float s_t[K];
    const uint32_t nd = hdr->ndefer;
    const int want = n - 1 < (int64_t)K ? (int)(n - 1) : K;
    for (uint32_t q = blockIdx.x; q < nd; q += gridDim.x) {
        const uint32_t i = defer[q];
        float x, y, z;
        ol_load(pts, stride, i, x, y, z);
        float best[K];
#pragma unroll
        for (int a = 0; a < K; ++a) best[a] = INFINITY;
        // four loads in flight per iteration (the scan is latency bound otherwise)
        int64_t j = threadIdx.x;
        for (; j + 3 * kOlFarThreads < n; j += 4 * kOlFarThreads) {
            float4 c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = spts[j + u * kOlFarThreads];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (__float_as_uint(c[u].w) == i) continue;
                const float ex = c[u].x - x, ey = c[u].y - y, ez = c[u].z - z;
                ol_insert<K>(best, __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)));
            }
        }
        for (; j < n; j += kOlFarThreads) {
            const float4 c = spts[j];
            if (__float_as_uint(c.w) == i) continue;
            const float ex = c.x - x, ey = c.y - y, ez = c.z - z;
            ol_insert<K>(best, __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)));
        }
#pragma unroll
        for (int a = 0; a < K; ++a) s_l[threadIdx.x * K + a] = best[a];
        __syncthreads();
        for (int sp = 1; sp < kOlFarThreads; sp <<= 1) {
            if ((threadIdx.x & (2 * sp - 1)) == 0) {
                const float *A = s_l + threadIdx.x * K, *B = s_l + (threadIdx.x + sp) * K;
                float m[K];
                int ia = 0, ib = 0;
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    const float va = A[ia], vb = B[ib];
                    const bool ta = va <= vb;
                    m[a] = ta ? va : vb;
                    ia += ta ? 1 : 0;
                    ib += ta ? 0 : 1;
                }
#pragma unroll
                for (int a = 0; a < K; ++a) s_l[threadIdx.x * K + a] = m[a];
            }
            __syncthreads();
        }
        if (threadIdx.x < K) s_t[threadIdx.x] = s_l[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 0) {
            float sum = 0.f;
            for (int a = 0; a < want; ++a) sum += sqrtf(s_t[a]);
            dmean[i] = want > 0 ? sum / (float)want : 0.f;
        }
        __syncthreads();   // s_l and s_t are reused by the next query
    }
}

// Compensated float32 sums: a value held as hi + lo, each addition through Knuth's
// TwoSum (the rounding error of hi + b is exact and goes to lo).
struct FF { float hi, lo; };
__device__ __forceinline__ FF ff_add(FF a, float b) {
    const float s = a.hi + b, bb = s - a.hi;
    return FF{s, a.lo + ((a.hi - (s - bb)) + (b - bb))};
}
__device__ __forceinline__ FF ff_merge(FF a, FF b) {
    const float s = a.hi + b.hi, bb = s - a.hi;
    return FF{s, (a.lo + b.lo) + ((a.hi - (s - bb)) + (b.hi - bb))};
}
__device__ __forceinline__ FF ff_wave(FF a) {   // butterfly over the wave, the same order every run
    for (int o = 32; o > 0; o >>= 1) a = ff_merge(a, FF{__shfl_xor(a.hi, o), __shfl_xor(a.lo, o)});
    return a;
}
// the workgroup's 256-thread sum (every wave reaches it), fixed order; valid in thread 0
__device__ __forceinline__ FF ff_block(FF a, FF (*s)[1]) {
    a = ff_wave(a);
    if (lane_id() == 0) s[threadIdx.x >> 6][0] = a;
    __syncthreads();
    return ff_merge(ff_merge(s[0][0], s[1][0]), ff_merge(s[2][0], s[3][0]));
}
// sum of the nblk partials part[0..nblk) by one wave (lanes stride, then the butterfly)
__device__ __forceinline__ FF ff_parts(const float2 *__restrict__ part, int nblk) {
    FF a{0.f, 0.f};
    for (int k = (int)lane_id(); k < nblk; k += 64) a = ff_merge(a, FF{part[k].x, part[k].y});
    return ff_wave(a);
}

// 4a. per workgroup: compensated sum of D -> part[blk]
__global__ __launch_bounds__(256) void k_ol_sum(const float *__restrict__ dmean, int64_t n, float2 *__restrict__ part) {
    __shared__ FF s[4][1];
    FF a{0.f, 0.f};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a = ff_add(a, dmean[i]);
    a = ff_block(a, s);
    if (threadIdx.x == 0) part[blockIdx.x] = make_float2(a.hi, a.lo);
}

// 4b. per workgroup: mu from the partial sums (every workgroup the same bits), then the
// compensated sum of (D - mu)^2 -> part2[blk]; workgroup 0 stores mu
__global__ __launch_bounds__(256) void k_ol_var(const float *__restrict__ dmean, int64_t n, const float2 *__restrict__ part,
                                                int nblk, float2 *__restrict__ part2, OlHdr *__restrict__ hdr) {
    __shared__ FF s[4][1];
    __shared__ float s_mu;
    if (threadIdx.x < 64) {
        const FF t = ff_parts(part, nblk);
        if (threadIdx.x == 0) s_mu = (t.hi + t.lo) / (float)n;
    }
    __syncthreads();
    const float mu = s_mu;
    FF a{0.f, 0.f};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = dmean[i] - mu;
        a = ff_add(a, d * d);
    }
    a = ff_block(a, s);
    if (threadIdx.x == 0) {
        part2[blockIdx.x] = make_float2(a.hi, a.lo);
        if (blockIdx.x == 0) hdr->mu = mu;
    }
}

// 4c. threshold from the summed squares: one wave, a fixed order (the same on every run)
__global__ __launch_bounds__(64) void k_ol_thr(const float2 *__restrict__ part2, int nblk, int64_t n, float std_ratio,
                                               OlHdr *__restrict__ hdr) {
    const FF t = ff_parts(part2, nblk);
    if (lane_id() != 0) return;
    const float sigma = sqrtf(fmaxf((t.hi + t.lo) / (float)n, 0.f));
    hdr->sigma = sigma;
    hdr->thr = hdr->mu + std_ratio * sigma;
}

// 4d. keep mask and kept count per workgroup of kOlBlock points
__global__ __launch_bounds__(256) void k_ol_keep(const float *__restrict__ dmean, int64_t n, const OlHdr *__restrict__ hdr,
                                                 uint8_t *__restrict__ keep, uint32_t *__restrict__ part) {
    __shared__ uint32_t s_w[4];
    const float thr = hdr->thr;
    const int64_t base = (int64_t)blockIdx.x * kOlBlock;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kOlItems; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < n) {
            const bool kp = dmean[i] <= thr;
            keep[i] = kp ? 1 : 0;
            c += kp ? 1u : 0u;
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// 4e. compaction of the kept points in input order (offsets from the scanned counts)
__global__ __launch_bounds__(256) void k_ol_write(const float *__restrict__ pts, int64_t n, int64_t stride,
                                                  const uint8_t *__restrict__ keep, const uint32_t *__restrict__ part,
                                                  float *__restrict__ out, int64_t out_stride) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kOlBlock;
    const int l = (int)lane_id(), w = (int)(threadIdx.x >> 6);
    uint32_t run = part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kOlItems; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        const bool take = i < n && keep[i] != 0;
        const uint64_t bal = __ballot(take);
        const uint32_t below = (uint32_t)__popcll(bal & ((1ull << l) - 1ull));
        if (l == 0) s_w[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = run;
        for (int q = 0; q < w; ++q) before += s_w[q];
        const uint32_t total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
        if (take) {
            const int64_t o = (int64_t)before + below;
            out[o] = pts[i];
            out[out_stride + o] = pts[stride + i];
            out[2 * out_stride + o] = pts[2 * stride + i];
        }
        run += total;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int outlier_slot_bits(int64_t n) {
    int b = 12;   // at least 4 bits per axis
    while (b < 22 && ((int64_t)1 << b) < 2 * n) ++b;
    return b;
}

static size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Workspace pieces for n points (offsets in bytes, in this order).
struct OlLayout {
    size_t hdr, keys0, vals0, keys1, vals1, hist, shist, scount, ranges, bpart, spart, kpart, defer, slow, spts, total;
};

size_t sort_count_words(uint64_t);

static OlLayout ol_layout(int64_t n) {
    OlLayout L;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t slots = (size_t)1 << outlier_slot_bits(n);
    size_t o = 0;
    auto take = [&](size_t b) { const size_t at = o; o += al(b); return at; };
    L.hdr = take(sizeof(OlHdr));
    L.keys0 = take(4 * nn);
    L.vals0 = take(4 * nn);
    L.keys1 = take(4 * nn);
    L.vals1 = take(4 * nn);
    L.hist = take(4 * 256 * kMaxPasses);
    L.shist = take(4 * 3 * kOlBins);
    L.scount = take(4 * sort_count_words((uint64_t)nn));
    L.ranges = take(8 * slots);
    L.bpart = take(4 * 6 * kOlRedBlocks);
    L.spart = take(8 * 2 * kOlRedBlocks);   // two float2 partials per reduction workgroup
    L.kpart = take(4 * ((nn + kOlBlock - 1) / kOlBlock + 1));
    L.defer = take(4 * nn);
    L.slow = take(4 * nn);
    L.spts = take(16 * nn);
    L.total = o;
    return L;
}

size_t outlier_workspace_bytes(int64_t n) { return ol_layout(n).total; }

template <int K>
static void knn_launch(const float *pts, int64_t n, int64_t stride, OlHdr *hdr, const float4 *spts,
                       const uint2 *ranges, uint32_t *slow, uint32_t *defer, float *dmean, hipStream_t st) {
    hipLaunchKernelGGL((k_ol_knn<K>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, spts, n, hdr, ranges, slow,
                       defer, dmean);
    const unsigned wb = (unsigned)((n + 3) / 4 < kOlWaveBlocks ? (n + 3) / 4 : kOlWaveBlocks);
    hipLaunchKernelGGL((k_ol_knn_wave<K>), dim3(wb), dim3(256), 0, st, spts, n, hdr, ranges, slow, defer, dmean);
    const unsigned far = (unsigned)(n < kOlFarBlocks ? n : kOlFarBlocks);
    hipLaunchKernelGGL((k_ol_knn_far<K>), dim3(far), dim3(kOlFarThreads), 0, st, spts, pts, n, stride, hdr, defer,
                       dmean);
}

// k in {4, 8, 16, 32}: false (nothing launched) otherwise. out may be null (no compaction).
bool launch_outliers(const float *pts, int64_t n, int64_t stride, int k, float std_ratio, float *dmean, uint8_t *keep,
                     float *out, int64_t out_stride, uint32_t *count, void *ws, hipStream_t st) {
    if (k != 4 && k != 8 && k != 16 && k != 32) return false;
    const OlLayout L = ol_layout(n);
    char *b = (char *)ws;
    OlHdr *hdr = (OlHdr *)(b + L.hdr);
    uint32_t *k0 = (uint32_t *)(b + L.keys0), *v0 = (uint32_t *)(b + L.vals0);
    uint32_t *k1 = (uint32_t *)(b + L.keys1), *v1 = (uint32_t *)(b + L.vals1);
    uint32_t *kpart = (uint32_t *)(b + L.kpart);
    if (n == 0) {
        launch_excl_scan_u32(kpart, 0u, count, st);   // writes the count 0
        return true;
    }
    const int bits = outlier_slot_bits(n);
    const uint32_t slots = 1u << bits;
    const int rb = (int)((n + 255) / 256 < kOlRedBlocks ? (n + 255) / 256 : kOlRedBlocks);
    hipLaunchKernelGGL(k_ol_bbox, dim3(rb), dim3(256), 0, st, pts, n, stride, (float *)(b + L.bpart));
    hipLaunchKernelGGL(k_ol_bbox_final, dim3(1), dim3(384), 0, st, (const float *)(b + L.bpart), rb, hdr);
    launch_fill_u32((uint32_t *)(b + L.shist), 0u, 3 * kOlBins, st);
    hipLaunchKernelGGL(k_ol_hist, dim3(rb), dim3(256), 0, st, pts, n, stride, hdr, (uint32_t *)(b + L.shist));
    hipLaunchKernelGGL(k_ol_setup, dim3(1), dim3(192), 0, st, (const uint32_t *)(b + L.shist), n, (uint32_t)bits, hdr);
    hipLaunchKernelGGL(k_ol_key, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pts, n, stride, hdr, k0, v0);
    launch_fill_u32((uint32_t *)(b + L.hist), 0u, 256 * kMaxPasses, st);
    const int alt = radix_sort_u32(k0, v0, k1, v1, (uint32_t)n, 0u, bits, (uint32_t *)(b + L.hist),
                                   (uint32_t *)(b + L.scount), st);
    const uint32_t *sk = alt ? k1 : k0, *sv = alt ? v1 : v0;
    uint2 *ranges = (uint2 *)(b + L.ranges);
    launch_fill_u32((uint32_t *)ranges, 0u, 2 * (int64_t)slots, st);
    launch_ranges32(sk, (uint32_t)n, ranges, st, nullptr);
    uint32_t *defer = (uint32_t *)(b + L.defer), *slow = (uint32_t *)(b + L.slow);
    float4 *spts = (float4 *)(b + L.spts);
    hipLaunchKernelGGL(k_ol_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pts, n, stride, sv, spts);
    if (k == 4) knn_launch<4>(pts, n, stride, hdr, spts, ranges, slow, defer, dmean, st);
    else if (k == 8) knn_launch<8>(pts, n, stride, hdr, spts, ranges, slow, defer, dmean, st);
    else if (k == 16) knn_launch<16>(pts, n, stride, hdr, spts, ranges, slow, defer, dmean, st);
    else knn_launch<32>(pts, n, stride, hdr, spts, ranges, slow, defer, dmean, st);
    float2 *sp1 = (float2 *)(b + L.spart), *sp2 = sp1 + kOlRedBlocks;
    hipLaunchKernelGGL(k_ol_sum, dim3(rb), dim3(256), 0, st, dmean, n, sp1);
    hipLaunchKernelGGL(k_ol_var, dim3(rb), dim3(256), 0, st, dmean, n, sp1, rb, sp2, hdr);
    hipLaunchKernelGGL(k_ol_thr, dim3(1), dim3(64), 0, st, sp2, rb, n, std_ratio, hdr);
    const uint32_t nblk = (uint32_t)((n + kOlBlock - 1) / kOlBlock);
    hipLaunchKernelGGL(k_ol_keep, dim3(nblk), dim3(256), 0, st, dmean, n, hdr, keep, kpart);
    launch_excl_scan_u32(kpart, nblk, count, st);
    if (out)
        hipLaunchKernelGGL(k_ol_write, dim3(nblk), dim3(256), 0, st, pts, n, stride, keep, kpart, out, out_stride);
    return true;
}

}  // namespace recogs
