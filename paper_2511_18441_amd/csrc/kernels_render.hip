// Render path kernels: preprocess (EWA projection, SH colour, tile rectangle),
// exclusive scan of tile counts, key emission, tile ranges, front-to-back blend.
#include "render_device.hpp"

namespace recogs {

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Also zeroes zero[0, zero_words) (the render's header, histograms, emission sums and
// tile ranges, which only later kernels use): one launch fewer than a separate fill.
template <int DT, int DEG>
__global__ __launch_bounds__(256) void k_preprocess(SceneDev sc, CamDev cam, RecolorDev rc, int keep_bwd,
                                                    SplatRec *__restrict__ rec, float4 *__restrict__ bwd,
                                                    uint32_t *__restrict__ zbits, uint2 *__restrict__ rect,
                                                    uint32_t *__restrict__ count, uint32_t *__restrict__ zero,
                                                    int64_t zero_words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t z = i; z < zero_words; z += (int64_t)gridDim.x * blockDim.x) zero[z] = 0u;
    if (i < sc.n) preprocess_one<DT, DEG>(sc, cam, rc, keep_bwd, i, i, rec, bwd, zbits, rect, count);
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

// HIST: also the chunk's counts of the low 8 depth bits (ScanSort), dcnt[d * nchunks + chunk]
template <bool HIST>
__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ zbits,
                                                     int64_t n, uint64_t *__restrict__ pk, uint32_t *__restrict__ pv,
                                                     uint32_t *__restrict__ pzmn, uint32_t *__restrict__ pzmx,
                                                     uint32_t *__restrict__ dcnt, uint32_t nchunks) {
    __shared__ uint64_t s_k[4];
    __shared__ uint32_t s_v[4], s_zmn[4], s_zmx[4];
    __shared__ uint32_t s_h[HIST ? 256 : 1];
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    if constexpr (HIST) {
        s_h[threadIdx.x] = 0u;
        __syncthreads();
    }
    // striped (coalesced): only sums, minima and maxima are taken here
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    uint64_t tsum = 0;
    uint32_t vsum = 0, zmn = 0xffffffffu, zmx = 0u;
    uint32_t cv[kScanItems], zv[kScanItems];   // every load issued before any is used
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * 256;
        cv[k] = (i < n) ? cnt[i] : 0u;
        zv[k] = (i < n) ? zbits[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t v = cv[k];
        tsum += v;
        if (v) {
            const uint32_t z = zv[k];
            zmn = min(zmn, z);
            zmx = max(zmx, z);
            ++vsum;
            if constexpr (HIST) atomicAdd(&s_h[z & 255u], 1u);
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
    if constexpr (HIST) dcnt[(size_t)threadIdx.x * nchunks + blockIdx.x] = s_h[threadIdx.x];
}

// One workgroup: exclusive scans of the chunk partials in place; header gets K, V and
// the depth range (minimum stored as its complement).
__global__ __launch_bounds__(1024) void k_scan_top(uint64_t *__restrict__ pk, uint32_t *__restrict__ pv,
                                                   const uint32_t *__restrict__ pzmn, const uint32_t *__restrict__ pzmx,
                                                   uint32_t nchunks, uint64_t key_capacity, uint32_t *__restrict__ header) {
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
        header[H_ZMIN_RAW] = runv ? zmn : 0u;
        header[H_KEFF] = runk <= key_capacity ? (uint32_t)runk : 0u;
        header[H_OVERFLOW] = runk > key_capacity ? 1u : 0u;
    }
}

// Down-sweep over one chunk of 4,096 counts. Loads and stores are coalesced through
// LDS: counts and depth bits come in striped, each thread scans 16 consecutive ones,
// and the offsets and the compacted (depth bits, index) pairs go out striped.
// EMIT (tile-first order): instead of the depth bits, the compaction carries what the
// key emission of index-ordered Gaussians needs: each one's tile rectangle (srect) and
// key offset (eoff), and efirst[b] = the compacted Gaussian owning key b * kEmitKeys for
// the blocks b < nblk of the key capacity.
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }   // LDS padding: no 16-way bank conflicts
// With few chunks the down pass scans the chunk partials itself (FOLD): each workgroup
// sums the partials of the chunks before its own, and workgroup 0 also the totals and
// the depth range, which it writes to the header as k_scan_top would; one launch fewer.
struct ScanFold {
    const uint32_t *pzmn, *pzmx;
    uint32_t nchunks;
    uint64_t key_capacity;
    uint32_t *header;
};
__device__ __forceinline__ void scan_fold_prefix(const uint64_t *__restrict__ pk, const uint32_t *__restrict__ pv,
                                                 const ScanFold &f, uint64_t &pre_k, uint32_t &pre_v) {
    __shared__ uint64_t s_k[4];
    __shared__ uint32_t s_v[4], s_mn[4], s_mx[4];
    const uint32_t t = threadIdx.x, w = t >> 6;
    const uint32_t upto = blockIdx.x == 0 ? f.nchunks : blockIdx.x;   // workgroup 0: the totals
    uint64_t k = 0;
    uint32_t v = 0, mn = 0xffffffffu, mx = 0u;
    for (uint32_t c = t; c < upto; c += 256) {
        k += pk[c];
        v += pv[c];
        if (blockIdx.x == 0) { mn = min(mn, f.pzmn[c]); mx = max(mx, f.pzmx[c]); }
    }
    k = wave_sum(k);
    v = wave_sum(v);
    if (blockIdx.x == 0) { mn = wave_min(mn); mx = wave_max(mx); }
    if (lane_id() == 0) { s_k[w] = k; s_v[w] = v; s_mn[w] = mn; s_mx[w] = mx; }
    __syncthreads();
    k = ((s_k[0] + s_k[1]) + s_k[2]) + s_k[3];
    v = ((s_v[0] + s_v[1]) + s_v[2]) + s_v[3];
    if (blockIdx.x == 0) {
        if (t == 0) {
            mn = min(min(s_mn[0], s_mn[1]), min(s_mn[2], s_mn[3]));
            mx = max(max(s_mx[0], s_mx[1]), max(s_mx[2], s_mx[3]));
            f.header[H_K_LO] = (uint32_t)k;
            f.header[H_K_HI] = (uint32_t)(k >> 32);
            f.header[H_V] = v;
            f.header[H_ZMIN] = v ? ~mn : 0u;
            f.header[H_ZMAX] = v ? mx : 0u;
            f.header[H_ZMIN_RAW] = v ? mn : 0u;
            f.header[H_KEFF] = k <= f.key_capacity ? (uint32_t)k : 0u;
            f.header[H_OVERFLOW] = k > f.key_capacity ? 1u : 0u;
        }
        pre_k = 0;
        pre_v = 0;
    } else {
        pre_k = k;
        pre_v = v;
    }
    __syncthreads();
}

// MODE: SD_COMPACT writes the (depth bits, index) pairs of the Gaussians with keys
// compacted in index order; SD_EMIT the tile-first order's compaction (ScanEmit);
// SD_SORT the pairs ordered by their low 8 depth bits (ScanSort: the depth sort's
// first pass, ranked as k_radix_down ranks, from the digit offsets in dcnt).
enum : int { SD_COMPACT = 0, SD_EMIT = 1, SD_SORT = 2 };
template <int MODE>
__global__ __launch_bounds__(256) void k_scan_down(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ zbits,
                                                   uint32_t *__restrict__ off, int64_t n, const uint64_t *__restrict__ pk,
                                                   const uint32_t *__restrict__ pv, uint32_t *__restrict__ dkeys,
                                                   uint32_t *__restrict__ dvals, const uint2 *__restrict__ rect,
                                                   uint2 *__restrict__ srect, uint32_t *__restrict__ eoff,
                                                   uint32_t *__restrict__ efirst, uint32_t nblk, int fold, ScanFold f,
                                                   const uint32_t *__restrict__ dcnt, const uint32_t *__restrict__ dtot) {
    constexpr bool EMIT = MODE == SD_EMIT;
    __shared__ uint64_t s_wk[4];
    __shared__ uint32_t s_wv[4];
    __shared__ uint32_t s_a[kScanChunk + kScanChunk / 32];
    __shared__ uint32_t s_dk[kScanChunk], s_dv[kScanChunk];
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
    // SD_SORT loads the counts wave-striped (wave w: entries 1024 w + 64 r + lane, the
    // order its ranking takes them in) and keeps them, with the depth bits and the digit
    // offsets, in registers: every global load of the workgroup is issued here
    uint32_t cw[MODE == SD_SORT ? kScanItems : 1], zk[MODE == SD_SORT ? kScanItems : 1];
    uint32_t dtot_t = 0, dcnt_t = 0;
    if constexpr (MODE == SD_SORT) {
        const uint32_t wl = (uint32_t)t >> 6, ln = lane_id();
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) {
            const int i = (int)(wl * (64 * kScanItems) + r * 64 + ln);
            cw[r] = (c0 + i < n) ? cnt[c0 + i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) {
            const int i = (int)(wl * (64 * kScanItems) + r * 64 + ln);
            zk[r] = (c0 + i < n) ? zbits[c0 + i] : 0u;
        }
        dtot_t = dtot[t];
        dcnt_t = dcnt[(size_t)t * gridDim.x + blockIdx.x];
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) s_a[scan_pad((int)(wl * (64 * kScanItems) + r * 64 + ln))] = cw[r];
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = k * 256 + t;
            s_a[scan_pad(i)] = (c0 + i < n) ? cnt[c0 + i] : 0u;
        }
    }
    __syncthreads();
    uint32_t v[kScanItems];
    uint64_t tsum = 0;
    uint32_t vsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = s_a[scan_pad(t * kScanItems + k)];
        tsum += v[k];
        vsum += v[k] ? 1u : 0u;
    }
    uint64_t ktot, pre_k;
    uint32_t vtot, pre_v;
    if (fold) {
        scan_fold_prefix(pk, pv, f, pre_k, pre_v);
    } else {   // scanned by k_scan_top
        pre_k = pk[blockIdx.x];
        pre_v = pv[blockIdx.x];
    }
    uint64_t run = pre_k + block_excl_scan<uint64_t, 4>(tsum, s_wk, ktot);
    uint32_t vloc = block_excl_scan<uint32_t, 4>(vsum, s_wv, vtot);   // (the scans end with a barrier)
    const uint32_t vbase = pre_v;
    if constexpr (EMIT) {
        // compacted key offsets; the owners of the key blocks starting in this chunk
        uint64_t r = run;
        uint32_t q = vloc;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (v[k]) {
                s_dk[q] = (uint32_t)r;
                for (uint64_t b = (r + kEmitKeys - 1) / kEmitKeys; b < nblk && b * kEmitKeys < r + v[k]; ++b)
                    efirst[b] = vbase + q;
                s_dv[q] = (uint32_t)(c0 + t * kScanItems + k);
                ++q;
            }
            r += v[k];
        }
        __syncthreads();
        for (uint32_t j = t; j < vtot; j += 256) {
            eoff[vbase + j] = s_dk[j];
            dvals[vbase + j] = s_dv[j];
            srect[vbase + j] = rect[s_dv[j]];   // within the chunk's 4,096 Gaussians: few lines
        }
        __syncthreads();
    } else if constexpr (MODE == SD_COMPACT) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = k * 256 + t;
            s_a[scan_pad(i)] = (c0 + i < n) ? zbits[c0 + i] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (v[k]) {
                const int i = t * kScanItems + k;
                s_dk[vloc] = s_a[scan_pad(i)];
                s_dv[vloc] = (uint32_t)(c0 + i);
                ++vloc;
            }
        }
        __syncthreads();
    } else {
        // wave w ranks Gaussians [1024 w, 1024 w + 1024) of the chunk, 64 per round, so
        // the ranks follow index order; then digit order through LDS (s_dk, s_dv) and out
        // as contiguous runs at the digits' offsets
        __shared__ uint32_t s_whist[4][256];
        __shared__ uint32_t s_gbase[256], s_lstart[256];
        const uint32_t lane = lane_id(), w = (uint32_t)t >> 6;
        for (int i = t; i < 4 * 256; i += 256) (&s_whist[0][0])[i] = 0u;
        {
            uint32_t all;
            const uint32_t dbase = block_excl_scan<uint32_t, 4>(dtot_t, s_wv, all);
            s_gbase[t] = dbase + dcnt_t;
        }
        __syncthreads();
        uint32_t rk[kScanItems], vm = 0u;
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) vm |= (cw[r] != 0u ? 1u : 0u) << r;
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) {
            const bool valid = (vm >> r) & 1u;
            const uint32_t d = zk[r] & 255u;
            uint64_t m = wave_ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = wave_ballot(bit);
                m &= bit ? bb : ~bb;
            }
            const uint32_t below = rank_below(m);
            uint32_t prior = 0;
            if (valid) prior = s_whist[w][d];
            rk[r] = prior + below;
            if (valid && below == 0) s_whist[w][d] = prior + (uint32_t)__popcll(m);
        }
        __syncthreads();
        uint32_t dt = 0;   // thread t = digit t: prefix over the waves, then over the digits
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            const uint32_t x = s_whist[ww][t];
            s_whist[ww][t] = dt;
            dt += x;
        }
        uint32_t ntot;
        const uint32_t ls = block_excl_scan<uint32_t, 4>(dt, s_wv, ntot);
        s_lstart[t] = ls;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kScanItems; ++r) {
            if ((vm >> r) & 1u) {
                const uint32_t d = zk[r] & 255u;
                const uint32_t pos = s_lstart[d] + s_whist[w][d] + rk[r];
                s_dk[pos] = zk[r];
                s_dv[pos] = (uint32_t)(c0 + (int64_t)(w * (64 * kScanItems) + r * 64 + lane));
            }
        }
        __syncthreads();
        for (uint32_t j = t; j < ntot; j += 256) {
            const uint32_t z = s_dk[j], d = z & 255u;
            const uint32_t dst = s_gbase[d] + (j - s_lstart[d]);
            dkeys[dst] = z;
            dvals[dst] = s_dv[j];
        }
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        s_a[scan_pad(t * kScanItems + k)] = (uint32_t)run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int i = k * 256 + t;
        if (c0 + i < n) off[c0 + i] = s_a[scan_pad(i)];
    }
    if constexpr (MODE == SD_COMPACT) {
        for (uint32_t j = t; j < vtot; j += 256) {
            dkeys[vbase + j] = s_dk[j];
            dvals[vbase + j] = s_dv[j];
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
// (tile, depth, index) order.
//   k_emit_reduce:  per chunk of 1,024 depth-ordered Gaussians, gathers each one's
//                   tile rectangle once and sums the chunk's key counts (for one view
//                   the depth sort's last pass does this as it writes the order)
//   k_scan_top_u32: chunk sums -> chunk key offsets (more than 2,048 chunks)
//   k_emit_offsets: per-Gaussian key offsets, and for every block of kEmitKeys keys
//                   the Gaussian owning its first key
//   k_emit_down:    one workgroup per block of kEmitKeys keys (the work is balanced by
//                   keys, not by Gaussians, whose counts range from 1 to thousands);
//                   the owner of each key comes from a max-scan of the Gaussians'
//                   start positions in LDS, and keys are written coalesced
// ---------------------------------------------------------------------------
// also gathers each depth-ordered Gaussian's tile rectangle once (srect, coalesced
// for k_emit_down); every Gaussian in the order has at least one key
__global__ __launch_bounds__(256) void k_emit_reduce(const uint32_t *__restrict__ order, uint32_t V,
                                                     const uint2 *__restrict__ rect, uint2 *__restrict__ srect,
                                                     uint32_t *__restrict__ esum, const uint32_t *dynV) {
    if (dynV) V = *dynV;
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

// fold: epre holds the chunks' unscanned key counts, and each workgroup adds those of the
// chunks before its own (few chunks; one launch fewer than a separate scan)
__global__ __launch_bounds__(256) void k_emit_offsets(const uint2 *__restrict__ srect, uint32_t V,
                                                      const uint32_t *__restrict__ epre, uint32_t *__restrict__ eoff,
                                                      uint32_t *__restrict__ efirst, uint32_t nblk,
                                                      const uint32_t *dynV, const uint32_t *overflow, int fold) {
    if (dynV) V = *dynV;
    if (overflow && *overflow) return;
    const uint32_t base = blockIdx.x * (uint32_t)kEmitChunk;
    if (base >= V) return;
    __shared__ uint32_t s_w[4];
    const uint32_t t = threadIdx.x;
    constexpr int R = kEmitChunk / 256;
    uint2 rr[R];   // the chunk's rectangles, loaded before the chunk sums
#pragma unroll
    for (int r = 0; r < R; ++r) {  // thread t holds Gaussians base + R t + r (blocked)
        const uint32_t j = base + R * t + r;
        rr[r] = j < V ? srect[j] : make_uint2(0u, 0u);
    }
    uint32_t pre;
    if (fold) {
        uint32_t a = 0;
        for (uint32_t c = t; c < blockIdx.x; c += 256) a += epre[c];
        a = wave_sum(a);
        if (lane_id() == 0) s_w[t >> 6] = a;
        __syncthreads();
        pre = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
        __syncthreads();
    } else {
        pre = epre[blockIdx.x];
    }
    uint32_t c[R], sum = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t j = base + R * t + r;
        c[r] = j < V ? rect_count(rr[r]) : 0u;
        sum += c[r];
    }
    uint32_t tot;
    uint32_t run = pre + block_excl_scan<uint32_t, 4>(sum, s_w, tot);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t j = base + R * t + r;
        if (j < V) {
            eoff[j] = run;
            // key blocks whose first key lies in [run, run + c)
            for (uint32_t b = (run + kEmitKeys - 1) / kEmitKeys; b < nblk && b * kEmitKeys < run + c[r]; ++b) efirst[b] = j;
            run += c[r];
        }
    }
}

// exclusive max-scan over the workgroup of one value per thread (256 threads; 0 for thread 0)
__device__ __forceinline__ uint32_t block_excl_max256(uint32_t v, uint32_t *s_w) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t x = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc = x > inc ? x : inc;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = __shfl_up(inc, 1, 64);
    if (lane == 0) pre = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < (int)w) pre = s_w[k] > pre ? s_w[k] : pre;
    __syncthreads();
    return pre;
}

// Batches (nviews > 1): values are (view, Gaussian) pair indices and tile ids are global,
// tile_base(view) + local id; vtab[v] = (pair_base, tile_base, tiles_x, -) per view.
__global__ __launch_bounds__(256) void k_emit_down(const uint32_t *__restrict__ order, uint32_t V, uint32_t K,
                                                   const uint2 *__restrict__ srect, const uint32_t *__restrict__ eoff,
                                                   const uint32_t *__restrict__ efirst, int tiles_x,
                                                   uint32_t *__restrict__ tkeys, uint32_t *__restrict__ tvals,
                                                   const uint32_t *dynV, const uint32_t *dynK, const uint32_t *overflow,
                                                   const uint4 *__restrict__ vtab, int nviews, KeyCount kc) {
    if (dynV) V = *dynV;
    if (dynK) K = *dynK;
    if (overflow && *overflow) return;
    const uint32_t k0 = blockIdx.x * kEmitKeys;
    if (k0 >= K) return;
    const uint32_t k1 = min(K, k0 + kEmitKeys);
    constexpr int E = kEmitKeys / 256;
    __shared__ uint32_t s_own[kEmitKeys];
    __shared__ uint32_t s_st[256], s_val[256], s_tb[256], s_tx[256];
    __shared__ uint2 s_rect[256];
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_end;
    __shared__ uint32_t s_kc[256];
    const uint32_t t = threadIdx.x;
    const uint32_t kmask = (1u << kc.nbits) - 1u;
    if (kc.cnt) s_kc[t] = 0u;   // (the first round's barriers order these before the adds)
    uint32_t g = efirst[blockIdx.x];  // owns key k0
    uint32_t kb = k0;
    while (kb < k1) {
        // a round: up to 256 consecutive Gaussians from g, and the keys they own in [kb, k1)
        const uint32_t gi = g + t;
        // the three loads go out together (the rectangle and value are not known to be
        // needed until the start offset is in)
        const uint32_t st = gi < V ? eoff[gi] : 0xffffffffu;
        const uint2 rc = gi < V ? srect[gi] : make_uint2(0u, 0u);
        const uint32_t gv = gi < V ? order[gi] : 0u;
        const bool in = gi < V && st < k1;
        if (in) {
            uint32_t tb = 0, txn = (uint32_t)tiles_x;
            if (nviews > 1) {  // view of the pair: last v with pair_base <= gv
                int lo = 0, hi = nviews - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (vtab[mid].x <= gv) lo = mid;
                    else hi = mid - 1;
                }
                tb = vtab[lo].y;
                txn = vtab[lo].z;
            }
            s_st[t] = st;
            s_rect[t] = rc;
            s_val[t] = gv;
            s_tb[t] = tb;
            s_tx[t] = txn;
            if (t == 255) s_end = min(k1, st + rect_count(rc));
        } else if (t == 255) {
            s_end = k1;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) s_own[e * 256 + t] = 0u;
        __syncthreads();
        const uint32_t ke = s_end;
        // starts strictly increase and Gaussian g starts at or before kb
        if (in && t > 0 && st < ke) s_own[st - kb] = t;
        __syncthreads();
        // owner of every key: inclusive max-scan of the marks (thread t: entries E t ..)
        uint32_t loc[E], m = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t x = s_own[E * t + e];
            m = x > m ? x : m;
            loc[e] = m;
        }
        const uint32_t pre = block_excl_max256(m, s_w);
#pragma unroll
        for (int e = 0; e < E; ++e) s_own[E * t + e] = loc[e] > pre ? loc[e] : pre;
        __syncthreads();
        for (uint32_t q = kb + t; q < ke; q += 256) {
            const uint32_t i = s_own[q - kb];
            const uint32_t k = q - s_st[i];
            const uint2 rc = s_rect[i];
            const uint32_t tx0 = rc.x & 0xffffu, tx1 = rc.x >> 16, ty0 = rc.y & 0xffffu;
            const uint32_t wd = tx1 - tx0 + 1;
            const uint32_t ty = ty0 + k / wd, tx = tx0 + k % wd;
            const uint32_t tile = s_tb[i] + ty * s_tx[i] + tx;
            tkeys[q] = tile;
            tvals[q] = s_val[i];
            if (kc.cnt) atomicAdd(&s_kc[tile & kmask], 1u);
        }
        __syncthreads();
        kb = ke;
        g += 256;
    }
    if (kc.cnt && t <= kmask) kc.cnt[(size_t)t * kc.chunks + blockIdx.x] = s_kc[t];
}

// [first, last+1) of each tile in tile-sorted 32-bit tile ids (ranges zeroed beforehand).
// A thread takes 4 consecutive keys with one 16-byte load (the last group of a ragged
// K key by key) and compares each with its neighbour.
__global__ __launch_bounds__(256) void k_ranges32(const uint32_t *__restrict__ tiles, uint32_t K, uint2 *__restrict__ ranges,
                                                  const uint32_t *dynK) {
    if (dynK) K = *dynK;
    const uint32_t groups = (K + 3) / 4;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < groups; g += gridDim.x * blockDim.x) {
        const uint32_t k0 = 4 * g;
        uint32_t v[4];
        if (k0 + 3 < K) {
            const uint4 q = *reinterpret_cast<const uint4 *>(tiles + k0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = k0 + j < K ? tiles[k0 + j] : 0xffffffffu;
        }
        uint32_t prev = k0 > 0 ? tiles[k0 - 1] : 0xffffffffu;
        const uint32_t next = k0 + 4 < K ? tiles[k0 + 4] : 0xffffffffu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t k = k0 + j;
            if (k < K) {
                const uint32_t t = v[j];
                const uint32_t after = j < 3 ? v[j + 1] : next;
                if (prev != t) ranges[t].x = k;
                if (k == K - 1 || after != t) ranges[t].y = k + 1;
                prev = t;
            }
        }
    }
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
// its pixels have. Output HWC image and, with STATE (for the backward), the final
// transmittance and per pixel the count of tile-list entries up to and including
// the last blended one.
// ---------------------------------------------------------------------------
template <int TW, int TH, int PPT, bool STATE>
__global__ __launch_bounds__(TW *TH / PPT) void k_blend(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                                       const SplatRec *__restrict__ rec, int W, int H, int tiles_x,
                                                       float bg0, float bg1, float bg2, float *__restrict__ image,
                                                       int chw, float *__restrict__ finalT, uint32_t *__restrict__ nproc) {
    __shared__ BlendStage sm;
    blend_tile<TW, TH, PPT, STATE>(blockIdx.x, ranges[blockIdx.x], vals, rec, W, H, tiles_x, bg0, bg1, bg2, image, chw,
                                   finalT, nproc, sm);
}

// Region form: one wave per 8 x 8*PPT region. Workgroup b runs on XCD b mod 8; the
// regions of a tile take consecutive workgroups of one XCD (so its list is read
// through one L2), and the tiles are dealt to the XCDs in turn. DEPTH: also the rough
// depth map (depth [H][W], from the per-record depth bits zbits and threshold tau).
template <int TW, int TH, int PPT, bool STATE, bool DEPTH>
__global__ __launch_bounds__(64) void k_blend_region(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                                    const SplatRec *__restrict__ rec, int W, int H, int tiles_x,
                                                    uint32_t ntiles, float bg0, float bg1, float bg2,
                                                    float *__restrict__ image, int chw, float *__restrict__ finalT,
                                                    uint32_t *__restrict__ nproc, const uint32_t *__restrict__ zbits,
                                                    float tau, float *__restrict__ depth) {
    constexpr uint32_t NR = (TW / 8) * (TH / (8 * PPT));
    __shared__ BlendRec sm[64];
    const uint32_t b = blockIdx.x, j = b >> 3;
    const uint32_t tile = (j / NR) * 8u + (b & 7u);
    if (tile >= ntiles) return;
    blend_region<TW, TH, PPT, STATE, DEPTH>((int)tile, (int)(j % NR), ranges[tile], vals, rec, W, H, tiles_x, bg0, bg1,
                                            bg2, image, chw, finalT, nproc, sm, zbits, tau, depth);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// p[0, mult * (*dyn)) = v, the count read on the device (at most max_count words)
__global__ __launch_bounds__(256) void k_fill_u32_dyn(uint32_t *__restrict__ p, uint32_t v, const uint32_t *dyn,
                                                      uint32_t mult, int64_t max_count) {
    const int64_t c = (int64_t)mult * (int64_t)*dyn;
    const int64_t count = c < max_count ? c : max_count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

void launch_fill_u32_dyn(uint32_t *p, uint32_t v, const uint32_t *dyn, uint32_t mult, int64_t max_count, hipStream_t st) {
    if (max_count <= 0) return;
    int64_t blocks = (max_count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32_dyn, dim3((unsigned)blocks), dim3(256), 0, st, p, v, dyn, mult, max_count);
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, count);
}

#define RECOGS_PRE(D)                                                                                                  \
    hipLaunchKernelGGL((k_preprocess<DT, D>), g, dim3(256), 0, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, zero, zw)
template <int DT>
static void preprocess_dt(int deg, dim3 g, hipStream_t st, const SceneDev &sc, const CamDev &cam, const RecolorDev &rc,
                          int keep, SplatRec *rec, float4 *bwd, uint32_t *zb, uint2 *rect, uint32_t *cnt, uint32_t *zero,
                          int64_t zw) {
    switch (deg) {
    case 0: RECOGS_PRE(0); break;
    case 1: RECOGS_PRE(1); break;
    case 2: RECOGS_PRE(2); break;
    default: RECOGS_PRE(3); break;
    }
}
#undef RECOGS_PRE

// zero (optional): zero_words words zeroed by the same launch (with no Gaussian, a fill)
void launch_preprocess(int dt, int deg, const SceneDev &sc, const CamDev &cam, const RecolorDev &rc, int keep,
                       SplatRec *rec, float4 *bwd, uint32_t *zb, uint2 *rect, uint32_t *cnt, hipStream_t st,
                       uint32_t *zero, int64_t zero_words) {
    if (!zero) zero_words = 0;
    if (sc.n <= 0) {
        launch_fill_u32(zero, 0u, zero_words, st);
        return;
    }
    const dim3 g((unsigned)((sc.n + 255) / 256));
    if (dt == RECOGS_F32) preprocess_dt<RECOGS_F32>(deg, g, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, zero, zero_words);
    else if (dt == RECOGS_F16) preprocess_dt<RECOGS_F16>(deg, g, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, zero, zero_words);
    else preprocess_dt<RECOGS_BF16>(deg, g, st, sc, cam, rc, keep, rec, bwd, zb, rect, cnt, zero, zero_words);
}

void launch_rowscan(uint32_t *cnt, uint32_t chunks, uint32_t chunk_keys, uint32_t *tot, uint32_t K, int nbits,
                    hipStream_t st);

// emit non-null (tile-first order): the compaction carries rect -> emit->srect, key offsets
// -> emit->eoff and the key blocks' owners -> emit->efirst (blocks of the key capacity);
// otherwise the depth bits -> dkeys. sort (optional, not with emit): the scan is also the
// depth sort's first pass (ScanSort).
void launch_scan(const uint32_t *cnt, const uint32_t *zbits, uint32_t *off, int64_t n, uint64_t *pk, uint32_t *pv,
                 uint32_t *pzmn, uint32_t *pzmx, uint32_t *dkeys, uint32_t *dvals, uint32_t *hdr, int64_t key_capacity,
                 hipStream_t st, const ScanEmit *emit, const ScanSort *sort) {
    if (n <= 0) return;
    const uint32_t nchunks = (uint32_t)((n + kScanChunk - 1) / kScanChunk);
    if (sort) {
        hipLaunchKernelGGL(k_scan_reduce<true>, dim3(nchunks), dim3(256), 0, st, cnt, zbits, n, pk, pv, pzmn, pzmx,
                           sort->dcnt, nchunks);
        launch_rowscan(sort->dcnt, nchunks, (uint32_t)kScanChunk, sort->dtot, (uint32_t)n, 8, st);
    } else {
        hipLaunchKernelGGL(k_scan_reduce<false>, dim3(nchunks), dim3(256), 0, st, cnt, zbits, n, pk, pv, pzmn, pzmx,
                           nullptr, nchunks);
    }
    // up to 1,024 chunks (4M Gaussians) the down pass scans the partials itself
    const int fold = nchunks <= 1024u;
    const ScanFold f{pzmn, pzmx, nchunks, (uint64_t)key_capacity, hdr};
    if (!fold)
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, pk, pv, pzmn, pzmx, nchunks, (uint64_t)key_capacity, hdr);
    if (emit) {
        const uint32_t nblk = (uint32_t)(((uint64_t)key_capacity + kEmitKeys - 1) / kEmitKeys);
        hipLaunchKernelGGL(k_scan_down<SD_EMIT>, dim3(nchunks), dim3(256), 0, st, cnt, zbits, off, n, pk, pv, dkeys, dvals,
                           emit->rect, emit->srect, emit->eoff, emit->efirst, nblk, fold, f, nullptr, nullptr);
    } else if (sort) {
        hipLaunchKernelGGL(k_scan_down<SD_SORT>, dim3(nchunks), dim3(256), 0, st, cnt, zbits, off, n, pk, pv, sort->keys,
                           sort->vals, nullptr, nullptr, nullptr, nullptr, 0u, fold, f, sort->dcnt, sort->dtot);
    } else {
        hipLaunchKernelGGL(k_scan_down<SD_COMPACT>, dim3(nchunks), dim3(256), 0, st, cnt, zbits, off, n, pk, pv, dkeys,
                           dvals, nullptr, nullptr, nullptr, nullptr, 0u, fold, f, nullptr, nullptr);
    }
}

// Key emission of the Gaussians the scan compacted in index order (tile-first order):
// one workgroup per block of kEmitKeys keys, from the compaction's rectangles, offsets
// and block owners (k_emit_down). V and K are counts or, with dynV / dynK, bounds.
void launch_emit_compacted(const uint32_t *order, uint32_t V, const uint2 *srect, const uint32_t *eoff,
                           const uint32_t *efirst, uint32_t K, int tiles_x, uint32_t *tkeys, uint32_t *tvals, hipStream_t st,
                           const uint32_t *dynV, const uint32_t *dynK, const uint32_t *hdr, const uint4 *vtab, int nviews,
                           const KeyCount *kc) {
    if (V == 0 || K == 0) return;
    const uint32_t nblk = (K + kEmitKeys - 1) / kEmitKeys;
    const KeyCount none{nullptr, 0u, 0};
    hipLaunchKernelGGL(k_emit_down, dim3(nblk), dim3(256), 0, st, order, V, K, srect, eoff, efirst, tiles_x, tkeys, tvals,
                       dynV, dynK, hdr ? hdr + H_OVERFLOW : nullptr, vtab, nviews, kc ? *kc : none);
}

// V is the count or, with dynV, its upper bound; hdr (optional) supplies the overflow flag.
void launch_emit_sorted(const uint32_t *order, uint32_t V, const uint2 *rect, uint2 *srect, int tiles_x,
                        uint32_t *esum, uint32_t *eoff, uint32_t *efirst, uint32_t K, uint32_t *tkeys, uint32_t *tvals,
                        hipStream_t st, const uint32_t *dynV, const uint32_t *dynK, const uint32_t *hdr,
                        const uint4 *vtab, int nviews, int folded, const KeyCount *kc) {
    if (V == 0 || K == 0) return;
    const uint32_t chunks = (V + kEmitChunk - 1) / kEmitChunk;
    const uint32_t nblk = (K + kEmitKeys - 1) / kEmitKeys;
    const uint32_t *ovf = hdr ? hdr + H_OVERFLOW : nullptr;
    // folded: the depth sort's last pass has gathered srect and summed esum (EmitFold)
    if (!folded) hipLaunchKernelGGL(k_emit_reduce, dim3(chunks), dim3(256), 0, st, order, V, rect, srect, esum, dynV);
    // up to 2,048 chunks (2M depth-ordered Gaussians) the offsets pass scans the sums itself
    const int fold = chunks <= 2048u;
    if (!fold) hipLaunchKernelGGL(k_scan_top_u32, dim3(1), dim3(1024), 0, st, esum, chunks);
    hipLaunchKernelGGL(k_emit_offsets, dim3(chunks), dim3(256), 0, st, srect, V, esum, eoff, efirst, nblk, dynV, ovf, fold);
    const KeyCount none{nullptr, 0u, 0};
    hipLaunchKernelGGL(k_emit_down, dim3(nblk), dim3(256), 0, st, order, V, K, srect, eoff, efirst, tiles_x, tkeys, tvals,
                       dynV, dynK, ovf, vtab, nviews, kc ? *kc : none);
}

uint32_t emit_blocks(uint32_t K) { return (K + kEmitKeys - 1) / kEmitKeys; }

void launch_ranges32(const uint32_t *tiles, uint32_t K, uint2 *ranges, hipStream_t st, const uint32_t *dynK) {
    if (K == 0) return;
    uint32_t blocks = ((K + 3) / 4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_ranges32, dim3(blocks), dim3(256), 0, st, tiles, K, ranges, dynK);
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
                      int H, int tiles_x, const float *bg, float *image, int chw, float *finalT, uint32_t *nproc,
                      const uint32_t *zbits, float tau, float *depth) {
    if constexpr (region_shape(TW, TH, PPT)) {
        constexpr uint32_t NR = (TW / 8) * (TH / (8 * PPT));
        const dim3 g((unsigned)(((uint32_t)ntiles + 7u) / 8u * 8u * NR));
#define RECOGS_REGION(S, D)                                                                                          \
    hipLaunchKernelGGL((k_blend_region<TW, TH, PPT, S, D>), g, dim3(64), 0, st, ranges, vals, rec, W, H, tiles_x,    \
                       (uint32_t)ntiles, bg[0], bg[1], bg[2], image, chw, finalT, nproc, zbits, tau, depth)
        if (finalT && depth) RECOGS_REGION(true, true);
        else if (finalT) RECOGS_REGION(true, false);
        else if (depth) RECOGS_REGION(false, true);
        else RECOGS_REGION(false, false);
#undef RECOGS_REGION
    } else {
        if (finalT)
            hipLaunchKernelGGL((k_blend<TW, TH, PPT, true>), dim3(ntiles), dim3(TW * TH / PPT), 0, st, ranges, vals, rec, W,
                               H, tiles_x, bg[0], bg[1], bg[2], image, chw, finalT, nproc);
        else
            hipLaunchKernelGGL((k_blend<TW, TH, PPT, false>), dim3(ntiles), dim3(TW * TH / PPT), 0, st, ranges, vals, rec,
                               W, H, tiles_x, bg[0], bg[1], bg[2], image, chw, nullptr, nullptr);
    }
}

// chw: write the image as [3][H][W] instead of [H][W][3]. depth non-null: also the
// rough depth map (region shapes only: false otherwise, nothing launched).
bool launch_blend(int tw, int th, int ppt, int ntiles, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec,
                  int W, int H, int tiles_x, const float *bg, float *image, int chw, float *finalT, uint32_t *nproc,
                  const uint32_t *zbits, float tau, float *depth, hipStream_t st) {
    if (depth && !region_shape(tw, th, ppt)) return false;
#define RECOGS_BLEND_CASE(A, B, P)                                                                                      \
    if (tw == A && th == B && ppt == P) {                                                                               \
        blend_one<A, B, P>(ntiles, st, ranges, vals, rec, W, H, tiles_x, bg, image, chw, finalT, nproc, zbits, tau,    \
                           depth);                                                                                      \
        return true;                                                                                                    \
    }
    RECOGS_BLEND_CASE(16, 16, 1) RECOGS_BLEND_CASE(16, 16, 2) RECOGS_BLEND_CASE(16, 16, 4)
    RECOGS_BLEND_CASE(8, 8, 1) RECOGS_BLEND_CASE(8, 8, 2) RECOGS_BLEND_CASE(8, 8, 4)
    RECOGS_BLEND_CASE(32, 8, 1) RECOGS_BLEND_CASE(32, 8, 2) RECOGS_BLEND_CASE(32, 8, 4)
    RECOGS_BLEND_CASE(32, 16, 1) RECOGS_BLEND_CASE(32, 16, 2) RECOGS_BLEND_CASE(32, 16, 4)
    RECOGS_BLEND_CASE(32, 32, 1) RECOGS_BLEND_CASE(32, 32, 2) RECOGS_BLEND_CASE(32, 32, 4)
#undef RECOGS_BLEND_CASE
    return false;
}

}  // namespace recogs
