// Device radix sort (stable LSD, up to 8-bit digits) with 32-bit values, used for
// the (tile, depth) order of the tile lists.
//
// Keys are 64-bit (tile << 32) | depth_bits or 32-bit (depth bits or tile id). The
// digits come from a view of the key that keeps only its significant bits:
//   KV_TILE_DEPTH (64-bit): (tile << dbits) | (depth_bits - zmin)
//   KV_SUB        (32-bit): key - zmin
// Both views preserve the key order among the keys of one render.
//
// Each pass is reduce-then-scan, with no waiting between workgroups:
//   up:      per chunk of 4,096 keys, the digit counts -> matrix [digit][chunk]
//   rowscan: one workgroup per digit scans its row in place and writes the row total
//   down:    per chunk, the digits' global bases come from an exclusive scan of the
//            row totals (256 words, done by every workgroup); keys are ranked stably
//            per digit with wave ballots (a 64-lane match mask built from one ballot
//            per digit bit, rank = popcount of the lower lanes), staged through LDS in
//            digit order and written as contiguous runs at the offsets of the matrix.
// A single-pass "decoupled look-back" form was measured slower here: its prefix
// frontier advances only a window of chunks per cross-XCD round trip.
#include "recogs_internal.hpp"

namespace recogs {

enum : int { KV_TILE_DEPTH = 0, KV_SUB = 1 };

template <typename KT, int VIEW>
__device__ __forceinline__ uint32_t digit_of(KT key, uint32_t zmin, int dbits, int shift, uint32_t dmask) {
    if constexpr (VIEW == KV_TILE_DEPTH) return (uint32_t)(sort_view((uint64_t)key, zmin, dbits) >> shift) & dmask;
    else return ((uint32_t)key - zmin) >> shift & dmask;
}

// exclusive scan of one value per thread over a 256-thread workgroup
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *s_w, uint32_t &total) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t x = s_w[k];
        if (k < (int)w) pre += x;
        total += x;
    }
    __syncthreads();
    return pre + inc - v;
}

// Counts and the depth minimum may live in device memory (dyn_count, dyn_zmin non-null:
// the graph-capturable batch, whose host code never reads them back); grids are then
// sized for the capacity and workgroups past the live count return at once.
__device__ __forceinline__ void dyn_args(const uint32_t *dyn_count, const uint32_t *dyn_zmin, uint32_t &K, uint32_t &zmin) {
    if (dyn_count) K = *dyn_count;
    if (dyn_zmin) zmin = *dyn_zmin;
}

// per-chunk digit counts -> cnt[digit * chunks + chunk]; a chunk is 256 x ITEMS keys.
// spec (a device count whose bound K is near it): the chunk's keys are loaded below the
// bound before the count arrives, so the count costs no round trip of its own
template <typename KT, int VIEW, int ITEMS>
__global__ __launch_bounds__(256) void k_radix_up(const KT *__restrict__ kin, uint32_t K, uint32_t zmin, int dbits,
                                                  int shift, int nbits, uint32_t *__restrict__ cnt, uint32_t chunks,
                                                  const uint32_t *dyn_count, const uint32_t *dyn_zmin, int spec) {
    constexpr uint32_t CHUNK = 256 * ITEMS;
    const uint32_t t = threadIdx.x;
    const uint32_t base = blockIdx.x * CHUNK;
    KT kk[ITEMS];
    if (spec) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) kk[r] = base + r * 256 + t < K ? kin[base + r * 256 + t] : (KT)0;
    }
    dyn_args(dyn_count, dyn_zmin, K, zmin);
    if (base >= K) return;
    __shared__ uint32_t h[256];
    h[t] = 0;
    __syncthreads();
    const uint32_t dmask = (1u << nbits) - 1u;
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base + r * 256 + t;
        if (idx < K) atomicAdd(&h[digit_of<KT, VIEW>(spec ? kk[r] : kin[idx], zmin, dbits, shift, dmask)], 1u);
    }
    __syncthreads();
    if (t <= dmask) cnt[(size_t)t * chunks + blockIdx.x] = h[t];
}

// workgroup d: cnt[d][c] <- sum_{c' < c} cnt[d][c'];  tot[d] <- sum_c cnt[d][c].
// Four counts per thread, so a row of up to 1,024 chunks is one round of loads.
__global__ __launch_bounds__(256) void k_radix_rowscan(uint32_t *__restrict__ cnt, uint32_t chunks, uint32_t chunk_keys,
                                                       uint32_t *__restrict__ tot, uint32_t K,
                                                       const uint32_t *dyn_count) {
    __shared__ uint32_t s_w[4];
    const uint32_t d = blockIdx.x, t = threadIdx.x;
    uint32_t *row = cnt + (size_t)d * chunks;
    // the row's first 1,024 entries are loaded before the device count arrives (it would
    // cost a memory round trip of its own); entries past the live chunks are not summed
    uint32_t v0[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v0[i] = 4 * t + i < chunks ? row[4 * t + i] : 0u;
    if (dyn_count) K = *dyn_count;
    const uint32_t live = (K + chunk_keys - 1) / chunk_keys;   // chunks holding keys; row stride stays `chunks`
    uint32_t run = 0, total;
    for (uint32_t c0 = 0; c0 < live; c0 += 1024) {
        const uint32_t c = c0 + 4 * t;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = c + i < live ? (c0 == 0 ? v0[i] : row[c + i]) : 0u;
            sum += v[i];
        }
        uint32_t e = run + block_excl_scan256(sum, s_w, total);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (c + i < live) row[c + i] = e;
            e += v[i];
        }
        run += total;
    }
    if (t == 0) tot[d] = run;
}

// EF (the last pass of the depth order): also the emission fold (EmitFold).
template <typename KT, int VIEW, int ITEMS, bool EF>
__global__ __launch_bounds__(256) void k_radix_down(const KT *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                    KT *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t K,
                                                    uint32_t zmin, int dbits, int shift, int nbits,
                                                    const uint32_t *__restrict__ off, const uint32_t *__restrict__ dtot,
                                                    uint32_t chunks, const uint32_t *dyn_count,
                                                    const uint32_t *dyn_zmin, EmitFold ef, int spec) {
    constexpr uint32_t CHUNK = 256 * ITEMS;
    const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
    const uint32_t chunk = blockIdx.x;
    const uint32_t cbase = chunk * (uint32_t)CHUNK;
    // every global load of the workgroup goes out first (the chunk's keys and values, the
    // digit totals, this chunk's digit offsets): one memory round trip, not three; with
    // spec (as k_radix_up) the keys and values go out before a device count too
    KT key[ITEMS];
    uint32_t val[ITEMS], rank[ITEMS];
    auto load_items = [&]() {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint32_t idx = cbase + w * (64 * ITEMS) + r * 64 + lane;
            const bool valid = idx < K;
            key[r] = valid ? kin[idx] : (KT)0;
            val[r] = valid ? vin[idx] : 0u;
        }
    };
    if (spec) load_items();
    dyn_args(dyn_count, dyn_zmin, K, zmin);
    if (cbase >= K) return;
    if (!spec) load_items();
    __shared__ uint32_t s_whist[4][256];   // per-wave digit counts, then per-wave digit prefix
    __shared__ uint32_t s_gbase[256];      // global position of this chunk's first key of each digit
    __shared__ uint32_t s_lstart[256];     // position in the LDS stage of each digit
    __shared__ uint32_t s_w[4];
    __shared__ KT s_keys[CHUNK];
    __shared__ uint32_t s_vals[CHUNK];

    const uint32_t dmask = (1u << nbits) - 1u;
    const uint32_t tot_t = t <= dmask ? dtot[t] : 0u;
    const uint32_t off_t = t <= dmask ? off[(size_t)t * chunks + chunk] : 0u;
    for (int i = t; i < 4 * 256; i += 256) (&s_whist[0][0])[i] = 0;
    {
        uint32_t all;
        const uint32_t dbase = block_excl_scan256(tot_t, s_w, all);
        if (t <= dmask) s_gbase[t] = dbase + off_t;
    }
    __syncthreads();
    // stable rank within the wave, round by round (wave w holds a contiguous quarter)
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = cbase + w * (64 * ITEMS) + r * 64 + lane;
        const bool valid = idx < K;
        const uint32_t d = digit_of<KT, VIEW>(key[r], zmin, dbits, shift, dmask);
        uint64_t m = wave_ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = wave_ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = rank_below(m);
        uint32_t prior = 0;
        if (valid) prior = s_whist[w][d];
        rank[r] = prior + below;
        if (valid && below == 0) s_whist[w][d] = prior + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // per digit (thread t = digit t): prefix over waves and chunk total
    uint32_t tot = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
        const uint32_t c = s_whist[ww][t];
        s_whist[ww][t] = tot;
        tot += c;
    }
    uint32_t total;
    s_lstart[t] = block_excl_scan256(tot, s_w, total);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = cbase + w * (64 * ITEMS) + r * 64 + lane;
        if (idx < K) {
            const uint32_t d = digit_of<KT, VIEW>(key[r], zmin, dbits, shift, dmask);
            const uint32_t pos = s_lstart[d] + s_whist[w][d] + rank[r];
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();
    const uint32_t nvalid = min((uint32_t)CHUNK, K - cbase);
    if constexpr (!EF) {
        for (uint32_t j = t; j < nvalid; j += 256) {
            const KT k = s_keys[j];
            const uint32_t d = digit_of<KT, VIEW>(k, zmin, dbits, shift, dmask);
            const uint32_t dst = s_gbase[d] + (j - s_lstart[d]);
            kout[dst] = k;
            vout[dst] = s_vals[j];
        }
    } else {
        // dst grows with j (the digit runs are laid out in digit order), so each emission
        // chunk present in a wave is a run of its lanes: from one prefix sum over the wave,
        // the run's last lane adds the inclusive sum and its first lane subtracts the
        // exclusive one (integer adds: the order of the atomics does not matter)
        for (uint32_t j0 = 0; j0 < nvalid; j0 += 256) {
            const uint32_t j = j0 + t;
            const bool ok = j < nvalid;
            uint32_t cid = 0xffffffffu, c = 0u;
            if (ok) {
                const KT k = s_keys[j];
                const uint32_t d = digit_of<KT, VIEW>(k, zmin, dbits, shift, dmask);
                const uint32_t dst = s_gbase[d] + (j - s_lstart[d]);
                kout[dst] = k;
                const uint32_t v = s_vals[j];
                vout[dst] = v;
                const uint2 r = ef.rect[v];
                if (dst < ef.srect_cap) ef.srect[dst] = r;
                c = rect_count(r);
                cid = dst / (uint32_t)kEmitChunk;
            }
            const uint32_t inc = wave_incl_scan(c);
            const uint32_t prev = __shfl_up(cid, 1, 64), next = __shfl_down(cid, 1, 64);
            if (ok && (lane == 63 || next != cid)) atomicAdd(ef.esum + cid, inc);
            if (ok && lane > 0 && prev != cid) atomicAdd(ef.esum + cid, c - inc);
        }
    }
}

// ---------------------------------------------------------------------------
// Host side: sort K (key, value) pairs across the two buffers over `total_bits`
// significant bits (passes of equal width, <= 8 bits each). Returns 1 if the result
// is in the alternate buffers (kb/vb), 0 if in ka/va. `ghist` holds 8 x 256 words
// (each pass's digit totals); `cnt` 256 x ceil(K / 4096) words of scratch.
// ---------------------------------------------------------------------------
int sort_passes(int total_bits) { return (total_bits + 7) / 8; }

// keys per thread of a pass over K keys: long chunks (long contiguous output runs) when
// there are enough keys to fill the GPU with them, shorter ones otherwise
static int sort_items(uint32_t K) { return K >= (1u << 22) ? 16 : (K >= (1u << 20) ? 8 : 4); }

// Words of the digit-count matrix any sort of at most K_max keys needs: chunks of the
// shortest length (1,024 keys), whatever length a sort takes or is given.
size_t sort_count_words(uint64_t K_max) {
    const uint64_t chunks = (K_max + 1023) / 1024;
    return 256 * (size_t)(chunks > 0 ? chunks : 1);
}

// The first pass of a sort whose digit counts the key emission writes (KeyCount): the
// sort then runs with chunks of 2,048 keys (kKeyCountItems per thread).
constexpr int kKeyCountItems = 8;
static_assert(256u * kKeyCountItems == kEmitKeys, "a counted chunk is one emission block");
KeyCount key_sort_first_count(uint32_t *cnt, uint32_t K_max, int total_bits) {
    if (total_bits <= 0) return KeyCount{nullptr, 0u, 0};   // one tile: no pass to count for
    const int passes = sort_passes(total_bits);
    const int per = (total_bits + passes - 1) / passes;
    const uint32_t chunk = 256u * (uint32_t)kKeyCountItems;
    return KeyCount{cnt, (K_max + chunk - 1) / chunk, per < total_bits ? per : total_bits};
}

template <typename KT, int VIEW>
static int radix_sort(KT *ka, uint32_t *va, KT *kb, uint32_t *vb, uint32_t K, uint32_t zmin, int dbits, int total_bits,
                      uint32_t *ghist, uint32_t *cnt, hipStream_t st, const uint32_t *dyn_count = nullptr,
                      const uint32_t *dyn_zmin = nullptr, const EmitFold *ef = nullptr, int first_shift = 0,
                      bool first_counted = false, bool spec = false) {
    if (K == 0 || total_bits == 0) return 0;   // K is the count, or its upper bound with dyn_count
    const int passes = sort_passes(total_bits);
    const int per = (total_bits + passes - 1) / passes;
    uint32_t bits = 0;
    int rem = total_bits;
    for (int p = 0; p < passes; ++p) {
        const int nb = rem < per ? rem : per;
        bits |= (uint32_t)nb << (4 * p);
        rem -= nb;
    }
    // first_counted: the first pass's counts are in cnt already (KeyCount), in its chunks
    const int items = first_counted ? kKeyCountItems : sort_items(K);
    const uint32_t chunk_keys = 256u * (uint32_t)items;
    const uint32_t chunks = (K + chunk_keys - 1) / chunk_keys;
    const EmitFold none{nullptr, nullptr, nullptr, 0u};
    int alt = 0, shift = first_shift;
    for (int p = 0; p < passes; ++p) {
        const int nb = (bits >> (4 * p)) & 15;
        const KT *kin = alt ? kb : ka;
        const uint32_t *vin = alt ? vb : va;
        KT *kout = alt ? ka : kb;
        uint32_t *vout = alt ? va : vb;
        uint32_t *tot = ghist + 256 * p;
        const bool fold = ef && p == passes - 1;
#define RECOGS_PASS(IT)                                                                                                    \
    if (p > 0 || !first_counted)                                                                                           \
        hipLaunchKernelGGL((k_radix_up<KT, VIEW, IT>), dim3(chunks), dim3(256), 0, st, kin, K, zmin, dbits, shift, nb,     \
                           cnt, chunks, dyn_count, dyn_zmin, (int)spec);                                                   \
    hipLaunchKernelGGL(k_radix_rowscan, dim3(1u << nb), dim3(256), 0, st, cnt, chunks, chunk_keys, tot, K, dyn_count);     \
    if (fold)                                                                                                              \
        hipLaunchKernelGGL((k_radix_down<KT, VIEW, IT, true>), dim3(chunks), dim3(256), 0, st, kin, vin, kout, vout, K,    \
                           zmin, dbits, shift, nb, cnt, tot, chunks, dyn_count, dyn_zmin, *ef, (int)spec);                 \
    else                                                                                                                   \
        hipLaunchKernelGGL((k_radix_down<KT, VIEW, IT, false>), dim3(chunks), dim3(256), 0, st, kin, vin, kout, vout, K,   \
                           zmin, dbits, shift, nb, cnt, tot, chunks, dyn_count, dyn_zmin, none, (int)spec);
        if (items == 16) { RECOGS_PASS(16) }
        else if (items == 8) { RECOGS_PASS(8) }
        else { RECOGS_PASS(4) }
#undef RECOGS_PASS
        alt ^= 1;
        shift += nb;
    }
    return alt;
}

// One row scan of a digit-count matrix [2^nbits][chunks] (K keys, chunk_keys per chunk).
void launch_rowscan(uint32_t *cnt, uint32_t chunks, uint32_t chunk_keys, uint32_t *tot, uint32_t K, int nbits,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_radix_rowscan, dim3(1u << nbits), dim3(256), 0, st, cnt, chunks, chunk_keys, tot, K, nullptr);
}

int radix_sort_tile_depth64(uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb, uint32_t K, uint32_t zmin, int dbits,
                            int total_bits, uint32_t *ghist, uint32_t *cnt, hipStream_t st) {
    return radix_sort<uint64_t, KV_TILE_DEPTH>(ka, va, kb, vb, K, zmin, dbits, total_bits, ghist, cnt, st);
}

// ef (optional): the depth order's last pass also does the emission fold.
// first_counted: the key emission wrote the first pass's counts (key_sort_first_count).
int radix_sort_u32(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t K, uint32_t sub, int total_bits,
                   uint32_t *ghist, uint32_t *cnt, hipStream_t st, const EmitFold *ef, bool first_counted) {
    return radix_sort<uint32_t, KV_SUB>(ka, va, kb, vb, K, sub, 0, total_bits, ghist, cnt, st, nullptr, nullptr, ef, 0,
                                        first_counted);
}

// The same with the count and the subtracted minimum read from device memory; K_max
// bounds the count (sizes the grids and the count matrix). The digits start at bit
// first_shift of the key (bits below it already ordered by an earlier pass). spec: the
// count is expected near K_max (the workgroups past it then load their chunk for
// nothing), and the chunks are loaded before it arrives.
int radix_sort_u32_dyn(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t K_max, const uint32_t *dyn_count,
                       const uint32_t *dyn_sub, int total_bits, uint32_t *ghist, uint32_t *cnt, hipStream_t st,
                       const EmitFold *ef, int first_shift, bool first_counted, bool spec) {
    return radix_sort<uint32_t, KV_SUB>(ka, va, kb, vb, K_max, 0u, 0, total_bits, ghist, cnt, st, dyn_count, dyn_sub, ef,
                                        first_shift, first_counted, spec);
}

}  // namespace recogs
