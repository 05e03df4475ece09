// Device radix sort of the 64-bit (tile, depth) keys with 32-bit values.
//
// Stable LSD sort with 8-bit digits over only the significant bits: the digits are
// taken from the view  (tile << dbits) | (depth_bits - min_depth_bits),  whose order
// equals the order of the stored key (tile << 32) | depth_bits for the keys of one
// render, and which needs ceil(log2 tiles) + dbits bits instead of 64.
//
// One histogram pass counts the digits of every pass at once; then each pass is a
// single kernel ("onesweep"): a workgroup takes a chunk of 4,096 keys from an atomic
// ticket, ranks them stably per digit with wave ballots (64-lane match masks built
// from 8 ballots, rank = popcount of the lower lanes), publishes its per-digit counts
// and resolves its global offsets by decoupled look-back over earlier chunks, then
// stages the chunk through LDS in digit order so global writes are contiguous runs.
#include "recogs_internal.hpp"

namespace recogs {

__device__ __forceinline__ uint32_t digit_of(uint64_t key, uint32_t zmin, int dbits, int shift) {
    return (uint32_t)(sort_view(key, zmin, dbits) >> shift) & 255u;
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

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ keys, uint32_t K, uint32_t zmin,
                                                    int dbits, int passes, uint32_t *__restrict__ ghist) {
    __shared__ uint32_t h[kMaxPasses][256];
    for (int i = threadIdx.x; i < kMaxPasses * 256; i += 256) (&h[0][0])[i] = 0;
    __syncthreads();
    for (uint32_t k = blockIdx.x * 256 + threadIdx.x; k < K; k += gridDim.x * 256) {
        const uint64_t x = sort_view(keys[k], zmin, dbits);
        for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(uint32_t)(x >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int p = 0; p < passes; ++p) {
        const uint32_t v = h[p][threadIdx.x];
        if (v) atomicAdd(&ghist[p * 256 + threadIdx.x], v);
    }
}

__global__ __launch_bounds__(256) void k_radix_pass(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint32_t K,
                                                    uint32_t zmin, int dbits, int shift,
                                                    const uint32_t *__restrict__ ghist, uint32_t *__restrict__ status,
                                                    uint32_t *__restrict__ ticket) {
    __shared__ uint32_t s_whist[4][256];   // per-wave digit counts, then per-wave digit prefix
    __shared__ uint32_t s_gbase[256];      // global position of this chunk's first key of each digit
    __shared__ uint32_t s_lstart[256];     // position in the LDS stage of each digit
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_chunk;
    __shared__ uint64_t s_keys[kSortChunk];
    __shared__ uint32_t s_vals[kSortChunk];

    const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
    if (t == 0) s_chunk = atomicAdd(ticket, 1u);
    for (int i = t; i < 4 * 256; i += 256) (&s_whist[0][0])[i] = 0;
    __syncthreads();
    const uint32_t chunk = s_chunk;
    const uint32_t cbase = chunk * (uint32_t)kSortChunk;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems], rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t idx = cbase + w * (64 * kSortItems) + r * 64 + lane;
        const bool valid = idx < K;
        key[r] = valid ? kin[idx] : 0ull;
        val[r] = valid ? vin[idx] : 0u;
    }
    // stable rank within the wave, round by round
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t idx = cbase + w * (64 * kSortItems) + r * 64 + lane;
        const bool valid = idx < K;
        const uint32_t d = digit_of(key[r], zmin, dbits, shift);
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
    // decoupled look-back over earlier chunks for digit t
    uint32_t excl = 0;
    if (chunk == 0) {
        __hip_atomic_store(&status[t], kRFlagInc | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(&status[chunk * 256 + t], kRFlagAgg | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // windowed look-back: kLookback predecessors loaded at once, consumed in order
        // until an inclusive prefix is found; a not-yet-published entry ends the window
        int64_t j = (int64_t)chunk - 1;
        while (true) {
            uint32_t s[kLookback];
#pragma unroll
            for (int k = 0; k < kLookback; ++k)
                s[k] = (j - k >= 0) ? __hip_atomic_load(&status[(j - k) * 256 + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : kRFlagInc;
            bool stop = false, done = false;
            int used = 0;
#pragma unroll
            for (int k = 0; k < kLookback; ++k) {
                if (!stop) {
                    const uint32_t f = s[k] & kRFlagMask;
                    if (f == 0) {
                        stop = true;
                    } else {
                        excl += s[k] & ~kRFlagMask;
                        ++used;
                        if (f == kRFlagInc) stop = done = true;
                    }
                }
            }
            if (done) break;
            j -= used;
            if (used == 0) __builtin_amdgcn_s_sleep(1);
        }
        __hip_atomic_store(&status[chunk * 256 + t], kRFlagInc | (excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t total;
    const uint32_t gpre = block_excl_scan256(ghist[t], s_w, total);
    s_gbase[t] = gpre + excl;
    s_lstart[t] = block_excl_scan256(tot, s_w, total);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t idx = cbase + w * (64 * kSortItems) + r * 64 + lane;
        if (idx < K) {
            const uint32_t d = digit_of(key[r], zmin, dbits, shift);
            const uint32_t pos = s_lstart[d] + s_whist[w][d] + rank[r];
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();
    const uint32_t nvalid = min((uint32_t)kSortChunk, K - cbase);
    for (uint32_t j = t; j < nvalid; j += 256) {
        const uint64_t k = s_keys[j];
        const uint32_t d = digit_of(k, zmin, dbits, shift);
        const uint32_t dst = s_gbase[d] + (j - s_lstart[d]);
        kout[dst] = k;
        vout[dst] = s_vals[j];
    }
}

// ---------------------------------------------------------------------------
void launch_radix_hist(const uint64_t *keys, uint32_t K, uint32_t zmin, int dbits, int passes, uint32_t *ghist,
                       hipStream_t st) {
    if (K == 0) return;
    uint32_t blocks = (K + 256 * 16 - 1) / (256 * 16);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_radix_hist, dim3(blocks), dim3(256), 0, st, keys, K, zmin, dbits, passes, ghist);
}

void launch_radix_pass(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout, uint32_t K, uint32_t zmin,
                       int dbits, int shift, const uint32_t *ghist, uint32_t *status, uint32_t *ticket, hipStream_t st) {
    if (K == 0) return;
    const uint32_t chunks = (K + kSortChunk - 1) / kSortChunk;
    hipLaunchKernelGGL(k_radix_pass, dim3(chunks), dim3(256), 0, st, kin, vin, kout, vout, K, zmin, dbits, shift, ghist,
                       status, ticket);
}

}  // namespace recogs
