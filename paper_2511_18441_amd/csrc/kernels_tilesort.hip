// Tile-first key order: after a stable sort of the index-ordered keys by tile id, each
// tile's list holds its Gaussians in index order; sorting each list stably by depth
// gives the (tile, depth, index) order of the blend. Tile lists are short next to the
// whole key set (at 1080p with 32x32 tiles about 1,650 keys on average and 6,300 at
// most for a million Gaussians), so each is sorted by one workgroup:
//   - lists of at most kTsCap keys in LDS: an LSD radix sort over the depth bits above
//     the frame's minimum, keys held in registers (a wave owns consecutive keys), ranks
//     within the wave from ballot match masks (one ballot per digit bit), digit starts
//     from per-wave histograms, one scatter into LDS per pass;
//   - longer lists (dense views of large scenes) by the same workgroup in chunks of
//     kTsCap, each pass a histogram over the list, then the chunks in order ranked and
//     scattered to global scratch, ping-ponging with the list itself.
// The sort replaces a global depth sort of every Gaussian with keys plus an emission in
// depth order: one launch instead of a dozen, and each list is read through one CU.
#include "recogs_internal.hpp"

namespace recogs {

// Two workgroup shapes by list length (each launch skips the tiles of the other):
//   4 waves, 16 keys per thread:  lists of up to 4,096 keys (most tiles);
//   8 waves, 16 keys per thread:  up to 8,192 keys in LDS, longer ones through memory.
// The LDS a shape needs sets how many of its workgroups a CU holds: the short lists get
// four concurrent workgroups per CU instead of waiting for the 64 KB of the larger shape.
// (A one-wave shape with 32 keys per lane for lists up to 2,048 keys measured slower.)
template <int NT, int IT>
struct TsShared {
    static constexpr int CAP = NT * IT;
    uint32_t k[CAP];
    uint32_t v[CAP];
    uint32_t wh[NT / 64][256];    // per-wave digit counts, then the wave's offset within each digit
    uint32_t dstart[256];         // exclusive start of each digit among this round's keys
    uint32_t tot[256];            // digit totals (the chunk's, for the global form)
    uint32_t gb[256];             // global form: where the chunk's first key of each digit goes
    uint32_t w4[NT / 64];
};

// exclusive scan over the NT threads of one value each; every thread receives its prefix
template <int NT>
__device__ __forceinline__ uint32_t ts_excl_scan(uint32_t x, uint32_t *w4, uint32_t &total) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(x);
    if constexpr (NT == 64) {
        total = __shfl(inc, 63, 64);
        return inc - x;
    } else {
        if (lane == 63) w4[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
        total = 0;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) {
            const uint32_t y = w4[k];
            if (k < (int)w) pre += y;
            total += y;
        }
        __syncthreads();
        return pre + inc - x;
    }
}

// index of round r of this thread among the chunk's keys (wave w owns 64 R consecutive keys)
__device__ __forceinline__ uint32_t ts_idx(int R, int r) {
    return (threadIdx.x >> 6) * 64u * (uint32_t)R + (uint32_t)r * 64u + lane_id();
}

// Stable ranking of up to CAP keys held in registers: round r of a thread holds key
// ts_idx(R, r), the first `len` keys valid. On return pos[r] is the key's position in
// digit order (stable) among the `len` keys, sh.dstart[d] the start of digit d and
// sh.tot[d] its count. Digits are (key >> shift) & (2^nb - 1), nb <= 8.
template <int NT, int IT>
__device__ __forceinline__ void ts_rank(const uint32_t (&key)[IT], uint32_t (&pos)[IT], int R, uint32_t len, int shift,
                                        int nb, TsShared<NT, IT> &sh) {
    constexpr int NW = NT / 64;
    constexpr int DPT = NT >= 256 ? 1 : 256 / NT;   // digits per thread in the digit phase
    const uint32_t t = threadIdx.x, w = t >> 6;
    const uint32_t dmask = (1u << nb) - 1u;
    for (uint32_t i = t; i < NW * 256; i += NT) (&sh.wh[0][0])[i] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        if (r >= R) continue;   // uniform: the loop stays fully unrolled
        const bool valid = ts_idx(R, r) < len;
        const uint32_t d = (key[r] >> shift) & dmask;
        uint64_t m = wave_ballot(valid);
        for (int b = 0; b < nb; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = wave_ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = rank_below(m);
        uint32_t prior = 0;
        if (valid) prior = sh.wh[w][d];
        pos[r] = prior + below;
        if (valid && below == 0) sh.wh[w][d] = prior + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // per digit (thread t: digits DPT t .. DPT t + DPT - 1): offsets of the waves within
    // it and its total; then the digit starts by a scan over the threads
    uint32_t dt[DPT], sum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const uint32_t d = t * DPT + j;
        uint32_t c = 0;
        if (d < 256) {
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t x = sh.wh[ww][d];
                sh.wh[ww][d] = c;
                c += x;
            }
        }
        dt[j] = c;
        sum += c;
    }
    uint32_t all;
    uint32_t ds = ts_excl_scan<NT>(sum, sh.w4, all);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const uint32_t d = t * DPT + j;
        if (d < 256) {
            sh.dstart[d] = ds;
            sh.tot[d] = dt[j];
        }
        ds += dt[j];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IT; ++r) {
        if (r >= R) continue;   // uniform: the loop stays fully unrolled
        if (ts_idx(R, r) < len) {
            const uint32_t d = (key[r] >> shift) & dmask;
            pos[r] += sh.dstart[d] + sh.wh[w][d];
        }
    }
}

// Sorts each tile's list vals[first, last) with lo < last - first <= hi by the depth bits
// zbits[val] - zmin (stable, so equal depths keep index order). Depth bit range from the
// header (the count scan's minimum and maximum). Lists above the shape's LDS capacity
// (the largest shape only) go through the scratch sk / sv (same indexing as vals).
template <int NT, int IT>
__global__ __launch_bounds__(NT) void k_tile_depth_sort(const uint2 *__restrict__ ranges, uint32_t *vals,
                                                        const uint32_t *__restrict__ zbits,
                                                        const uint32_t *__restrict__ hdr, uint32_t *sk, uint32_t *sv,
                                                        uint32_t lo, uint32_t hi) {
    constexpr int CAP = NT * IT;
    __shared__ TsShared<NT, IT> sh;
    const uint2 rg = ranges[blockIdx.x];
    const uint32_t len = rg.y - rg.x;
    if (rg.y <= rg.x + 1u || len <= lo || len > hi) return;
    const uint32_t zmin = hdr[H_ZMIN_RAW], zspan = hdr[H_ZMAX] - zmin;
    int dbits = 0;
    while (dbits < 32 && (zspan >> dbits) != 0u) ++dbits;
    if (dbits == 0) return;   // one depth: index order is the order
    const int passes = (dbits + 7) / 8, per = (dbits + passes - 1) / passes;
    const uint32_t t = threadIdx.x;
    uint32_t *list = vals + rg.x;
    uint32_t key[IT], val[IT], pos[IT];

    if (len <= (uint32_t)CAP) {
        const int R = (int)((len + NT - 1) / NT);
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            if (r >= R) continue;   // uniform: the loop stays fully unrolled
            const uint32_t idx = ts_idx(R, r);
            val[r] = idx < len ? list[idx] : 0u;
            key[r] = idx < len ? zbits[val[r]] - zmin : 0u;
        }
        int shift = 0;
        for (int p = 0; p < passes; ++p) {
            const int nb = dbits - shift < per ? dbits - shift : per;
            ts_rank<NT, IT>(key, pos, R, len, shift, nb, sh);
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                if (r >= R) continue;   // uniform: the loop stays fully unrolled
                if (ts_idx(R, r) < len) {
                    sh.k[pos[r]] = key[r];
                    sh.v[pos[r]] = val[r];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                if (r >= R) continue;   // uniform: the loop stays fully unrolled
                const uint32_t idx = ts_idx(R, r);
                if (idx < len) {
                    key[r] = sh.k[idx];
                    val[r] = sh.v[idx];
                }
            }
            __syncthreads();   // sh is rewritten by the next pass
            shift += nb;
        }
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            if (r >= R) continue;   // uniform: the loop stays fully unrolled
            const uint32_t idx = ts_idx(R, r);
            if (idx < len) list[idx] = val[r];
        }
        return;
    }
    if constexpr (NT == 512) {
        // long list: passes over global memory, chunks of CAP in order, between the list
        // (values only: keys recomputed from zbits) and the scratch (keys and values)
        uint32_t *xk = sk + rg.x, *xv = sv + rg.x;
        bool from_list = true;
        int shift = 0;
        for (int p = 0; p < passes; ++p) {
            const int nb = dbits - shift < per ? dbits - shift : per;
            const uint32_t dmask = (1u << nb) - 1u;
            const uint32_t *src_v = from_list ? list : xv;
            // digit starts over the whole list
            if (t < 256) sh.tot[t] = 0;
            __syncthreads();
            for (uint32_t i = t; i < len; i += NT) {
                const uint32_t k = from_list ? zbits[src_v[i]] - zmin : xk[i];
                atomicAdd(&sh.tot[(k >> shift) & dmask], 1u);
            }
            __syncthreads();
            uint32_t all;
            uint32_t gbase = ts_excl_scan<NT>(t < 256 ? sh.tot[t] : 0u, sh.w4, all);   // thread d: digit d's next slot
            for (uint32_t c0 = 0; c0 < len; c0 += CAP) {
                const uint32_t clen = len - c0 < (uint32_t)CAP ? len - c0 : (uint32_t)CAP;
                const int R = (int)((clen + NT - 1) / NT);
#pragma unroll
                for (int r = 0; r < IT; ++r) {
                    if (r >= R) continue;   // uniform: the loop stays fully unrolled
                    const uint32_t idx = ts_idx(R, r);
                    val[r] = idx < clen ? src_v[c0 + idx] : 0u;
                    key[r] = idx < clen ? (from_list ? zbits[val[r]] - zmin : xk[c0 + idx]) : 0u;
                }
                ts_rank<NT, IT>(key, pos, R, clen, shift, nb, sh);
                if (t < 256) sh.gb[t] = gbase;
                __syncthreads();
#pragma unroll
                for (int r = 0; r < IT; ++r) {
                    if (r >= R) continue;   // uniform: the loop stays fully unrolled
                    if (ts_idx(R, r) < clen) {
                        const uint32_t d = (key[r] >> shift) & dmask;
                        const uint32_t dst = sh.gb[d] + (pos[r] - sh.dstart[d]);
                        if (from_list) {
                            xk[dst] = key[r];
                            xv[dst] = val[r];
                        } else {
                            list[dst] = val[r];
                        }
                    }
                }
                if (t < 256) gbase += sh.tot[t];
                __syncthreads();   // sh is rewritten by the next chunk
            }
            // this pass's outputs are read by every thread of the next one (one workgroup:
            // its stores are visible to it after the barrier)
            __threadfence_block();
            __syncthreads();
            from_list = !from_list;
            shift += nb;
        }
        if (!from_list) {   // the last pass wrote the scratch
            for (uint32_t i = t; i < len; i += NT) list[i] = xv[i];
        }
    }
}

// One launch per workgroup shape, each over every tile (a workgroup whose tile is not
// of its length class returns at once). sk / sv: scratch of at least the key count (the
// key sort's free buffers).
void launch_tile_depth_sort(const uint2 *ranges, uint32_t ntiles, uint32_t *vals, const uint32_t *zbits,
                            const uint32_t *hdr, uint32_t *sk, uint32_t *sv, hipStream_t st) {
    if (ntiles == 0) return;
    constexpr uint32_t c4 = 256 * 16;
    hipLaunchKernelGGL((k_tile_depth_sort<256, 16>), dim3(ntiles), dim3(256), 0, st, ranges, vals, zbits, hdr, sk, sv, 1u,
                       c4);
    hipLaunchKernelGGL((k_tile_depth_sort<512, 16>), dim3(ntiles), dim3(512), 0, st, ranges, vals, zbits, hdr, sk, sv, c4,
                       0xffffffffu);
}

}  // namespace recogs
