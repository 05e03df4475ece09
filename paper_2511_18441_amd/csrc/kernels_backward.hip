// Backward of the blend and of the colour / fused-recolour step (eq. 8 restricted to
// opacity, SH DC and the recolour matrix), and the L2 loss gradient.
//
// Per-tile recomputation: a workgroup replays its tile's sorted list front to back
// for each pixel, over the entries the forward processed (it stored their count),
// taking the same threshold decisions with the same float32 arithmetic. With the
// forward output y, the colour behind splat i is R_i = y - A_i - rgb_i alpha_i T_i
// (A_i: colour accumulated in front of it), and
//   dL/drgb_i   += alpha_i T_i g
//   dL/dalpha_i  = g . (rgb_i T_i - R_i / (1 - alpha_i))
//   dL/dsigma_i += dL/dalpha_i G_i(p)   (0 where alpha is clamped at 0.99)
// No float atomics: every (Gaussian, tile) pair owns one slot of a per-key gradient
// array, Gaussian-contiguous (slot = the Gaussian's key offset from the count scan +
// the tile's row-major rank in its tile rectangle). A splat's four sums over one wave
// come from one transposed reduction (wave_sum4), the waves of the tile add theirs in
// LDS, and one float4 store
// per (splat, tile) writes the slot; k_grad_finish then sums each Gaussian's slots in
// a fixed order, so the gradients are deterministic.
#include "optim_device.hpp"
#include "render_device.hpp"

namespace recogs {

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st);

template <int TW, int TH, int PPT>
__global__ __launch_bounds__(TW *TH / PPT) void k_blend_bwd(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
                                                           const SplatRec *__restrict__ rec, const uint2 *__restrict__ rect,
                                                           const uint32_t *__restrict__ koff, int W, int H, int tiles_x,
                                                           const float *__restrict__ image, const float *__restrict__ dldy,
                                                           const uint32_t *__restrict__ nproc,
                                                           float4 *__restrict__ gk) {
#pragma clang fp contract(off)
    using Map = TileMap<TW, TH, PPT>;
    constexpr int NT = Map::NT;
    constexpr int NW = (NT + 63) / 64;
    // records staged per batch: 256 where the workgroup has a thread for each (half the
    // barriers of 128; the LDS, 44 KB, still fits the three workgroups per CU that the
    // registers allow)
    constexpr int BATCH = NT >= 256 ? 256 : kBlendBatch;
    struct Stage { BlendRec r[BATCH]; };
    __shared__ Stage sm;   // BlendRec.pad holds the (Gaussian, tile) slot, rgb.w the opacity
    __shared__ float4 s_acc[NW][BATCH];
    const int tile = blockIdx.x;
    const uint32_t tcx = (uint32_t)(tile % tiles_x), tcy = (uint32_t)(tile / tiles_x);
    const int tx0 = (int)tcx * TW, ty0 = (int)tcy * TH;
    const int t = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(Map::wave(t));
    const int wv = t >> 6;   // this thread's wave in the workgroup (slot of s_acc)
    int lx, lrow;
    Map::pixel(t, lx, lrow);
    const int px = tx0 + lx;
    const float pxc = (float)px + 0.5f;
    // Per pixel only g-weighted sums are carried: with s_i = g . rgb_i and
    // Gr = g . (y - A) (the g-weighted colour not yet accounted for, starting at g . y),
    // g . R_i = Gr - alpha_i T_i s_i, so dL/dalpha_i = T_i s_i - (Gr - alpha_i T_i s_i) / (1 - alpha_i)
    // and Gr decreases by alpha_i T_i s_i after splat i.
    float pyc[PPT], T[PPT], Gr[PPT], g0[PPT], g1[PPT], g2[PPT];
    uint32_t np[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = ty0 + lrow * PPT + j;
        pyc[j] = (float)py + 0.5f;
        T[j] = 1.f;
        np[j] = 0;
        Gr[j] = g0[j] = g1[j] = g2[j] = 0.f;
        if (px < W && py < H) {
            const int64_t p = (int64_t)py * W + px;
            np[j] = nproc[p];
            g0[j] = dldy[p * 3]; g1[j] = dldy[p * 3 + 1]; g2[j] = dldy[p * 3 + 2];
            Gr[j] = g0[j] * image[p * 3] + g1[j] * image[p * 3 + 1] + g2[j] * image[p * 3 + 2];
        }
    }
    uint32_t npmax = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) npmax = max(npmax, np[j]);
    // with full waves, the wave's largest replay count: entries at or past it are left
    // out of the wave's bit sets, so the walk needs no test per entry
    constexpr int L = NT < 64 ? NT : 64;
    uint32_t npw = 0;
    if constexpr (L == 64) npw = wave_max(npmax);

    const uint2 rg = ranges[tile];
    // With a thread per staged record (NT >= BATCH), the records of batch b + 1, their
    // tile rectangles and key offsets are loaded into registers while batch b is
    // replayed, so the dependent list -> record loads are off the critical path.
    constexpr bool PIPE = NT >= BATCH;
    float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0, f2 = f0;
    uint2 frc = make_uint2(0u, 0u);
    uint32_t fko = 0;
    auto fetch = [&](uint32_t start) {
        const uint32_t k = start + (uint32_t)t;
        if (t < BATCH && k < rg.y) {
            const uint32_t gid = vals[k];
            const SplatRec *sp = rec + gid;
            f0 = sp->r0; f1 = sp->r1; f2 = sp->r2;
            frc = rect[gid];
            fko = koff[gid];
        }
    };
    auto stage = [&](int q, float4 r0, float4 r1, float4 r2, uint2 rc, uint32_t ko) {
        const uint32_t rx0 = rc.x & 0xffffu, rx1 = rc.x >> 16, ry0 = rc.y & 0xffffu;
        BlendRec b;
        b.uv = make_float2(r0.x, r0.y);
        b.mask = Map::wave_mask(r0, r1, (float)tx0, (float)ty0);
        b.pad = ko + (tcy - ry0) * (rx1 - rx0 + 1) + (tcx - rx0);
        b.r1 = r1;
        b.rgb = r2;
        sm.r[q] = b;
    };
    if constexpr (PIPE) fetch(rg.x);
    for (uint32_t start = rg.x; start < rg.y; start += BATCH) {
        if (__syncthreads_and(start - rg.x >= npmax)) break;
        if constexpr (PIPE) {
            if (t < BATCH) {
                if (start + (uint32_t)t < rg.y) stage(t, f0, f1, f2, frc, fko);
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) s_acc[ww][t] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
            for (int q = t; q < BATCH; q += NT) {
                const uint32_t k = start + q;
                if (k < rg.y) {
                    const uint32_t gid = vals[k];
                    const SplatRec sp = rec[gid];
                    stage(q, sp.r0, sp.r1, sp.r2, rect[gid], koff[gid]);
                }
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) s_acc[ww][q] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        __syncthreads();
        if constexpr (PIPE) fetch(start + BATCH);
        const int nb = (int)min((uint32_t)BATCH, rg.y - start);
        // the batch's records this wave takes (scalar bit sets), walked in order while
        // some pixel of the wave still replays
        uint64_t todo[BATCH / 64];
#pragma unroll
        for (int c = 0; c < BATCH / 64; ++c) {
            todo[c] = 0;
#pragma unroll
            for (int sub = 0; sub < 64 / L; ++sub) {
                const int q = c * 64 + sub * L + (int)lane_id();
                const bool live = L < 64 || start + (uint32_t)q - rg.x < npw;
                todo[c] |= wave_ballot(q < nb && live && ((sm.r[q].mask >> w) & 1u)) << (sub * L);
            }
        }
        bool quit = false;
#pragma unroll
        for (int c = 0; c < BATCH / 64; ++c) {
            uint64_t mm = todo[c];
            while (mm && !quit) {
                const int q = c * 64 + (int)__builtin_ctzll(mm);
                mm &= mm - 1;
                const uint32_t krel = start + q - rg.x;
                if constexpr (L < 64) {
                    if (!wave_ballot(krel < npmax)) {
                        quit = true;
                        break;
                    }
                }
                const float4 *br = reinterpret_cast<const float4 *>(&sm.r[q]);
                const float4 h = br[0], r1 = br[1], r2 = br[2];
                const float2 uv = make_float2(h.x, h.y);
                // 1 / sigma to about 1 ulp: it only scales this splat's opacity gradient
                float inv_sigma = __builtin_amdgcn_rcpf(r2.w);
                // here, not sunk into the branch below: the record's last 16 bytes then
                // come in one LDS read with the rest, not a second read and wait
                asm volatile("" : "+v"(inv_sigma));
                const ExpRow er = exp_row(r1, pxc - uv.x);
                float ds, dr, dg, db;
                bool any = false;
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    // the forward's decisions, replayed with its arithmetic: entries up to
                    // the pixel's last blended one, alpha at or above 1/255
                    const float e = exp_at(er, r1, pyc[j] - uv.y);
                    const bool act = krel < np[j] && !(e < kLog2AlphaMin);
                    any = any || act;
                    const float araw = __builtin_amdgcn_exp2f(e);
                    const float a = fminf(kAlphaMax, araw);
                    const float wgt = act ? a * T[j] : 0.f;
                    const float sg = g0[j] * r2.x + g1[j] * r2.y + g2[j] * r2.z;
                    const float ws = wgt * sg;
                    // (finite: 1 - a >= 0.01) computed on every lane, selected by a factor
                    const float dal = T[j] * sg - (Gr[j] - ws) * __builtin_amdgcn_rcpf(1.f - a);
                    const float vs = dal * ((act && araw < kAlphaMax) ? araw * inv_sigma : 0.f);
                    if (j == 0) {   // (no adds of zero: x + 0 is not folded, for the sign of zero)
                        dr = wgt * g0[j]; dg = wgt * g1[j]; db = wgt * g2[j]; ds = vs;
                    } else {
                        dr += wgt * g0[j]; dg += wgt * g1[j]; db += wgt * g2[j]; ds += vs;
                    }
                    Gr[j] -= ws;
                    T[j] = act ? __builtin_fmaf(-a, T[j], T[j]) : T[j];
                }
                if (wave_ballot(any)) {
                    if constexpr (L == 64) {
                        const float tot = wave_sum4(ds, dr, dg, db);
                        const uint32_t l = lane_id();
                        if (l < 4) ((float *)&s_acc[wv][q])[sum4_part(l)] = tot;
                    } else {
                        ds = wave_sum_dpp<L>(ds); dr = wave_sum_dpp<L>(dr); dg = wave_sum_dpp<L>(dg); db = wave_sum_dpp<L>(db);
                        if (lane_id() == 0) s_acc[wv][q] = make_float4(ds, dr, dg, db);
                    }
                }
            }
        }
        __syncthreads();
        for (int q = t; q < nb; q += NT) {
            float4 v = s_acc[0][q];
#pragma unroll
            for (int ww = 1; ww < NW; ++ww) {
                const float4 x = s_acc[ww][q];
                v.x += x.x; v.y += x.y; v.z += x.z; v.w += x.w;
            }
            if (v.x != 0.f || v.y != 0.f || v.z != 0.f || v.w != 0.f) gk[sm.r[q].pad] = v;
        }
    }
}

// Block form of the backward: a workgroup per tile with one wave per 8 x 8*PPT pixel
// block (the forward's region form, its blocks in the same order). Each wave walks the
// tile's list on its own, 64 entries at a time, one per lane: the entries region_hit
// admits for its block are compacted into the wave's LDS in list order and replayed,
// with the arithmetic of k_blend_bwd, until every pixel of the block has passed its
// last blended entry. No barrier couples the waves while they replay.
// Gradients stay deterministic without float atomics: a wave writes its sums, one float4
// per entry with an active pixel, densely in list order from sub[b * cap + first] (b: the
// block, first: the tile's first list position), and per chunk of 64 positions the word
// fw[b * fstride + first / 64 + tile + chunk] = (bit set per position written, count
// written before the chunk) (the tile term keeps the words of neighbouring tiles apart);
// the words of chunks past the block's replay count are never read. After the one
// barrier the workgroup adds, for each position of the tile, the written block sums in
// block order and writes the (Gaussian, tile) slot of k_blend_bwd, so k_grad_finish reads
// the same slots in either form.
template <int TW, int TH, int PPT>
__global__ __launch_bounds__((TW / 8) * (TH / (8 * PPT)) * 64) void k_blend_bwd_blocks(
    const uint2 *__restrict__ ranges, const uint32_t *__restrict__ vals, const SplatRec *__restrict__ rec,
    const uint2 *__restrict__ rect, const uint32_t *__restrict__ koff, int W, int H, int tiles_x,
    const float *__restrict__ image, const float *__restrict__ dldy, const uint32_t *__restrict__ nproc,
    float4 *__restrict__ sub, ulonglong2 *__restrict__ fw, uint32_t cap, uint32_t fstride, float4 *__restrict__ gk) {
#pragma clang fp contract(off)
    constexpr uint32_t NR = (TW / 8) * (TH / (8 * PPT));
    __shared__ float4 sm[NR][64][3];   // per wave: (u, v, -, 1-based position), conic row, colour and sigma
    __shared__ uint32_t s_npl[NR];
    const uint32_t tile = blockIdx.x;
    const uint32_t region = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t tcx = tile % (uint32_t)tiles_x, tcy = tile / (uint32_t)tiles_x;
    const int l = (int)lane_id();
    const int bx = (int)tcx * TW + (int)(region % (TW / 8)) * 8;
    const int by = (int)tcy * TH + (int)(region / (TW / 8)) * 8 * PPT;
    const int px = bx + (l & 7);
    const float pxc = (float)px + 0.5f;
    const float x0 = (float)bx + 0.5f, x1 = x0 + 7.f;
    const float y0 = (float)by + 0.5f, y1 = y0 + (float)(8 * PPT - 1);
    float pyc[PPT], T[PPT], Gr[PPT], g0[PPT], g1[PPT], g2[PPT];
    uint32_t np[PPT], npl = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int py = by + (l >> 3) * PPT + j;
        pyc[j] = (float)py + 0.5f;
        T[j] = 1.f;
        np[j] = 0;
        Gr[j] = g0[j] = g1[j] = g2[j] = 0.f;
        if (px < W && py < H) {
            const int64_t p = (int64_t)py * W + px;
            np[j] = nproc[p];
            g0[j] = dldy[p * 3]; g1[j] = dldy[p * 3 + 1]; g2[j] = dldy[p * 3 + 2];
            Gr[j] = g0[j] * image[p * 3] + g1[j] * image[p * 3 + 1] + g2[j] * image[p * 3 + 2];
        }
        npl = max(npl, np[j]);
    }
    // the block's largest replay count: entries past it are read by no pixel here
    npl = wave_max(npl);
    const uint2 rg = ranges[tile];
    float4 *wsub = sub + (size_t)region * cap + rg.x;
    ulonglong2 *wfw = fw + (size_t)region * fstride + (rg.x >> 6) + tile;
    uint32_t wcount = 0;   // sums written so far
    // software pipeline as in the forward: the records of chunk c are in registers while
    // chunk c - 1 is replayed, the list values of chunk c + 1 on their way
    float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0, p2 = p0;
    uint32_t vnext = 0;
    {
        const uint32_t k = rg.x + (uint32_t)l;
        if (k < rg.y) {
            const SplatRec *sp = rec + vals[k];
            p0 = sp->r0; p1 = sp->r1; p2 = sp->r2;
        }
        if (k + 64u < rg.y) vnext = vals[k + 64u];
    }
    for (uint32_t start = rg.x; start < rg.y && start - rg.x < npl; start += 64) {
        const uint32_t pos = start + 1u - rg.x + (uint32_t)l;
        const bool in = start + (uint32_t)l < rg.y;
        // replayed: admitted for the block and within its replay count (the admitted
        // entries are compacted in list order, so these are the first nh of them)
        const bool hit = in && region_hit(p0, p1, x0, x1, y0, y1) && pos <= npl;
        const uint64_t mm = wave_ballot(hit);
        const int nh = (int)__builtin_popcountll(mm);
        const uint32_t rank = rank_below(mm);
        if (hit) {
            sm[region][rank][0] = make_float4(p0.x, p0.y, 0.f, __uint_as_float(pos));
            sm[region][rank][1] = p1;
            sm[region][rank][2] = p2;
        }
        wave_sync();   // the lanes' LDS writes before any lane reads
        {
            const uint32_t k = start + 64u + (uint32_t)l;
            if (k < rg.y) {
                const SplatRec *sp = rec + vnext;
                p0 = sp->r0; p1 = sp->r1; p2 = sp->r2;
            }
            if (k + 64u < rg.y) vnext = vals[k + 64u];
        }
        uint64_t wrote = 0;   // bit q: compacted entry q had an active pixel here
        for (int q = 0; q < nh; ++q) {
            const float4 h = sm[region][q][0], r1 = sm[region][q][1], r2 = sm[region][q][2];
            const uint32_t krel = __float_as_uint(h.w);
            const float2 uv = make_float2(h.x, h.y);
            // 1 / sigma to about 1 ulp: it only scales this splat's opacity gradient
            const float inv_sigma = __builtin_amdgcn_rcpf(r2.w);
            const ExpRow er = exp_row(r1, pxc - uv.x);
            float ds, dr, dg, db;
            bool any = false;
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const float e = exp_at(er, r1, pyc[j] - uv.y);
                const bool act = krel <= np[j] && !(e < kLog2AlphaMin);
                any = any || act;
                const float araw = __builtin_amdgcn_exp2f(e);
                const float a = fminf(kAlphaMax, araw);
                const float wgt = act ? a * T[j] : 0.f;
                const float sg = g0[j] * r2.x + g1[j] * r2.y + g2[j] * r2.z;
                const float ws = wgt * sg;
                // (finite: 1 - a >= 0.01) computed on every lane, selected by a factor
                const float dal = T[j] * sg - (Gr[j] - ws) * __builtin_amdgcn_rcpf(1.f - a);
                const float vs = dal * ((act && araw < kAlphaMax) ? araw * inv_sigma : 0.f);
                if (j == 0) {   // (no adds of zero: x + 0 is not folded, for the sign of zero)
                    dr = wgt * g0[j]; dg = wgt * g1[j]; db = wgt * g2[j]; ds = vs;
                } else {
                    dr += wgt * g0[j]; dg += wgt * g1[j]; db += wgt * g2[j]; ds += vs;
                }
                Gr[j] -= ws;
                T[j] = act ? __builtin_fmaf(-a, T[j], T[j]) : T[j];
            }
            if (wave_ballot(any)) {
                const float tot = wave_sum4(ds, dr, dg, db);
                if (l < 4) ((float *)(wsub + wcount + __builtin_popcountll(wrote)))[sum4_part((uint32_t)l)] = tot;
                wrote |= 1ull << q;
            }
        }
        const uint64_t wm = wave_ballot(hit && ((wrote >> rank) & 1ull));
        if (l == 0) wfw[(start - rg.x) >> 6] = make_ulonglong2(wm, wcount);
        wcount += (uint32_t)__builtin_popcountll(wm);
        wave_sync();   // all reads of this chunk before the next chunk's writes
    }
    // wave w adds the chunks w, w + NR, ... of the tile's list, U at a time so that their
    // loads are in flight together. The slots of its first U chunks (gathers of the
    // Gaussians' rectangles and key offsets) are fetched before the barrier, while other
    // waves may still replay.
    const uint32_t L = rg.y - rg.x;
    const uint32_t nchunks = (L + 63u) >> 6;
    constexpr int U = NR >= 16 ? 2 : 4;
    uint32_t slot[U];
    auto slots = [&](uint32_t c0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = (c0 + (uint32_t)u * NR) * 64u + (uint32_t)l;
            slot[u] = 0;
            if (i < L) {
                const uint32_t gid = vals[rg.x + i];
                const uint2 rc = rect[gid];
                const uint32_t rx0 = rc.x & 0xffffu, rx1 = rc.x >> 16, ry0 = rc.y & 0xffffu;
                slot[u] = koff[gid] + (tcy - ry0) * (rx1 - rx0 + 1u) + (tcx - rx0);
            }
        }
    };
    slots(region);
    if (l == 0) s_npl[region] = npl;
    __syncthreads();   // every block's sums and flags, and the replay counts, before the adds
    const ulonglong2 *words = fw + (rg.x >> 6) + tile;
    const uint64_t below = (1ull << l) - 1ull;   // lanes under this one
    for (uint32_t c0 = region; c0 < nchunks; c0 += NR * U) {
        if (c0 != region) slots(c0);
        uint32_t fm[U], at[U][NR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t c = c0 + (uint32_t)u * NR;   // wave-uniform
            const uint32_t i = c * 64u + (uint32_t)l;
            fm[u] = 0;
#pragma unroll
            for (uint32_t r = 0; r < NR; ++r) {
                at[u][r] = 0;
                if (c < nchunks && c * 64u < s_npl[r]) {   // chunk walked by block r: its word was written
                    const ulonglong2 wd = words[(size_t)r * fstride + c];
                    fm[u] |= (i < s_npl[r] ? (uint32_t)(wd.x >> l) & 1u : 0u) << r;
                    at[u][r] = (uint32_t)wd.y + (uint32_t)__builtin_popcountll(wd.x & below);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if ((c0 + (uint32_t)u * NR) * 64u + (uint32_t)l >= L) continue;
            float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (uint32_t r = 0; r < NR; ++r) {
                if ((fm[u] >> r) & 1u) {
                    const float4 x = sub[(size_t)r * cap + rg.x + at[u][r]];
                    a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
                }
            }
            gk[slot[u]] = a;
        }
    }
}

// Per Gaussian: dL/dsigma, and the chain through the clamp and the fused recolour to
// the colour before them: gh = dL/drgb where the pre-clamp colour > 0, g = M^T gh for
// selected Gaussians (dL/dM += gh (f + 1/2)^T) and g = gh otherwise. The colour of
// eq. 2 is linear in the SH coefficients, so dL/dC_{k,c} = Y_k(d) g_c:
//   DEG < 0:  the DC term only, out[c][n] = Y00 g_c;
//   DEG >= 0: every coefficient, out[(k * 3 + c) * stride + i] = Y_k(d) g_c (the scene's
//             plane layout), d the view direction.
// dL/dM is reduced without atomics: each workgroup writes its 9 partial sums to
// part[block][9] and k_dm_reduce adds them in a fixed order (deterministic).
// ADAM (DEG >= 0): instead of writing dL/dSH, apply one Adam step with it to the SH
// planes psh in place (moments am, av, same layout): the gradient never goes to memory.
// prev + x for the accumulate mode, never fused with the multiply that produced x: an
// accumulated gradient is then the float32 sum of the single-view gradients
__device__ __forceinline__ float acc_add(float prev, float x) {
#pragma clang fp contract(off)
    return prev + x;
}

template <int DEG, bool ADAM>
__global__ __launch_bounds__(256) void k_grad_finish(const float4 *__restrict__ gk, const uint32_t *__restrict__ koff,
                                                     const float4 *__restrict__ bwd, const uint32_t *__restrict__ count,
                                                     int64_t n, const float *__restrict__ M, float *__restrict__ dop,
                                                     float *__restrict__ out, float *__restrict__ part,
                                                     const float *__restrict__ means, int64_t stride, CamDev cam,
                                                     int acc, float *__restrict__ psh, float *__restrict__ am,
                                                     float *__restrict__ av, AdamArgs aa, uint64_t slots,
                                                     const uint32_t *overflow) {
    constexpr uint32_t kPiece = 256;   // slots staged per wave and round
    __shared__ float s_dm[4][9];
    __shared__ float4 s_slot[4][kPiece];
    const bool ovf = overflow && *overflow;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    bool sel = false;
    float gh[3] = {0.f, 0.f, 0.f}, f[3] = {0.f, 0.f, 0.f};
    // The Gaussian's (Gaussian, tile) slots [s0, s1), added in order. A render that
    // overflowed its key capacity (overflow flag set) has empty tile lists and no slot
    // written: nothing is read and the sums stay zero; slots (the gradient buffer's
    // capacity) bounds the reads in any case. The slots are Gaussian-major and the wave's
    // Gaussians consecutive, so the wave's slots are one run [lo, hi): it is read
    // coalesced into LDS, a piece at a time, and each lane adds its own from there.
    const uint32_t c = i < n ? count[i] : 0u;
    const uint32_t ko = i < n ? koff[i] : 0u;
    const bool use = !ovf && c > 0 && (uint64_t)ko + c <= slots;
    const uint32_t s0 = use ? ko : 0xffffffffu, s1 = use ? ko + c : 0u;
    const uint32_t lo = wave_min(s0), hi = wave_max(s1);
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t base = lo; base < hi; base += kPiece) {
        for (uint32_t j = lane; j < kPiece && base + j < hi; j += 64) s_slot[w][j] = gk[base + j];
        wave_sync();
        if (use) {
            const uint32_t k0 = s0 > base ? s0 : base, k1 = s1 < base + kPiece ? s1 : base + kPiece;
            for (uint32_t k = k0; k < k1; ++k) {
                const float4 x = s_slot[w][k - base];
                a.x += x.x; a.y += x.y; a.z += x.z; a.w += x.w;
            }
        }
        wave_sync();
    }
    if (i < n) {
        uint32_t flags = 0;
        if (use) {
            const float4 b = bwd[i];
            flags = __float_as_uint(b.w);
            f[0] = b.x; f[1] = b.y; f[2] = b.z;
        }
        gh[0] = (flags & 1u) ? a.y : 0.f;
        gh[1] = (flags & 2u) ? a.z : 0.f;
        gh[2] = (flags & 4u) ? a.w : 0.f;
        sel = (flags & 8u) != 0;
        dop[i] = acc ? acc_add(dop[i], a.x) : a.x;
        float g[3];
        if (sel) {
#pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = M[c] * gh[0] + M[3 + c] * gh[1] + M[6 + c] * gh[2];
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = gh[c];
        }
        if constexpr (DEG < 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float x = kSH0 * g[c];
                out[c * n + i] = acc ? acc_add(out[c * n + i], x) : x;
            }
        } else {
            constexpr int NC = (DEG + 1) * (DEG + 1);
            float Y[16];
            if (c > 0) {
                view_basis<DEG>(cam, means[i], means[stride + i], means[2 * stride + i], Y);
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) Y[k] = 0.f;
            }
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t o = (int64_t)(k * 3 + c) * stride + i;
                    if constexpr (ADAM) {
                        float pp = ld_stream(psh + o), mm = ld_stream(am + o), vv = ld_stream(av + o);
                        adam_update(pp, Y[k] * g[c], mm, vv, aa);
                        st_stream(am + o, mm);
                        st_stream(av + o, vv);
                        st_stream(psh + o, pp);
                    } else {
                        const float x = Y[k] * g[c];
                        out[o] = acc ? acc_add(out[o], x) : x;
                    }
                }
        }
    }
    if (!M) return;  // uniform: no recolour, no dL/dM
    if (wave_ballot(sel)) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float v = wave_sum(sel ? gh[r] * f[c] : 0.f);
                if (lane_id() == 0) s_dm[w][r * 3 + c] = v;
            }
    } else if (lane_id() < 9) {
        s_dm[w][lane_id()] = 0.f;
    }
    __syncthreads();
    if (threadIdx.x < 9)
        part[(size_t)blockIdx.x * 9 + threadIdx.x] =
            ((s_dm[0][threadIdx.x] + s_dm[1][threadIdx.x]) + s_dm[2][threadIdx.x]) + s_dm[3][threadIdx.x];
}

// dM[k] = sum over blocks of part[block][k] (added to dM[k] with acc), one workgroup,
// fixed summation order
__global__ __launch_bounds__(256) void k_dm_reduce(const float *__restrict__ part, uint32_t nblocks, float *__restrict__ dM,
                                                   int acc) {
    // thread t adds blocks t, t + 256, ... in order, all nine sums at once (independent
    // loads); then a fixed tree over lanes and waves: the order never depends on timing
    __shared__ float s_w[4][9];
    float v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = 0.f;
    for (uint32_t b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] += part[(size_t)b * 9 + k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float x = wave_sum(v[k]);
        if (lane_id() == 0) s_w[threadIdx.x >> 6][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const int k = threadIdx.x;
        const float v = ((s_w[0][k] + s_w[1][k]) + s_w[2][k]) + s_w[3][k];
        dM[k] = acc ? acc_add(dM[k], v) : v;
    }
}

// L2 loss: loss += scale sum (y - t)^2, dL/dy = 2 scale (y - t). With vec (all three
// arrays 16-byte aligned) each thread takes 4 consecutive elements per step with one
// 16-byte access per array; the remainder (or everything, without vec) one by one.
__global__ __launch_bounds__(1024) void k_loss_l2(const float *__restrict__ y, const float *__restrict__ tg, int64_t count,
                                                 float scale, float *__restrict__ dldy, float *__restrict__ loss, int vec) {
    __shared__ float s_w[16];
    float sum = 0.f;
    const int64_t n4 = vec ? count / 4 : 0;
    const float4 *y4 = reinterpret_cast<const float4 *>(y), *t4 = reinterpret_cast<const float4 *>(tg);
    float4 *d4 = reinterpret_cast<float4 *>(dldy);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto one = [&](const float4 a, const float4 b, int64_t i) {
        const float4 d = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
        d4[i] = make_float4(2.f * scale * d.x, 2.f * scale * d.y, 2.f * scale * d.z, 2.f * scale * d.w);
        sum += d.x * d.x + d.y * d.y + d.z * d.z + d.w * d.w;
    };
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {   // four groups' loads in flight
        float4 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { a[u] = y4[i + u * stride]; b[u] = t4[i + u * stride]; }
#pragma unroll
        for (int u = 0; u < 4; ++u) one(a[u], b[u], i + u * stride);
    }
    for (; i < n4; i += stride) one(y4[i], t4[i], i);
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const float d = y[i] - tg[i];
        dldy[i] = 2.f * scale * d;
        sum += d * d;
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float w = 0.f;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) w += s_w[k];   // the waves' sums in order
        atomicAdd(loss, scale * w);
    }
}

// ---------------------------------------------------------------------------
template <int TW, int TH, int PPT>
static void bwd_one(int ntiles, hipStream_t st, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec,
                    const uint2 *rect, const uint32_t *koff, int W, int H, int tiles_x, const float *image,
                    const float *dldy, const uint32_t *nproc, float4 *gk) {
    hipLaunchKernelGGL((k_blend_bwd<TW, TH, PPT>), dim3(ntiles), dim3(TW * TH / PPT), 0, st, ranges, vals, rec, rect, koff, W,
                       H, tiles_x, image, dldy, nproc, gk);
}

bool launch_blend_bwd(int tw, int th, int ppt, int ntiles, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec,
                      const uint2 *rect, const uint32_t *koff, int W, int H, int tiles_x, const float *image,
                      const float *dldy, const uint32_t *nproc, float4 *gk, hipStream_t st) {
#define RECOGS_BWD_CASE(A, B, P)                                                                                 \
    if (tw == A && th == B && ppt == P) {                                                                        \
        bwd_one<A, B, P>(ntiles, st, ranges, vals, rec, rect, koff, W, H, tiles_x, image, dldy, nproc, gk);      \
        return true;                                                                                             \
    }
    RECOGS_BWD_CASE(16, 16, 1) RECOGS_BWD_CASE(16, 16, 2) RECOGS_BWD_CASE(16, 16, 4)
    RECOGS_BWD_CASE(8, 8, 1) RECOGS_BWD_CASE(8, 8, 2) RECOGS_BWD_CASE(8, 8, 4)
    RECOGS_BWD_CASE(32, 8, 1) RECOGS_BWD_CASE(32, 8, 2) RECOGS_BWD_CASE(32, 8, 4)
    RECOGS_BWD_CASE(32, 16, 1) RECOGS_BWD_CASE(32, 16, 2) RECOGS_BWD_CASE(32, 16, 4)
    RECOGS_BWD_CASE(32, 32, 1) RECOGS_BWD_CASE(32, 32, 2) RECOGS_BWD_CASE(32, 32, 4)
#undef RECOGS_BWD_CASE
    return false;
}

// Block form of the backward (tile shapes with one wave per 8 x 8*PPT block): false when
// the shape has none. sub: nr * cap float4, fw: nr * fstride (bits, count) words (fstride >=
// cap / 64 + ntiles + 1); gk: the slots, all written.
template <int TW, int TH, int PPT>
static void bwd_blocks_one(int ntiles, hipStream_t st, const uint2 *ranges, const uint32_t *vals, const SplatRec *rec,
                           const uint2 *rect, const uint32_t *koff, int W, int H, int tiles_x, const float *image,
                           const float *dldy, const uint32_t *nproc, float4 *sub, ulonglong2 *fw, uint32_t cap,
                           uint32_t fstride, float4 *gk) {
    constexpr uint32_t NR = (TW / 8) * (TH / (8 * PPT));
    hipLaunchKernelGGL((k_blend_bwd_blocks<TW, TH, PPT>), dim3((unsigned)ntiles), dim3(NR * 64), 0, st, ranges, vals, rec,
                       rect, koff, W, H, tiles_x, image, dldy, nproc, sub, fw, cap, fstride, gk);
}

uint32_t bwd_blocks(int tw, int th, int ppt) { return region_shape(tw, th, ppt) ? (uint32_t)((tw / 8) * (th / (8 * ppt))) : 0u; }

bool launch_blend_bwd_blocks(int tw, int th, int ppt, int ntiles, const uint2 *ranges, const uint32_t *vals,
                             const SplatRec *rec, const uint2 *rect, const uint32_t *koff, int W, int H, int tiles_x,
                             const float *image, const float *dldy, const uint32_t *nproc, float4 *sub, ulonglong2 *fw,
                             uint32_t cap, uint32_t fstride, float4 *gk, hipStream_t st) {
#define RECOGS_BWDB_CASE(A, B, P)                                                                                   \
    if (tw == A && th == B && ppt == P) {                                                                           \
        bwd_blocks_one<A, B, P>(ntiles, st, ranges, vals, rec, rect, koff, W, H, tiles_x, image, dldy, nproc, sub, \
                                fw, cap, fstride, gk);                                                              \
        return true;                                                                                                \
    }
    RECOGS_BWDB_CASE(16, 16, 1) RECOGS_BWDB_CASE(16, 16, 2)
    RECOGS_BWDB_CASE(8, 8, 1)
    RECOGS_BWDB_CASE(32, 8, 1)
    RECOGS_BWDB_CASE(32, 16, 1) RECOGS_BWDB_CASE(32, 16, 2)
    RECOGS_BWDB_CASE(32, 32, 1) RECOGS_BWDB_CASE(32, 32, 2) RECOGS_BWDB_CASE(32, 32, 4)
#undef RECOGS_BWDB_CASE
    return false;
}

// part: (ceil(n / 256)) x 9 floats of scratch; dM is written whole (zeros without M or n).
// deg < 0: out = dL/dC0 [3][n]; deg 0..3: out = dL/dSH [3 (deg + 1)^2][stride], which needs
// the centres (means, plane stride) and the camera.
// acc: dop, out and dM are added to instead of written (a loss over several views).
// adam non-null (deg 0..3): one Adam step on psh / am / av instead of writing out.
void launch_grad_finish(const float4 *gk, const uint32_t *koff, const float4 *bwd, const uint32_t *count, int64_t n,
                        const float *M, float *dop, float *out, float *dM, float *part, int deg, const float *means,
                        int64_t stride, const CamDev &cam, int acc, hipStream_t st, float *psh, float *am, float *av,
                        const AdamArgs *adam, uint64_t slots, const uint32_t *overflow) {
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    const AdamArgs aa = adam ? *adam : AdamArgs{0.f, 0.f, 0.f, 1.f, 1.f, 1.f};
    if (n > 0) {
#define RECOGS_FIN(D, A)                                                                                              \
    hipLaunchKernelGGL((k_grad_finish<D, A>), dim3(blocks), dim3(256), 0, st, gk, koff, bwd, count, n, M, dop, out, part, \
                       means, stride, cam, acc, psh, am, av, aa, slots, overflow)
        if (adam) {
            switch (deg) {
            case 0: RECOGS_FIN(0, true); break;
            case 1: RECOGS_FIN(1, true); break;
            case 2: RECOGS_FIN(2, true); break;
            default: RECOGS_FIN(3, true); break;
            }
        } else {
            switch (deg) {
            case 0: RECOGS_FIN(0, false); break;
            case 1: RECOGS_FIN(1, false); break;
            case 2: RECOGS_FIN(2, false); break;
            case 3: RECOGS_FIN(3, false); break;
            default: RECOGS_FIN(-1, false); break;
            }
        }
#undef RECOGS_FIN
    }
    if (M && n > 0) hipLaunchKernelGGL(k_dm_reduce, dim3(1), dim3(256), 0, st, part, blocks, dM, acc);
    else if (!acc) launch_fill_u32((uint32_t *)dM, 0u, 9, st);
}

void launch_loss_l2(const float *y, const float *tg, int64_t count, float scale, float *dldy, float *loss, hipStream_t st) {
    if (count <= 0) return;
    // few workgroups (of 16 waves): each adds its partial sum with one same-address atomic
    int64_t blocks = (count + 1023) / 1024;
    if (blocks > 128) blocks = 128;
    const int vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(tg) | reinterpret_cast<uintptr_t>(dldy)) &
                     15u) == 0;
    hipLaunchKernelGGL(k_loss_l2, dim3((unsigned)blocks), dim3(1024), 0, st, y, tg, count, scale, dldy, loss, vec);
}

}  // namespace recogs
