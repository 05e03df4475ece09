// Internal declarations of the HIP library behind include/recogs.h (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/recogs.h"

namespace recogs {

// ---------------------------------------------------------------------------
// Constants of the rasteriser the paper builds on (Sec. 4: the original Gaussian
// splatting rasteriser). The paper states none of them; these are that
// rasteriser's published conventions.
// ---------------------------------------------------------------------------
constexpr float kAlphaMax = 0.99f;               // alpha clamp
constexpr float kTMin = 1e-4f;                   // stop before transmittance drops below
constexpr float kDilation = 0.3f;                // px^2 added to the 2D covariance diagonal
constexpr float kFrustumClamp = 1.3f;            // Jacobian evaluated inside 1.3x the frustum
constexpr float kQSlack = 1.0f / 64.0f;          // extent level = 2 ln(255 sigma) + 1/64
constexpr float kLog2AlphaMin = -7.9943534368588578f;  // log2(1/255)
constexpr float kLog2e = 1.4426950408889634f;

// Real SH with the Condon-Shortley phase (eq. 2), values of the closed forms
// c/(k sqrt(pi)) used by the basis below.
constexpr float kSH0 = 0.28209479177387814f;     // 1/(2 sqrt pi)
constexpr float kSH1 = 0.48860251190291992f;     // sqrt3/(2 sqrt pi)
constexpr float kSH2a = 1.0925484305920792f;     // sqrt15/(2 sqrt pi)
constexpr float kSH2b = 0.31539156525252005f;    // sqrt5/(4 sqrt pi)
constexpr float kSH2c = 0.54627421529603959f;    // sqrt15/(4 sqrt pi)
constexpr float kSH3a = 0.59004358992664352f;    // sqrt(35/2)/(4 sqrt pi)
constexpr float kSH3b = 2.8906114426405538f;     // sqrt105/(2 sqrt pi)
constexpr float kSH3c = 0.45704579946446572f;    // sqrt(21/2)/(4 sqrt pi)
constexpr float kSH3d = 0.37317633259011546f;    // sqrt7/(4 sqrt pi)
constexpr float kSH3e = 1.4453057213202769f;     // sqrt105/(4 sqrt pi)

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// storage dtype access
// ---------------------------------------------------------------------------
template <int DT> struct Store;
template <> struct Store<RECOGS_F32> {
    static __device__ __forceinline__ float ld(const void *p, int64_t i) { return __builtin_nontemporal_load((const float *)p + i); }
    static __device__ __forceinline__ float ldc(const void *p, int64_t i) { return ((const float *)p)[i]; }
    static __device__ __forceinline__ void st(void *p, int64_t i, float v) { ((float *)p)[i] = v; }
    static constexpr int bytes = 4;
};
template <> struct Store<RECOGS_F16> {
    static __device__ __forceinline__ float ld(const void *p, int64_t i) { return (float)((const _Float16 *)p)[i]; }
    static __device__ __forceinline__ float ldc(const void *p, int64_t i) { return (float)((const _Float16 *)p)[i]; }
    static __device__ __forceinline__ void st(void *p, int64_t i, float v) { ((_Float16 *)p)[i] = (_Float16)v; }
    static constexpr int bytes = 2;
};
template <> struct Store<RECOGS_BF16> {
    static __device__ __forceinline__ float ld(const void *p, int64_t i) {
        return __uint_as_float((uint32_t)((const uint16_t *)p)[i] << 16);
    }
    static __device__ __forceinline__ float ldc(const void *p, int64_t i) { return ld(p, i); }
    static __device__ __forceinline__ void st(void *p, int64_t i, float v) {
        uint32_t u = __float_as_uint(v);
        uint16_t r;
        if ((u & 0x7fffffffu) > 0x7f800000u) r = 0x7fc0u;                      // NaN
        else r = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);           // nearest, ties to even
        ((uint16_t *)p)[i] = r;
    }
    static constexpr int bytes = 2;
};

// ---------------------------------------------------------------------------
// Compensated dot product (Ogita, Rump, Oishi 2005, "Dot2"): a0 b0 + a1 b1 + a2 b2 + c
// as accurate as if computed in twice the working precision, then rounded. Used for
// the camera-space position so the float32 depth that orders splats is (almost
// always) the correctly rounded exact depth.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dot3c(float a0, float b0, float a1, float b1, float a2, float b2, float c) {
#pragma clang fp contract(off)
    float p0 = a0 * b0, e0 = __builtin_fmaf(a0, b0, -p0);
    float p1 = a1 * b1, e1 = __builtin_fmaf(a1, b1, -p1);
    float p2 = a2 * b2, e2 = __builtin_fmaf(a2, b2, -p2);
    float s = p0 + p1, bb = s - p0, t1 = (p0 - (s - bb)) + (p1 - bb);
    float s2 = s + p2;
    bb = s2 - s;
    float t2 = (s - (s2 - bb)) + (p2 - bb);
    float s3 = s2 + c;
    bb = s3 - s2;
    float t3 = (s2 - (s3 - bb)) + (c - bb);
    return s3 + (((e0 + e1) + e2) + ((t1 + t2) + t3));
}

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------
// Orders LDS accesses among the lanes of one wave (a wave's LDS operations execute in
// issue order, so no wait is needed; the fences keep the compiler from moving memory
// operations across this point). Not a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }
// number of set bits of m in lanes below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T> __device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, 64); v = w < v ? w : v; }
    return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, 64); v = w > v ? w : v; }
    return v;
}
// Sum of a float over the first LANES lanes of the wave (64, or 32 / 16 when the
// workgroup is smaller than a wave: the lanes past it do not exist and hold no
// defined value) with DPP moves, each step one VALU add and no LDS crossbar: pairs,
// quads, half rows and rows by lane permutes (every lane then holds its 16-lane
// row's sum), then rows 0+1 and 2+3 by the row-15 broadcast and all four by the
// row-31 broadcast. The total ends in lane LANES-1 and is returned to every lane.
template <int CTRL, int ROW_MASK> __device__ __forceinline__ float dpp_add(float x) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
template <int LANES> __device__ __forceinline__ float wave_sum_dpp(float v) {
    static_assert(LANES == 64 || LANES == 32 || LANES == 16, "16, 32 or 64 lanes");
    v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);  // row_mirror
    if constexpr (LANES >= 32) v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    if constexpr (LANES == 64) v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), LANES - 1));
}

// Totals of four floats over the 64 lanes of a wave, transposed as they are summed so
// that each step moves one value per lane: lanes l and l^1 trade halves (even lanes keep
// a and b, odd lanes c and d), lanes l and l^2 trade again (one value per lane: a, c, b,
// d in lanes 4m + 0, 1, 2, 3), the four same-value lanes of a row by rotations of 4 and
// 8 lanes, then the rows by lane exchanges across 16 and 32. Lanes 0..3 return the
// totals of a, c, b, d (lane l holds value ((l & 1) << 1) | ((l >> 1) & 1) of the
// four). Every addition has a fixed place, so the totals are the same bits on every run.
// All 64 lanes must be active.
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_sum4(float a, float b, float c, float d) {
    const uint32_t l = lane_id();
    const bool o1 = (l & 1u) != 0, o2 = (l & 2u) != 0;
    float k0 = o1 ? c : a;
    float k1 = o1 ? d : b;
    k0 += dpp_mov<0xb1>(o1 ? a : c);   // quad_perm [1,0,3,2]
    k1 += dpp_mov<0xb1>(o1 ? b : d);
    float k = o2 ? k1 : k0;
    k += dpp_mov<0x4e>(o2 ? k0 : k1);  // quad_perm [2,3,0,1]
    k = dpp_add<0x124, 0xf>(k);        // row_ror:4
    k = dpp_add<0x128, 0xf>(k);        // row_ror:8
    k += __shfl_xor(k, 16, 64);
    k += __shfl_xor(k, 32, 64);
    return k;
}
// which of the four totals of wave_sum4 lane l (0..3) holds: 0 a, 1 b, 2 c, 3 d
__device__ __forceinline__ uint32_t sum4_part(uint32_t l) { return ((l & 1u) << 1) | ((l >> 1) & 1u); }

// inclusive prefix sum across the wave
template <typename T> __device__ __forceinline__ T wave_incl_scan(T v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T w = __shfl_up(v, o, 64);
        if (l >= (uint32_t)o) v += w;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Device-side views of the host structs
// ---------------------------------------------------------------------------
struct CamDev {
    float R[9], t[3];
    float fx, fy, cx, cy, znear;
    float limx, limy;       // 1.3 * (W/2)/fx, 1.3 * (H/2)/fy
    float campos[3];
    int32_t W, H, tw, th, tiles_x, tiles_y;
    int32_t extent_rule;    // 0: alpha >= 1/255 box; 1: the 3DGS rasteriser's square (recogs_render_opts)
};

struct SceneDev {
    int64_t n, stride;
    const float *means;
    const float *cov3d;
    const void *opacity;
    const void *sh;
};

struct RecolorDev {
    const uint8_t *mask;   // null = no fused recolour
    const float *M;
    const float *b;
};

// Workspace header words (u32), zeroed before each render.
enum : int {
    H_K_LO = 0, H_K_HI = 1,      // number of keys (64-bit)
    H_ZMIN = 2, H_ZMAX = 3,      // complement of min / max float32 depth bits among splats with keys
    H_V = 4,                     // number of Gaussians with keys
    H_KEFF = 5,                  // keys emitted: K if it fits the capacity, else 0
    H_OVERFLOW = 6,              // 1 when K exceeds the key capacity (nothing is emitted)
    H_ZMIN_RAW = 7,              // min depth bits (not complemented)
    H_QUEUE = 8,                 // work counter of the persistent blend
    H_ORDER_HIST = 16,           // 32 words: tiles per list-length class
    H_ORDER_CUR = 48,            // 32 words: scatter cursors of the length classes
    H_XQUEUE = 128,              // 8 x 32 words: per-XCD work counters of the persistent
                                 // region blend, one per 128-byte line
    H_WORDS = 384
};

// Per-view description of a batch (device memory): the view's scene, camera and
// fused recolour, its output, and where its pairs, preprocess blocks and tiles start
// in the batch's flattened index spaces.
struct ViewDev {
    SceneDev sc;
    CamDev cam;
    RecolorDev rc;
    float *image;
    float bg[3];
    uint32_t pair_base, blk_base, tile_base, ntiles;
};

// Outputs of the count scan's compaction for the tile-first key order (see launch_scan).
struct ScanEmit {
    const uint2 *rect;     // tile rectangles, index order
    uint2 *srect;          // compacted rectangles
    uint32_t *eoff;        // compacted key offsets
    uint32_t *efirst;      // owner of the first key of each emission block
};

// The count scan as the first pass of the depth sort (one view, no host read-back): the
// scan's chunks are that pass's chunks. k_scan_reduce counts the low 8 bits of the depth
// bits of each chunk's Gaussians with keys into dcnt[digit][chunk] (row stride: the
// chunk count), a row scan makes them the chunks' digit offsets and dtot the digit
// totals, and k_scan_down writes the chunk's (depth bits, index) pairs stably ordered
// by those 8 bits (keys, vals) instead of compacted in index order.
struct ScanSort {
    uint32_t *dcnt;
    uint32_t *dtot;
    uint32_t *keys;
    uint32_t *vals;
};

// The first pass of the key sort counted by the key emission: block b of the emission
// (its keys [2048 b, 2048 b + 2048)) is chunk b of that pass, whose digit counts (the
// low nbits of the tile id) it writes to cnt[digit * chunks + b].
struct KeyCount {
    uint32_t *cnt;   // null: not counted
    uint32_t chunks;
    int nbits;
};

constexpr uint32_t kEmitKeys = 2048;                 // keys per workgroup of k_emit_down (256 threads x 8)
constexpr int kScanItems = 16;                       // counts per thread of the scan
constexpr int kScanChunk = 256 * kScanItems;         // counts per scan workgroup
constexpr int kMaxPasses = 8;
constexpr int kEmitItems = 4;                        // depth-ordered Gaussians per thread (emission reduce / offsets)
constexpr int kEmitChunk = 256 * kEmitItems;         // depth-ordered Gaussians per emission workgroup

// Tiles of a packed tile rectangle (x0 | x1 << 16, y0 | y1 << 16): its key count.
__device__ __forceinline__ uint32_t rect_count(uint2 r) {
    return ((r.x >> 16) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.y & 0xffffu) + 1u);
}

// Work of the key emission's reduce pass, done by the last pass of the depth sort as it
// writes the depth order: each Gaussian's tile rectangle gathered in that order (srect)
// and the key count of every kEmitChunk consecutive depth-ordered Gaussians added into
// esum (zeroed beforehand).
struct EmitFold {
    const uint2 *rect;   // tile rectangles, indexed by the sort's values
    uint2 *srect;        // srect_cap entries (positions past it are not written)
    uint32_t *esum;
    uint32_t srect_cap;
};

// Per-Gaussian splat record for compositing: three float4
//   r0 = (u, v, ex, ey)   centre (pixels) and half-extents of the alpha >= 1/255 box
//   r1 = (A, B, C, o)     log2(alpha) = o + A dx^2 + B dx dy + C dy^2
//   r2 = (r, g, b, sigma) clamped colour, activated opacity
struct SplatRec { float4 r0, r1, r2; };

// ---------------------------------------------------------------------------
// Thread -> pixel map of the blend kernels (forward and backward): a workgroup of
// TW*TH/PPT threads covers one TW x TH tile, each thread PPT vertically stacked
// pixels. Where the tile allows it, each wave covers a compact 8 x (8 PPT) block
// ("wave region"); otherwise the wave region is the whole tile.
// ---------------------------------------------------------------------------
// Largest e(dx, dy) = A dx^2 + B dx dy + C dy^2 + o (r1 = (A, B, C, o), A, C < 0: a
// concave quadratic with its maximum o at the splat centre) over the rectangle
// [dx0, dx1] x [dy0, dy1]. With the centre outside, the maximiser lies on an edge that
// faces the centre: from any other boundary point the direction to the centre points
// into the rectangle, along which e increases. So only the vertical line nearest the
// centre (x = clamp(0, dx0, dx1)) and the horizontal one (y = clamp(0, dy0, dy1)) are
// searched; where the centre's x lies in [dx0, dx1] that line passes through the
// centre and, lying inside the rectangle, cannot exceed the maximum. On each line the
// 1-D maximum is at the clamped stationary point.
__device__ __forceinline__ float emax_rect(float4 r1, float dx0, float dx1, float dy0, float dy1) {
    if (dx0 <= 0.f && 0.f <= dx1 && dy0 <= 0.f && 0.f <= dy1) return r1.w;
    // 1 / (-2A), 1 / (-2C) to about 1 ulp: they only place the candidate maximiser on
    // its line, where an error of that size changes the value by far less than the margin
    const float ia = -0.5f * __builtin_amdgcn_rcpf(r1.x), ic = -0.5f * __builtin_amdgcn_rcpf(r1.z);
    // clamps as one median-of-three each (the bounds are ordered and nothing is NaN)
    const float X = __builtin_amdgcn_fmed3f(0.f, dx0, dx1), Y = __builtin_amdgcn_fmed3f(0.f, dy0, dy1);
    const float dy = __builtin_amdgcn_fmed3f(r1.y * X * ic, dy0, dy1);
    const float mx = (r1.x * X + r1.y * dy) * X + r1.z * dy * dy + r1.w;
    const float dx = __builtin_amdgcn_fmed3f(r1.y * Y * ia, dx0, dx1);
    const float my = (r1.z * Y + r1.y * dx) * Y + r1.x * dx * dx + r1.w;
    return fmaxf(mx, my);
}
// exponent margin of the region test (alpha 0.3 % below 1/255), far above the float32
// error of either evaluation: pixel offsets dx = (px + 1/2) - u are exact (Sterbenz)
// and the quadratic carries a few ulps
constexpr float kMaskMargin = 4e-3f;

// true when the splat can reach alpha >= 1/255 at a pixel centre of the rectangle
// [x0, x1] x [y0, y1] (absolute pixel-centre coordinates): its alpha >= 1/255 box
// (centre u, v, half-extents ex, ey in r0) meets the rectangle, and the largest
// base-2 exponent over it (exact maximum of the concave quadratic, see emax_rect) is
// at least the threshold less a margin far above float32 error. Skipping a region
// that fails is therefore exact.
__device__ __forceinline__ bool region_hit(float4 r0, float4 r1, float x0, float x1, float y0, float y1) {
    if (r0.x + r0.z < x0 || r0.x - r0.z > x1 || r0.y + r0.w < y0 || r0.y - r0.w > y1) return false;
    return emax_rect(r1, x0 - r0.x, x1 - r0.x, y0 - r0.y, y1 - r0.y) >= kLog2AlphaMin - kMaskMargin;
}

// Tile shapes whose blend runs in region form (one wave per 8 x 8*PPT block).
constexpr bool region_shape(int tw, int th, int ppt) { return tw % 8 == 0 && th % (8 * ppt) == 0; }

template <int TW, int TH, int PPT> struct TileMap {
    static constexpr int NT = TW * TH / PPT;
    static constexpr bool BLOCKS = (TW % 8 == 0) && ((TH / PPT) % 8 == 0);
    static constexpr int NW = BLOCKS ? NT / 64 : 1;
    static __device__ __forceinline__ void pixel(int t, int &lx, int &lrow) {
        if constexpr (BLOCKS) {
            const int w = t >> 6, l = t & 63;
            lx = (w % (TW / 8)) * 8 + (l & 7);
            lrow = (w / (TW / 8)) * 8 + (l >> 3);
        } else {
            lx = t % TW;
            lrow = t / TW;
        }
    }
    static __device__ __forceinline__ int wave(int t) { return BLOCKS ? (t >> 6) : 0; }
    // pixel-centre bounds of wave region w, relative to the tile origin
    static __device__ __forceinline__ void bounds(int w, float &x0, float &x1, float &y0, float &y1) {
        if constexpr (BLOCKS) {
            x0 = (float)((w % (TW / 8)) * 8) + 0.5f;
            x1 = x0 + 7.f;
            y0 = (float)((w / (TW / 8)) * 8 * PPT) + 0.5f;
            y1 = y0 + (float)(8 * PPT - 1);
        } else {
            x0 = 0.5f; x1 = (float)TW - 0.5f;
            y0 = 0.5f; y1 = (float)TH - 0.5f;
        }
    }
    // bit w set when region_hit holds for wave region w
    static __device__ __forceinline__ uint32_t wave_mask(float4 r0, float4 r1, float tx0, float ty0) {
        uint32_t m = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            float x0, x1, y0, y1;
            bounds(w, x0, x1, y0, y1);
            m |= (region_hit(r0, r1, tx0 + x0, tx0 + x1, ty0 + y0, ty0 + y1) ? 1u : 0u) << w;
        }
        return m;
    }
};

// log2(alpha) of a splat at pixel-centre offset (dx, dy) from its centre, with the same
// float32 operations in forward and backward (they must take identical threshold
// decisions). Factored so the PPT pixels of a thread, which share dx, share work:
//   e = dy (C dy + B dx) + (A dx^2 + o),   r1 = (A, B, C, o).
struct ExpRow { float ax, bx; };
__device__ __forceinline__ ExpRow exp_row(float4 r1, float dx) {
#pragma clang fp contract(off)
    ExpRow r;
    r.ax = __builtin_fmaf(r1.x * dx, dx, r1.w);
    r.bx = r1.y * dx;
    return r;
}
__device__ __forceinline__ float exp_at(ExpRow r, float4 r1, float dy) {
    return __builtin_fmaf(dy, __builtin_fmaf(r1.z, dy, r.bx), r.ax);
}

// key layout: (tile << 32) | float32 depth bits
__device__ __forceinline__ uint64_t sort_view(uint64_t key, uint32_t zmin, int dbits) {
    return ((key >> 32) << dbits) | (uint64_t)((uint32_t)key - zmin);
}

}  // namespace recogs
