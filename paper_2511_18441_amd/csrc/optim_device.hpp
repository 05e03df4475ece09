// Device-side Adam update shared by the standalone optimiser step and the one fused
// into the SH gradient finish.
#pragma once
#include "recogs_internal.hpp"

namespace recogs {

// One Adam update of one value (the optimiser of the SH refit): the moments, then the
// parameter with the bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t. Shared by the
// standalone step and the one fused into the gradient finish, so both give the same bits.
struct AdamArgs {
    float lr, b1, b2, eps, ic1, ic2;   // ic1 = 1 / c1, ic2 = 1 / c2 (rounded from double on the host)
};
// Streaming (non-temporal) accesses for the optimiser's parameters and moments: each is
// read once and written once per step, so they are not kept in the caches (the fused
// SH step measured 0.892 -> 0.856 ms per refit step with them).
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ float4 ld_stream(const float4 *p) {
    const f32x4_t x = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t *>(p));
    return make_float4(x[0], x[1], x[2], x[3]);
}
__device__ __forceinline__ void st_stream(float4 *p, float4 v) {
    const f32x4_t x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<f32x4_t *>(p));
}

__device__ __forceinline__ void adam_update(float &p, float g, float &m, float &v, const AdamArgs &a) {
#pragma clang fp contract(off)   // the same operations wherever it is inlined
    m = a.b1 * m + (1.f - a.b1) * g;
    v = a.b2 * v + (1.f - a.b2) * (g * g);
    // hardware square root and reciprocal (about 1 ulp each)
    p -= a.lr * (m * a.ic1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v * a.ic2) + a.eps);
}

}  // namespace recogs
