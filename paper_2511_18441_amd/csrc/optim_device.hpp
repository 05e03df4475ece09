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
__device__ __forceinline__ void adam_update(float &p, float g, float &m, float &v, const AdamArgs &a) {
#pragma clang fp contract(off)   // the same operations wherever it is inlined
    m = a.b1 * m + (1.f - a.b1) * g;
    v = a.b2 * v + (1.f - a.b2) * (g * g);
    // hardware square root and reciprocal (about 1 ulp each)
    p -= a.lr * (m * a.ic1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v * a.ic2) + a.eps);
}

}  // namespace recogs
