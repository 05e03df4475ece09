// Device-side Adam update shared by the standalone optimiser step and the one fused
// into the SH gradient finish.
#pragma once
#include "recogs_internal.hpp"

namespace recogs {

// One Adam update of one value (the optimiser of the SH refit): the moments, then the
// parameter with the bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t. Shared by the
// standalone step and the one fused into the gradient finish, so both give the same bits.
struct AdamArgs {
    float lr, b1, b2, eps, c1, c2;
};
__device__ __forceinline__ void adam_update(float &p, float g, float &m, float &v, const AdamArgs &a) {
#pragma clang fp contract(off)   // the same operations wherever it is inlined
    m = a.b1 * m + (1.f - a.b1) * g;
    v = a.b2 * v + (1.f - a.b2) * (g * g);
    p -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
}

}  // namespace recogs
