// The emulated linear texture filter (Sec. 2: texel values at texel centres;
// Sec. 2.3: weights held in fixed point): per-axis weight rule and bilinear
// blend, shared by the texture-emulation and particle kernels.  Weight
// decisions are FP32 with every operation rounded as written.
#pragma once
#include "curves_impl.h"

namespace bzi {

// Fraction f in [0,1] held with F fractional bits: nearest with halves up
// (rnd 0) or truncation (rnd 1); F = 0 leaves it unrounded.
__device__ __forceinline__ float tx_round(float f, int F, int rnd) {
#pragma clang fp contract(off)
    if (F == 0) return f;
    const float sc = __builtin_ldexpf(f, F);
    const float q = rnd == 0 ? __builtin_floorf(sc + 0.5f) : __builtin_floorf(sc);
    return __builtin_ldexpf(q, -F);
}

// Weight of a two-texel axis sampled at parameter p in [0,1].
// Branch-free: clamping to [0, 1] before the rounding gives the edge weights
// 0 and 1 exactly (the rounding keeps both), and NaN passes through.
__device__ __forceinline__ float tx_axis_weight(float p, int F, int rnd) {
#pragma clang fp contract(off)
    const float x = 0.25f + 0.5f * p;  // normalised coordinate
    const float xb = 2.0f * x - 0.5f;  // texel-space position, centres at 0 and 1
    const float c = tx_round(__builtin_fminf(__builtin_fmaxf(xb, 0.0f), 1.0f), F, rnd);
    return xb != xb ? xb : c;
}

// Bilinear blend of a 2x2 layer L[row*2 + col]: x along a row, y across rows.
__device__ __forceinline__ float tx_bilinear(const float *L, float wx, float wy) {
    return lerp(lerp(L[0], L[1], wx), lerp(L[2], L[3], wx), wy);
}

}  // namespace bzi
