// Shared device and host helpers of the gfx950 library (not used by the
// oracle).  Everything here is CDNA4-specific HIP: 64-wide wavefronts,
// FMA-based lerps, non-temporal streaming stores.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <type_traits>

#include "bz.h"

namespace bzi {

constexpr int kMaxDegree = 15;
constexpr int kMaxDim = 4;
constexpr int kBlock = 256;

// ------------------------------------------------------------------ host
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
inline hipStream_t as_stream(bz_stream s) { return reinterpret_cast<hipStream_t>(s); }

#define BZ_CHECK_HIP(expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return ::bzi::hip_fail(e_, #expr); \
    } while (0)

// Launch-error check after hipLaunchKernelGGL.
#define BZ_CHECK_LAUNCH(name)                                \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) return ::bzi::hip_fail(e_, name); \
    } while (0)

// Every extern "C" entry point body runs inside this wrapper.
template <typename F>
int guarded(const char *name, F &&f) {
    try {
        return f();
    } catch (...) {
        return fail(BZ_ERR_INTERNAL, "%s: unexpected C++ exception", name);
    }
}

inline bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
inline int dtype_size(int dt) { return dt == BZ_F32 ? 4 : (dt == BZ_F16 || dt == BZ_BF16) ? 2 : 0; }

// Granlund-Montgomery division of 32-bit unsigned values by a fixed d >= 1:
// q = (hi + ((n - hi) >> 1)) >> (s - 1), hi = mulhi(n, m), for d > 1.
struct FastDiv {
    uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f{d, 0, 0};
    if (d <= 1) return f;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.m = static_cast<uint32_t>(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    f.s = l;
    return f;
}

// ------------------------------------------------------------------ device
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    if (f.d <= 1) return n;
    const uint32_t hi = __umulhi(n, f.m);
    return (hi + ((n - hi) >> 1)) >> (f.s - 1);
}

// L(a,b,t) = (1-t)a + tb as two FMAs; exact at t = 0 and t = 1.
__device__ __forceinline__ float lerp(float a, float b, float t) { return __builtin_fmaf(t, b, __builtin_fmaf(-t, a, a)); }
__device__ __forceinline__ double lerp(double a, double b, double t) { return __builtin_fma(t, b, __builtin_fma(-t, a, a)); }

// Storage element -> FP32.
template <typename T>
__device__ __forceinline__ float to_f32(T v);
template <>
__device__ __forceinline__ float to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f32<_Float16>(_Float16 v) { return static_cast<float>(v); }
struct bf16_t {
    uint16_t bits;
};
template <>
__device__ __forceinline__ float to_f32<bf16_t>(bf16_t v) { return __uint_as_float(static_cast<uint32_t>(v.bits) << 16); }

constexpr float binomf(int n, int k) {
    if (k < 0 || k > n) return 0.0f;
    double r = 1.0;
    for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
    return static_cast<float>(r);
}

__device__ __forceinline__ void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }

}  // namespace bzi
