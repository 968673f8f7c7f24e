// Curve evaluation kernels (integral and rational Bezier curves) for gfx950.
//
// One thread evaluates one (curve, parameter) query; query q = c*n_t + j,
// so a wavefront covers 64 consecutive parameters of one curve whenever
// n_t >= 64 and the control-point loads of the wave hit one or two cache
// lines.  Control points are held in registers, the evaluation form is
// unrolled at compile time for each degree 1..15 and dimension 1..4, and
// results go out with non-temporal stores to the planar out[dim][n*n_t].
#pragma once

#include "common.h"

namespace bzi {

enum Form { FORM_DC = 0, FORM_BERN = 1, FORM_SEILER = 2, FORM_SEILER_PRE = 3 };

// ---------------------------------------------------------------- forms
// de Casteljau (Sec. 2): d levels of lerps with the same t.
template <int D>
__device__ __forceinline__ float eval_dc(const float (&b)[D + 1], float t) {
    float p[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) p[i] = b[i];
#pragma unroll
    for (int lvl = 1; lvl <= D; ++lvl)
#pragma unroll
        for (int i = 0; i <= D - lvl; ++i) p[i] = lerp(p[i], p[i + 1], t);
    return p[0];
}

// Bernstein basis B_{i,D}(t) = C(D,i) t^i (1-t)^(D-i); exact 1/0 at the ends.
template <int D>
__device__ __forceinline__ void bernstein_basis(float t, float (&B)[D + 1]) {
    const float s = 1.0f - t;
    float tp[D + 1], sp[D + 1];
    tp[0] = 1.0f;
    sp[0] = 1.0f;
#pragma unroll
    for (int i = 1; i <= D; ++i) {
        tp[i] = tp[i - 1] * t;
        sp[i] = sp[i - 1] * s;
    }
#pragma unroll
    for (int i = 0; i <= D; ++i) B[i] = (binomf(D, i) * tp[i]) * sp[D - i];
}

template <int D>
__device__ __forceinline__ float dot_basis(const float (&B)[D + 1], const float (&b)[D + 1]) {
    float acc = B[0] * b[0];
#pragma unroll
    for (int i = 1; i <= D; ++i) acc = __builtin_fmaf(B[i], b[i], acc);
    return acc;
}

// Seiler difference terms by peeling (Sec. 3.1): Q - L(Q_0,Q_n,t) = st Q'
// with Q'_{i-1} = (Q_i - ((n-i)/n)Q_0 - (i/n)Q_n) * n(n-1)/(i(n-i)).
// Output order [b0, bd, d1, d_{d-1}, d2, d_{d-2}, ...].  The terms grow like
// C(d, d/2) and peeling cancels; the stand-alone conversion works in FP64
// (Acc = double) and rounds each term once.  Evaluations that derive the terms
// on the fly peel in FP32 at every degree: the evaluation multiplies term i by
// (st)^i <= 4^-i, which shrinks the peeling error of the large middle terms
// as much as it grows, so FP32 peeling ends within the error of FP64 peeling
// followed by the same FP32 evaluation (a few 1e-6 of the box at degree 15).
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int D, typename Acc = double, typename Out = float, typename In = float>
__device__ __forceinline__ void seiler_terms(const In (&b)[D + 1], Out (&sc)[D + 1]) {
    Acc Q[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) Q[i] = static_cast<Acc>(b[i]);
    sc[0] = static_cast<Out>(b[0]);
    sc[1] = static_cast<Out>(b[D]);
    int pos = 2;
#pragma unroll
    for (int n = D; n >= 2; n -= 2) {
        Acc R[D + 1];
#pragma unroll
        for (int i = 1; i <= n - 1; ++i) {
            const Acc a0 = static_cast<Acc>(n - i) / static_cast<Acc>(n);
            const Acc a1 = static_cast<Acc>(i) / static_cast<Acc>(n);
            const Acc sc_f = static_cast<Acc>(n * (n - 1)) / static_cast<Acc>(i * (n - i));
            const Acc r = Q[i] - fma_acc(a0, Q[0], a1 * Q[n]);
            R[i - 1] = r * sc_f;
        }
#pragma unroll
        for (int i = 0; i <= n - 2; ++i) Q[i] = R[i];
        sc[pos++] = static_cast<Out>(Q[0]);
        if (n - 2 > 0) sc[pos++] = static_cast<Out>(Q[n - 2]);
    }
}

// Seiler evaluation (Sec. 3.1), innermost level first:
// D = d_{d/2} (even d) or 0; D = L(d_i, d_{d-i}, t) + st D; C = L(b0,bd,t) + st D.
template <int D>
__device__ __forceinline__ float eval_seiler(const float (&sc)[D + 1], float t, float st) {
    constexpr int NP = (D - 1) / 2;
    float acc = (D % 2 == 0) ? sc[2 + 2 * NP] : 0.0f;
#pragma unroll
    for (int i = NP; i >= 1; --i) acc = __builtin_fmaf(st, acc, lerp(sc[2 * i], sc[2 * i + 1], t));
    return __builtin_fmaf(st, acc, lerp(sc[0], sc[1], t));
}

// Evaluate CH channels of degree-D data with form F.
template <int D, int CH, int F>
__device__ __forceinline__ void eval_channels(const float (&b)[CH][D + 1], float t, float (&r)[CH]) {
    if constexpr (F == FORM_DC) {
#pragma unroll
        for (int k = 0; k < CH; ++k) r[k] = eval_dc<D>(b[k], t);
    } else if constexpr (F == FORM_BERN) {
        float B[D + 1];
        bernstein_basis<D>(t, B);
#pragma unroll
        for (int k = 0; k < CH; ++k) r[k] = dot_basis<D>(B, b[k]);
    } else {
        const float st = (1.0f - t) * t;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if constexpr (F == FORM_SEILER) {
                float sc[D + 1];
                seiler_terms<D, float>(b[k], sc);
                r[k] = eval_seiler<D>(sc, t, st);
            } else {
                r[k] = eval_seiler<D>(b[k], t, st);
            }
        }
    }
}

// FP64 de Casteljau on homogeneous points, used to re-evaluate rational
// points whose weight sum is ill-conditioned in FP32.
template <int D, int DIM, typename T>
__device__ __attribute__((noinline)) void rational_fp64(const T *__restrict__ ctrl, const T *__restrict__ w, uint32_t c,
                                                        float t, float (&res)[DIM]) {
    const double td = static_cast<double>(t);
    double ww[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) ww[i] = static_cast<double>(to_f32<T>(w[static_cast<size_t>(c) * (D + 1) + i]));
    double W[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) W[i] = ww[i];
#pragma unroll
    for (int lvl = 1; lvl <= D; ++lvl)
#pragma unroll
        for (int i = 0; i <= D - lvl; ++i) W[i] = lerp(W[i], W[i + 1], td);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        double H[D + 1];
#pragma unroll
        for (int i = 0; i <= D; ++i)
            H[i] = ww[i] * static_cast<double>(to_f32<T>(ctrl[(static_cast<size_t>(c) * DIM + k) * (D + 1) + i]));
#pragma unroll
        for (int lvl = 1; lvl <= D; ++lvl)
#pragma unroll
            for (int i = 0; i <= D - lvl; ++i) H[i] = lerp(H[i], H[i + 1], td);
        res[k] = static_cast<float>(H[0] / W[0]);
    }
}

struct CurveArgs {
    const void *ctrl;      // storage of curves [c0, c0+n)
    const void *w;         // weights (rational) or nullptr
    const float *t;        // base of the full parameter array
    float *out;            // base of the full output array
    int64_t plane;         // total queries of the call (output plane stride)
    int64_t q0;            // first query of this launch (global index)
    int64_t c0;            // first curve of this launch
    uint32_t nq;           // queries in this launch
    FastDiv div_nt;        // division by n_t
    int per_object;        // t[n][n_t] vs t[n_t]
    float kappa;           // rational conditioning threshold (<= 0: off)
    uint32_t *n_fixed;     // nullable device counter
};

// UNI: n_t is a multiple of 64, so each wavefront evaluates one curve; its
// index is made wave-uniform and the control points come in through scalar
// loads instead of 64 identical vector loads.
template <int D, int DIM, int F, bool RAT, typename T, bool UNI>
__global__ __launch_bounds__(kBlock) void k_curves(CurveArgs a) {
    const uint32_t ql = blockIdx.x * kBlock + threadIdx.x;
    if (ql >= a.nq) return;
    uint32_t cl = fdiv(ql, a.div_nt);
    if constexpr (UNI) cl = __builtin_amdgcn_readfirstlane(cl);
    const uint32_t j = ql - cl * a.div_nt.d;
    const int64_t qg = a.q0 + ql;
    const float t = a.per_object ? a.t[qg] : a.t[j];

    constexpr int CH = DIM + (RAT ? 1 : 0);
    const T *__restrict__ P = static_cast<const T *>(a.ctrl) + static_cast<size_t>(cl) * DIM * (D + 1);
    float b[CH][D + 1];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i <= D; ++i) b[k][i] = to_f32<T>(P[k * (D + 1) + i]);

    float r[CH];
    if constexpr (!RAT) {
        eval_channels<D, CH, F>(b, t, r);
#pragma unroll
        for (int k = 0; k < DIM; ++k) st_stream(a.out + k * a.plane + qg, r[k]);
    } else {
        const T *__restrict__ Wp = static_cast<const T *>(a.w) + static_cast<size_t>(cl) * (D + 1);
        bool allpos = true;
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            const float wi = to_f32<T>(Wp[i]);
            allpos = allpos && (wi > 0.0f);
            b[DIM][i] = wi;
#pragma unroll
            for (int k = 0; k < DIM; ++k) b[k][i] *= wi;
        }
        eval_channels<D, CH, F>(b, t, r);
        const float W = r[DIM];
        bool fix = false;
        if (a.kappa > 0.0f && !(allpos && W > 0.0f && W < __builtin_inff())) {
            float aw[1][D + 1];
#pragma unroll
            for (int i = 0; i <= D; ++i) aw[0][i] = __builtin_fabsf(b[DIM][i]);
            float A[1];
            eval_channels<D, 1, F>(aw, t, A);
            fix = (t == t) && !(A[0] <= a.kappa * __builtin_fabsf(W));
        }
        float res[DIM];
        if (fix) {
            rational_fp64<D, DIM, T>(static_cast<const T *>(a.ctrl), static_cast<const T *>(a.w), cl, t, res);
        } else {
#pragma unroll
            for (int k = 0; k < DIM; ++k) res[k] = r[k] / W;
        }
        if (a.n_fixed) {
            const uint64_t m = __ballot(fix);
            if (m != 0 && __lane_id() == static_cast<unsigned>(__ffsll(static_cast<long long>(m)) - 1))
                atomicAdd(a.n_fixed, static_cast<uint32_t>(__popcll(m)));
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) st_stream(a.out + k * a.plane + qg, res[k]);
    }
}

// Seiler terms per (curve, coordinate): one thread per pair.
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void k_to_seiler(const T *__restrict__ ctrl, float *__restrict__ seiler, uint32_t n_rows) {
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_rows) return;
    float b[D + 1], sc[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) b[i] = to_f32<T>(ctrl[static_cast<size_t>(r) * (D + 1) + i]);
    seiler_terms<D>(b, sc);
#pragma unroll
    for (int i = 0; i <= D; ++i) seiler[static_cast<size_t>(r) * (D + 1) + i] = sc[i];
}

// ---------------------------------------------------------------- host
template <int F, bool RAT, typename T, int D, bool UNI>
int launch_curves_du(int dim, const CurveArgs &a, hipStream_t s) {
    const uint32_t blocks = (a.nq + kBlock - 1) / kBlock;
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_curves<D, 1, F, RAT, T, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_curves<D, 2, F, RAT, T, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_curves<D, 3, F, RAT, T, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_curves<D, 4, F, RAT, T, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: return fail(BZ_ERR_SHAPE, "dim %d out of range", dim);
    }
    BZ_CHECK_LAUNCH("k_curves");
    return BZ_OK;
}

template <int F, bool RAT, typename T, int D>
int launch_curves_d(int dim, const CurveArgs &a, hipStream_t s) {
    if (a.div_nt.d % 64 == 0) return launch_curves_du<F, RAT, T, D, true>(dim, a, s);
    return launch_curves_du<F, RAT, T, D, false>(dim, a, s);
}

// Launch one chunk of curve queries for form F (rational when RAT) with
// control points stored as T; explicitly instantiated per form in its own
// translation unit so the 15 x 4 specialisations compile in parallel.
template <int F, bool RAT, typename T>
int launch_curves_t(int degree, int dim, const CurveArgs &a, hipStream_t s) {
    switch (degree) {
        case 1: return launch_curves_d<F, RAT, T, 1>(dim, a, s);
        case 2: return launch_curves_d<F, RAT, T, 2>(dim, a, s);
        case 3: return launch_curves_d<F, RAT, T, 3>(dim, a, s);
        case 4: return launch_curves_d<F, RAT, T, 4>(dim, a, s);
        case 5: return launch_curves_d<F, RAT, T, 5>(dim, a, s);
        case 6: return launch_curves_d<F, RAT, T, 6>(dim, a, s);
        case 7: return launch_curves_d<F, RAT, T, 7>(dim, a, s);
        case 8: return launch_curves_d<F, RAT, T, 8>(dim, a, s);
        case 9: return launch_curves_d<F, RAT, T, 9>(dim, a, s);
        case 10: return launch_curves_d<F, RAT, T, 10>(dim, a, s);
        case 11: return launch_curves_d<F, RAT, T, 11>(dim, a, s);
        case 12: return launch_curves_d<F, RAT, T, 12>(dim, a, s);
        case 13: return launch_curves_d<F, RAT, T, 13>(dim, a, s);
        case 14: return launch_curves_d<F, RAT, T, 14>(dim, a, s);
        case 15: return launch_curves_d<F, RAT, T, 15>(dim, a, s);
        default: return fail(BZ_ERR_SHAPE, "degree %d out of range", degree);
    }
}

}  // namespace bzi
