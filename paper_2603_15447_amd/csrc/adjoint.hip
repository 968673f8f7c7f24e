// Adjoint of curve evaluation and a fused least-squares fitting step (loss,
// gradients through the hodograph, Adam) for gfx950.
//
// One wavefront per curve: the 64 lanes walk the curve's n_t parameters, each
// lane accumulating its share of dL/db (and dL/dw) in registers; a butterfly
// of cross-lane shuffles then sums the partials, so the per-curve reduction is
// deterministic and needs no atomics.  dL/dt is per query and is written by
// the lane that owns the query.
#include <cmath>
#include <vector>

#include "curves_impl.h"

namespace bzi {
namespace {

// Sum over the 64 lanes: a DPP butterfly inside each 16-lane row (swap
// neighbours, swap pairs, mirror the 8-lane halves, mirror the row) leaves
// every lane holding its row's sum; the four row sums are then read lane by
// lane.  The result is wave-uniform.  No LDS traffic.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror
    const int b = __builtin_bit_cast(int, v);
    return (__builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 0)) +
            __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 16))) +
           (__builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 32)) +
            __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 48)));
}

// Sums over each 32-lane half of the wavefront (two curves per wave): the
// same row butterfly, then rows 0+1 and rows 2+3.  Lanes get their half's sum.
__device__ __forceinline__ float half_sum(float v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    const int b = __builtin_bit_cast(int, v);
    const float lo = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 0)) +
                     __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 16));
    const float hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 32)) +
                     __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 48));
    return (threadIdx.x & 32) ? hi : lo;
}

// Exchange with lane ^ D inside each 32-lane half: DPP for D = 1, 2 (quad
// permutations), ds_swizzle in xor mode (and-mask 31) for D = 4..16.
template <int D>
__device__ __forceinline__ float xor_lane(float v) {
    if constexpr (D == 1) return dpp_mov<0xB1>(v);
    else if constexpr (D == 2) return dpp_mov<0x4E>(v);
    else return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), (D << 10) | 0x1F));
}

// Reduce-scatter over a 32-lane half: NV values per lane in, and lane l of
// the half leaves with the half's sum of value l mod NV (NV = 16 or 32).  At
// each exchange a lane keeps the half of its values selected by one bit of
// its index (most significant first) and adds its partner's copy of that
// half, so the work halves with every exchange.
template <int NV, int D = NV / 2>
__device__ __forceinline__ void reduce_scatter_level(float (&v)[NV], int sub) {
    if constexpr (D >= 1) {
        const bool hi = (sub & D) != 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float lo_v = v[j], hi_v = v[j + D];
            v[j] = (hi ? hi_v : lo_v) + xor_lane<D>(hi ? lo_v : hi_v);
        }
        reduce_scatter_level<NV, D / 2>(v, sub);
    }
}

template <int NV>
__device__ __forceinline__ float reduce_scatter32(float (&v)[NV], int sub) {
    reduce_scatter_level<NV>(v, sub);
    float r = v[0];
    if constexpr (NV == 16) r += xor_lane<16>(r);
    return r;
}

// Per-curve sums of the gradient partials gb[k][i], delivered to the lane
// that owns parameter sub = k*(D+1)+i (lanes past NP get unused values).
// Two curves per wavefront: reduce-scatter in each half; one curve: one
// wave sum per parameter.
template <int D, int DIM, int CPW>
__device__ __forceinline__ float reduce_grads(const float (&gb)[DIM][D + 1], int sub) {
    constexpr int NP = DIM * (D + 1);
    if constexpr (CPW == 2) {
        constexpr int NV = NP <= 16 ? 16 : 32;
        float v[NV];
#pragma unroll
        for (int e = 0; e < NV; ++e) v[e] = e < NP ? gb[e / (D + 1)][e % (D + 1)] : 0.0f;
        return reduce_scatter32<NV>(v, sub);
    } else {
        float mine = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int i = 0; i <= D; ++i) {
                const float v = wave_sum(gb[k][i]);
                if (sub == k * (D + 1) + i) mine = v;
            }
        return mine;
    }
}

struct AdjArgs {
    const float *ctrl;
    const float *w;
    const float *t;
    const float *gout;
    float *gctrl;
    float *gw;
    float *gt;
    int64_t n_curves;
    int64_t n_t;
    int64_t plane;
    int per_object;
};

// Per query: value C, derivative C' (hodograph), and the basis B.
template <int D, int DIM, bool RAT>
__device__ __forceinline__ void curve_and_derivative(const float (&b)[DIM][D + 1], const float (&wv)[D + 1], float t,
                                                     float (&B)[D + 1], float &W, float (&C)[DIM], float (&dC)[DIM]) {
    bernstein_basis<D>(t, B);
    float Bm[D];
    bernstein_basis<D - 1>(t, Bm);
    if constexpr (!RAT) {
        W = 1.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            C[k] = dot_basis<D>(B, b[k]);
            float d = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) d = __builtin_fmaf(b[k][i + 1] - b[k][i], Bm[i], d);
            dC[k] = static_cast<float>(D) * d;
        }
    } else {
        float wB[D + 1];
        W = 0.0f;
        float Wp = 0.0f;
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            wB[i] = wv[i] * B[i];
            W += wB[i];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) Wp = __builtin_fmaf(wv[i + 1] - wv[i], Bm[i], Wp);
        Wp *= static_cast<float>(D);
        const float iW = 1.0f / W;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const float H = dot_basis<D>(wB, b[k]);
            float Hp = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) Hp = __builtin_fmaf(wv[i + 1] * b[k][i + 1] - wv[i] * b[k][i], Bm[i], Hp);
            Hp *= static_cast<float>(D);
            C[k] = H * iW;
            dC[k] = (Hp - C[k] * Wp) * iW;
        }
    }
}

template <int D, int DIM, bool RAT>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t c = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (c >= a.n_curves) return;
    float b[DIM][D + 1], wv[D + 1];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i <= D; ++i) b[k][i] = a.ctrl[(c * DIM + k) * (D + 1) + i];
#pragma unroll
    for (int i = 0; i <= D; ++i) wv[i] = RAT ? a.w[c * (D + 1) + i] : 1.0f;
    float gb[DIM][D + 1] = {}, gwv[D + 1] = {};
    for (int64_t j = lane; j < a.n_t; j += 64) {
        const int64_t q = c * a.n_t + j;
        const float t = a.per_object ? a.t[q] : a.t[j];
        float B[D + 1], W, C[DIM], dC[DIM], g[DIM];
        curve_and_derivative<D, DIM, RAT>(b, wv, t, B, W, C, dC);
        float dt = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            g[k] = a.gout[k * a.plane + q];
            dt = __builtin_fmaf(g[k], dC[k], dt);
        }
        if (a.gt) a.gt[q] = dt;
        const float iW = RAT ? 1.0f / W : 1.0f;
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            const float s = RAT ? wv[i] * B[i] * iW : B[i];
#pragma unroll
            for (int k = 0; k < DIM; ++k) gb[k][i] = __builtin_fmaf(g[k], s, gb[k][i]);
            if constexpr (RAT) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < DIM; ++k) acc = __builtin_fmaf(g[k], b[k][i] - C[k], acc);
                gwv[i] = __builtin_fmaf(B[i] * iW, acc, gwv[i]);
            }
        }
    }
    if (a.gctrl) {
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int i = 0; i <= D; ++i) {
                const float v = wave_sum(gb[k][i]);
                if (lane == 0) a.gctrl[(c * DIM + k) * (D + 1) + i] = v;
            }
    }
    if (RAT && a.gw) {
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            const float v = wave_sum(gwv[i]);
            if (lane == 0) a.gw[c * (D + 1) + i] = v;
        }
    }
}

struct FitArgs {
    float *ctrl, *t;
    const float *y;
    float *m_c, *v_c, *m_t, *v_t;
    float *loss_part;
    int64_t n_curves, n_t, plane;
    float inv_m;        // 1 / (n_curves * n_t)
    float lr, b1, b2, eps;
    float ic1, ic2;  // 1 / (1 - b1^step), 1 / (1 - b2^step), rounded once from FP64
};

// Adam update with the bias corrections as multiplications by host-side
// reciprocals and the hardware square root and reciprocal (v_sqrt_f32,
// v_rcp_f32, about 1 ulp) instead of correctly rounded division and square
// root sequences: the update is a heuristic step, and the IEEE sequences cost
// a third of the fitting step's instructions.  Every rounding step is written
// out so that all kernels produce identical bits.
__device__ __forceinline__ float adam_c(float p, float g, float *m, float *v, const FitArgs &a, float ic1, float ic2) {
    const float mm = __builtin_fmaf(a.b1, *m, (1.0f - a.b1) * g);
    const float vv = __builtin_fmaf(a.b2, *v, ((1.0f - a.b2) * g) * g);
    *m = mm;
    *v = vv;
    const float mh = mm * ic1, vh = vv * ic2;
    const float upd = mh * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vh) + a.eps);
    return __builtin_fmaf(-a.lr, upd, p);
}

__device__ __forceinline__ float adam(float p, float g, float *m, float *v, const FitArgs &a) {
    return adam_c(p, g, m, v, a, a.ic1, a.ic2);
}

// Fused step: L = (1/M) sum |C(t) - y|^2, gradients, Adam on t (clamped to
// [0,1]) and on the control points.  All gradients use the parameters as they
// were at the start of the step.  Two curves per wavefront: lanes 0-31 work
// on curve 2w, lanes 32-63 on curve 2w+1, so one DPP butterfly reduces the
// per-curve sums of both.
template <int D, int DIM>
__global__ __launch_bounds__(kBlock) void k_fit_step(FitArgs a) {
    constexpr int NP = DIM * (D + 1);
    constexpr int CPW = NP <= 32 ? 2 : 1;  // curves per wavefront
    constexpr int L = 64 / CPW;            // lanes per curve
    const int lane = threadIdx.x & 63, sub = lane % L;
    const int64_t c0 = CPW * static_cast<int64_t>(__builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)));
    if (c0 >= a.n_curves) return;
    const bool has1 = CPW == 2 && c0 + 1 < a.n_curves;
    const int64_t c = (lane < L || !has1) ? c0 : c0 + 1;
    const bool live = lane < L || has1;  // the upper half idles when the curve count is odd
    // both curves' control points are wave-uniform: scalar loads, then a select
    float b[DIM][D + 1], wv[D + 1] = {};
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            const float v0 = a.ctrl[c0 * NP + k * (D + 1) + i];
            const float v1 = a.ctrl[(has1 ? c0 + 1 : c0) * NP + k * (D + 1) + i];
            b[k][i] = lane < L ? v0 : v1;
        }
    const int64_t pidx = c * NP + (sub < NP ? sub : 0);
    const float p_own = a.ctrl[pidx];
    float m_own = a.m_c[pidx], v_own = a.v_c[pidx];
    float gb[DIM][D + 1] = {};
    float loss = 0.0f;
    for (int64_t j = sub; live && j < a.n_t; j += L) {
        const int64_t q = c * a.n_t + j;
        const float t = a.t[q];
        float mt = a.m_t[q], vt = a.v_t[q];
        float yv[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) yv[k] = a.y[k * a.plane + q];
        float B[D + 1], W, C[DIM], dC[DIM];
        curve_and_derivative<D, DIM, false>(b, wv, t, B, W, C, dC);
        float dt = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const float r = C[k] - yv[k];
            loss = __builtin_fmaf(r, r, loss);
            const float g = 2.0f * r * a.inv_m;
            dt = __builtin_fmaf(g, dC[k], dt);
#pragma unroll
            for (int i = 0; i <= D; ++i) gb[k][i] = __builtin_fmaf(g, B[i], gb[k][i]);
        }
        float tn = adam(t, dt, &mt, &vt, a);
        tn = tn < 0.0f ? 0.0f : (tn > 1.0f ? 1.0f : tn);
        a.t[q] = tn;
        a.m_t[q] = mt;
        a.v_t[q] = vt;
    }
    loss = CPW == 2 ? half_sum(loss) : wave_sum(loss);
    if (a.loss_part && sub == 0 && live) a.loss_part[c] = loss * a.inv_m;
    const float mine = reduce_grads<D, DIM, CPW>(gb, sub);
    if (sub < NP && live) {
        const float pn = adam(p_own, mine, &m_own, &v_own, a);
        a.ctrl[pidx] = pn;
        a.m_c[pidx] = m_own;
        a.v_c[pidx] = v_own;
    }
}

// Gradient of the least-squares loss L = inv_m * sum |C(t) - y|^2 without an
// optimiser step: per-curve loss contributions, dL/db (one sum per control
// point, by the same reductions as the fused step) and dL/dt per query.  The
// lane mapping is that of k_fit_step (two curves per wavefront when a curve
// has at most 32 control-point coordinates); nothing is updated in place.
struct L2Args {
    const float *ctrl, *t, *y;
    float *loss_part, *gctrl, *gt;
    int64_t n_curves, n_t, plane;
    float inv_m;
};

template <int D, int DIM>
__global__ __launch_bounds__(kBlock) void k_l2_adjoint(L2Args a) {
    constexpr int NP = DIM * (D + 1);
    constexpr int CPW = NP <= 32 ? 2 : 1;
    constexpr int L = 64 / CPW;
    const int lane = threadIdx.x & 63, sub = lane % L;
    const int64_t c0 = CPW * static_cast<int64_t>(__builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)));
    if (c0 >= a.n_curves) return;
    const bool has1 = CPW == 2 && c0 + 1 < a.n_curves;
    const int64_t c = (lane < L || !has1) ? c0 : c0 + 1;
    const bool live = lane < L || has1;
    float b[DIM][D + 1], wv[D + 1] = {};
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            const float v0 = a.ctrl[c0 * NP + k * (D + 1) + i];
            const float v1 = a.ctrl[(has1 ? c0 + 1 : c0) * NP + k * (D + 1) + i];
            b[k][i] = lane < L ? v0 : v1;
        }
    float gb[DIM][D + 1] = {};
    float loss = 0.0f;
    for (int64_t j = sub; live && j < a.n_t; j += L) {
        const int64_t q = c * a.n_t + j;
        const float t = a.t[q];
        float yv[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) yv[k] = a.y[k * a.plane + q];
        float B[D + 1], W, C[DIM], dC[DIM];
        curve_and_derivative<D, DIM, false>(b, wv, t, B, W, C, dC);
        float dt = 0.0f;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const float r = C[k] - yv[k];
            loss = __builtin_fmaf(r, r, loss);
            const float g = 2.0f * r * a.inv_m;
            dt = __builtin_fmaf(g, dC[k], dt);
#pragma unroll
            for (int i = 0; i <= D; ++i) gb[k][i] = __builtin_fmaf(g, B[i], gb[k][i]);
        }
        if (a.gt) a.gt[q] = dt;
    }
    if (a.loss_part) {
        loss = CPW == 2 ? half_sum(loss) : wave_sum(loss);
        if (sub == 0 && live) a.loss_part[c] = loss * a.inv_m;
    }
    if (a.gctrl) {
        const float mine = reduce_grads<D, DIM, CPW>(gb, sub);
        if (sub < NP && live) a.gctrl[c * NP + sub] = mine;
    }
}

// Many fitting steps in one launch.  Curves are optimised independently, so
// a wavefront can keep its curves' samples, parameters and Adam moments in
// registers across all steps: HBM is read once and written once.  Each step
// performs exactly the arithmetic of k_fit_step, in the same order.  SPL:
// samples per lane (n_t <= SPL * lanes per curve).  bias[step] = (ic1, ic2).
template <int D, int DIM, int SPL>
__global__ __launch_bounds__(kBlock) void k_fit_run(FitArgs a, const float2 *__restrict__ bias, int n_steps) {
    constexpr int NP = DIM * (D + 1);
    constexpr int CPW = NP <= 32 ? 2 : 1;
    constexpr int L = 64 / CPW;
    const int lane = threadIdx.x & 63, sub = lane % L;
    const int64_t c0 = CPW * static_cast<int64_t>(__builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)));
    if (c0 >= a.n_curves) return;
    const bool has1 = CPW == 2 && c0 + 1 < a.n_curves;
    const int64_t c = (lane < L || !has1) ? c0 : c0 + 1;
    const bool live = lane < L || has1;
    const int base = lane < L ? 0 : L;  // first lane of this lane's curve
    const int64_t pidx = c * NP + (sub < NP ? sub : 0);
    float p_own = a.ctrl[pidx], m_own = a.m_c[pidx], v_own = a.v_c[pidx];
    float ts[SPL], mts[SPL], vts[SPL], ys[SPL][DIM];
    int64_t qs[SPL];
    bool ok[SPL];
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        const int64_t j = sub + static_cast<int64_t>(s) * L;
        ok[s] = live && j < a.n_t;
        qs[s] = c * a.n_t + (ok[s] ? j : 0);
        ts[s] = a.t[qs[s]];
        mts[s] = a.m_t[qs[s]];
        vts[s] = a.v_t[qs[s]];
#pragma unroll
        for (int k = 0; k < DIM; ++k) ys[s][k] = a.y[k * a.plane + qs[s]];
    }
    float b[DIM][D + 1], wv[D + 1] = {};
    float loss = 0.0f;
    const float two_inv_m = 2.0f * a.inv_m;
    for (int step = 0; step < n_steps; ++step) {
        // current control points of this lane's curve, from the owning lanes
        // (a lane-indexed permute through the LDS crossbar: one instruction per
        // parameter for both curves of the wave, none of them VALU)
        const int pb = __builtin_bit_cast(int, p_own);
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int i = 0; i <= D; ++i)
                b[k][i] = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((base + k * (D + 1) + i) << 2, pb));
        const float2 bc = bias[step];
        float gb[DIM][D + 1] = {};
        loss = 0.0f;
#pragma unroll
        for (int s = 0; s < SPL; ++s) {
            if (!ok[s]) continue;
            float B[D + 1], W, C[DIM], dC[DIM];
            curve_and_derivative<D, DIM, false>(b, wv, ts[s], B, W, C, dC);
            float dt = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const float r = C[k] - ys[s][k];
                loss = __builtin_fmaf(r, r, loss);
                const float g = r * two_inv_m;  // = (2r) inv_m exactly: scaling by 2 commutes with rounding
                dt = __builtin_fmaf(g, dC[k], dt);
#pragma unroll
                for (int i = 0; i <= D; ++i) gb[k][i] = __builtin_fmaf(g, B[i], gb[k][i]);
            }
            float tn = adam_c(ts[s], dt, &mts[s], &vts[s], a, bc.x, bc.y);
            ts[s] = tn < 0.0f ? 0.0f : (tn > 1.0f ? 1.0f : tn);
        }
        const float mine = reduce_grads<D, DIM, CPW>(gb, sub);
        if (sub < NP && live) p_own = adam_c(p_own, mine, &m_own, &v_own, a, bc.x, bc.y);
    }
    // only the last step's loss is reported, so only it is summed over the lanes
    loss = CPW == 2 ? half_sum(loss) : wave_sum(loss);
    if (a.loss_part && sub == 0 && live) a.loss_part[c] = loss * a.inv_m;
    if (sub < NP && live) {
        a.ctrl[pidx] = p_own;
        a.m_c[pidx] = m_own;
        a.v_c[pidx] = v_own;
    }
#pragma unroll
    for (int s = 0; s < SPL; ++s)
        if (ok[s]) {
            a.t[qs[s]] = ts[s];
            a.m_t[qs[s]] = mts[s];
            a.v_t[qs[s]] = vts[s];
        }
}

template <int D, int DIM>
int launch_fit_run_dd(const FitArgs &a, const float2 *bias, int n_steps, hipStream_t s) {
    constexpr int NP = DIM * (D + 1);
    constexpr int L = NP <= 32 ? 32 : 64;
    constexpr int CPW = 64 / L;
    const uint32_t blocks = static_cast<uint32_t>((a.n_curves + 4 * CPW - 1) / (4 * CPW));
    const int64_t spl = (a.n_t + L - 1) / L;
    if (spl <= 1) hipLaunchKernelGGL((k_fit_run<D, DIM, 1>), dim3(blocks), dim3(kBlock), 0, s, a, bias, n_steps);
    else if (spl <= 2) hipLaunchKernelGGL((k_fit_run<D, DIM, 2>), dim3(blocks), dim3(kBlock), 0, s, a, bias, n_steps);
    else hipLaunchKernelGGL((k_fit_run<D, DIM, 4>), dim3(blocks), dim3(kBlock), 0, s, a, bias, n_steps);
    BZ_CHECK_LAUNCH("k_fit_run");
    return BZ_OK;
}

template <int D>
int launch_fit_run_d(int dim, const FitArgs &a, const float2 *bias, int n_steps, hipStream_t s) {
    switch (dim) {
        case 1: return launch_fit_run_dd<D, 1>(a, bias, n_steps, s);
        case 2: return launch_fit_run_dd<D, 2>(a, bias, n_steps, s);
        case 3: return launch_fit_run_dd<D, 3>(a, bias, n_steps, s);
        default: return launch_fit_run_dd<D, 4>(a, bias, n_steps, s);
    }
}

int launch_fit_run(int degree, int dim, const FitArgs &a, const float2 *bias, int n_steps, hipStream_t s) {
    switch (degree) {
        case 1: return launch_fit_run_d<1>(dim, a, bias, n_steps, s);
        case 2: return launch_fit_run_d<2>(dim, a, bias, n_steps, s);
        case 3: return launch_fit_run_d<3>(dim, a, bias, n_steps, s);
        case 4: return launch_fit_run_d<4>(dim, a, bias, n_steps, s);
        case 5: return launch_fit_run_d<5>(dim, a, bias, n_steps, s);
        case 6: return launch_fit_run_d<6>(dim, a, bias, n_steps, s);
        case 7: return launch_fit_run_d<7>(dim, a, bias, n_steps, s);
        case 8: return launch_fit_run_d<8>(dim, a, bias, n_steps, s);
        case 9: return launch_fit_run_d<9>(dim, a, bias, n_steps, s);
        case 10: return launch_fit_run_d<10>(dim, a, bias, n_steps, s);
        case 11: return launch_fit_run_d<11>(dim, a, bias, n_steps, s);
        case 12: return launch_fit_run_d<12>(dim, a, bias, n_steps, s);
        case 13: return launch_fit_run_d<13>(dim, a, bias, n_steps, s);
        case 14: return launch_fit_run_d<14>(dim, a, bias, n_steps, s);
        default: return launch_fit_run_d<15>(dim, a, bias, n_steps, s);
    }
}

template <int D, bool RAT>
int launch_adj_d(int dim, const AdjArgs &a, hipStream_t s, uint32_t blocks) {
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_adjoint<D, 1, RAT>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_adjoint<D, 2, RAT>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_adjoint<D, 3, RAT>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_adjoint<D, 4, RAT>), dim3(blocks), dim3(kBlock), 0, s, a); break;
    }
    BZ_CHECK_LAUNCH("k_adjoint");
    return BZ_OK;
}

template <bool RAT>
int launch_adj(int degree, int dim, const AdjArgs &a, hipStream_t s, uint32_t blocks) {
    switch (degree) {
        case 1: return launch_adj_d<1, RAT>(dim, a, s, blocks);
        case 2: return launch_adj_d<2, RAT>(dim, a, s, blocks);
        case 3: return launch_adj_d<3, RAT>(dim, a, s, blocks);
        case 4: return launch_adj_d<4, RAT>(dim, a, s, blocks);
        case 5: return launch_adj_d<5, RAT>(dim, a, s, blocks);
        case 6: return launch_adj_d<6, RAT>(dim, a, s, blocks);
        case 7: return launch_adj_d<7, RAT>(dim, a, s, blocks);
        case 8: return launch_adj_d<8, RAT>(dim, a, s, blocks);
        case 9: return launch_adj_d<9, RAT>(dim, a, s, blocks);
        case 10: return launch_adj_d<10, RAT>(dim, a, s, blocks);
        case 11: return launch_adj_d<11, RAT>(dim, a, s, blocks);
        case 12: return launch_adj_d<12, RAT>(dim, a, s, blocks);
        case 13: return launch_adj_d<13, RAT>(dim, a, s, blocks);
        case 14: return launch_adj_d<14, RAT>(dim, a, s, blocks);
        default: return launch_adj_d<15, RAT>(dim, a, s, blocks);
    }
}

template <int D>
int launch_fit_d(int dim, const FitArgs &a, hipStream_t s) {
    const int cpw = dim * (D + 1) <= 32 ? 2 : 1;
    const uint32_t blocks = static_cast<uint32_t>((a.n_curves + 4 * cpw - 1) / (4 * cpw));
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_fit_step<D, 1>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_fit_step<D, 2>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_fit_step<D, 3>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_fit_step<D, 4>), dim3(blocks), dim3(kBlock), 0, s, a); break;
    }
    BZ_CHECK_LAUNCH("k_fit_step");
    return BZ_OK;
}

int launch_fit(int degree, int dim, const FitArgs &a, hipStream_t s) {
    switch (degree) {
        case 1: return launch_fit_d<1>(dim, a, s);
        case 2: return launch_fit_d<2>(dim, a, s);
        case 3: return launch_fit_d<3>(dim, a, s);
        case 4: return launch_fit_d<4>(dim, a, s);
        case 5: return launch_fit_d<5>(dim, a, s);
        case 6: return launch_fit_d<6>(dim, a, s);
        case 7: return launch_fit_d<7>(dim, a, s);
        case 8: return launch_fit_d<8>(dim, a, s);
        case 9: return launch_fit_d<9>(dim, a, s);
        case 10: return launch_fit_d<10>(dim, a, s);
        case 11: return launch_fit_d<11>(dim, a, s);
        case 12: return launch_fit_d<12>(dim, a, s);
        case 13: return launch_fit_d<13>(dim, a, s);
        case 14: return launch_fit_d<14>(dim, a, s);
        default: return launch_fit_d<15>(dim, a, s);
    }
}

template <int D>
int launch_l2_d(int dim, const L2Args &a, hipStream_t s) {
    const int cpw = dim * (D + 1) <= 32 ? 2 : 1;
    const uint32_t blocks = static_cast<uint32_t>((a.n_curves + 4 * cpw - 1) / (4 * cpw));
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_l2_adjoint<D, 1>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_l2_adjoint<D, 2>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_l2_adjoint<D, 3>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_l2_adjoint<D, 4>), dim3(blocks), dim3(kBlock), 0, s, a); break;
    }
    BZ_CHECK_LAUNCH("k_l2_adjoint");
    return BZ_OK;
}

int launch_l2(int degree, int dim, const L2Args &a, hipStream_t s) {
    switch (degree) {
        case 1: return launch_l2_d<1>(dim, a, s);
        case 2: return launch_l2_d<2>(dim, a, s);
        case 3: return launch_l2_d<3>(dim, a, s);
        case 4: return launch_l2_d<4>(dim, a, s);
        case 5: return launch_l2_d<5>(dim, a, s);
        case 6: return launch_l2_d<6>(dim, a, s);
        case 7: return launch_l2_d<7>(dim, a, s);
        case 8: return launch_l2_d<8>(dim, a, s);
        case 9: return launch_l2_d<9>(dim, a, s);
        case 10: return launch_l2_d<10>(dim, a, s);
        case 11: return launch_l2_d<11>(dim, a, s);
        case 12: return launch_l2_d<12>(dim, a, s);
        case 13: return launch_l2_d<13>(dim, a, s);
        case 14: return launch_l2_d<14>(dim, a, s);
        default: return launch_l2_d<15>(dim, a, s);
    }
}

int check_fit(const char *fn, float *ctrl, float *t, const float *y, int64_t n_curves, int degree, int dim, int64_t n_t,
              float *m_ctrl, float *v_ctrl, float *m_t, float *v_t, float lr, float beta1, float beta2, float eps) {
    if (degree < 1 || degree > kMaxDegree || dim < 1 || dim > kMaxDim)
        return fail(BZ_ERR_SHAPE, "%s: degree %d / dim %d out of range", fn, degree, dim);
    if (n_curves < 0 || n_t < 0 || n_t > 1024) return fail(BZ_ERR_SHAPE, "%s: need 0 <= n_t <= 1024", fn);
    if (n_curves > (int64_t(1) << 31) - 1) return fail(BZ_ERR_SHAPE, "%s: too many curves", fn);
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return fail(BZ_ERR_SHAPE, "%s: bad Adam hyper-parameters", fn);
    if (n_curves == 0 || n_t == 0) return BZ_OK;
    if (!ctrl || !t || !y || !m_ctrl || !v_ctrl || !m_t || !v_t) return fail(BZ_ERR_NULL, "%s: missing array", fn);
    return BZ_OK;
}

FitArgs make_fit_args(float *ctrl, float *t, const float *y, int64_t n_curves, int64_t n_t, float *m_ctrl,
                      float *v_ctrl, float *m_t, float *v_t, int step, float lr, float beta1, float beta2, float eps,
                      float *loss_part) {
    FitArgs a;
    a.ctrl = ctrl;
    a.t = t;
    a.y = y;
    a.m_c = m_ctrl;
    a.v_c = v_ctrl;
    a.m_t = m_t;
    a.v_t = v_t;
    a.loss_part = loss_part;
    a.n_curves = n_curves;
    a.n_t = n_t;
    a.plane = n_curves * n_t;
    a.inv_m = static_cast<float>(1.0 / static_cast<double>(n_curves * n_t));
    a.lr = lr;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.ic1 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(beta1), step)));
    a.ic2 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(beta2), step)));
    return a;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

int bz_adjoint_bezier(const float *ctrl, const float *w, int64_t n_curves, int degree, int dim, const float *t,
                      int64_t n_t, int t_mode, const float *grad_out, float *grad_ctrl, float *grad_w, float *grad_t,
                      bz_stream stream) {
    return guarded("bz_adjoint_bezier", [&]() -> int {
        const char *fn = "bz_adjoint_bezier";
        if (degree < 1 || degree > kMaxDegree || dim < 1 || dim > kMaxDim)
            return fail(BZ_ERR_SHAPE, "%s: degree %d / dim %d out of range", fn, degree, dim);
        if (n_curves < 0 || n_t < 0) return fail(BZ_ERR_SHAPE, "%s: negative count", fn);
        if (t_mode != BZ_T_SHARED && t_mode != BZ_T_PER_OBJECT) return fail(BZ_ERR_SHAPE, "%s: bad t_mode", fn);
        if (grad_t && t_mode != BZ_T_PER_OBJECT) return fail(BZ_ERR_UNSUPPORTED, "%s: grad_t needs per-object t", fn);
        if (grad_w && !w) return fail(BZ_ERR_NULL, "%s: grad_w needs w", fn);
        if (n_curves > (int64_t(1) << 31) - 1) return fail(BZ_ERR_SHAPE, "%s: too many curves", fn);
        if (n_curves == 0 || n_t == 0) return BZ_OK;
        if (!ctrl || !t || !grad_out) return fail(BZ_ERR_NULL, "%s: ctrl, t and grad_out are required", fn);
        AdjArgs a{ctrl, w, t, grad_out, grad_ctrl, grad_w, grad_t, n_curves, n_t, n_curves * n_t,
                  t_mode == BZ_T_PER_OBJECT};
        const uint32_t blocks = static_cast<uint32_t>((n_curves + 3) / 4);
        const hipStream_t s = as_stream(stream);
        return w ? launch_adj<true>(degree, dim, a, s, blocks) : launch_adj<false>(degree, dim, a, s, blocks);
    });
}

int bz_l2_fit_adjoint(const float *ctrl, int64_t n_curves, int degree, int dim, const float *t, int64_t n_t,
                      const float *target, float *loss_part, float *grad_ctrl, float *grad_t, bz_stream stream) {
    return guarded("bz_l2_fit_adjoint", [&]() -> int {
        const char *fn = "bz_l2_fit_adjoint";
        if (degree < 1 || degree > kMaxDegree || dim < 1 || dim > kMaxDim)
            return fail(BZ_ERR_SHAPE, "%s: degree %d / dim %d out of range", fn, degree, dim);
        if (n_curves < 0 || n_t < 0) return fail(BZ_ERR_SHAPE, "%s: negative count", fn);
        if (n_curves > (int64_t(1) << 31) - 1) return fail(BZ_ERR_SHAPE, "%s: too many curves", fn);
        if (n_curves == 0 || n_t == 0) return BZ_OK;
        if (!ctrl || !t || !target) return fail(BZ_ERR_NULL, "%s: ctrl, t and target are required", fn);
        if (!aligned(ctrl, 4) || !aligned(t, 4) || !aligned(target, 4) || !aligned(loss_part, 4) ||
            !aligned(grad_ctrl, 4) || !aligned(grad_t, 4))
            return fail(BZ_ERR_ALIGN, "%s: FP32 arrays need 4-byte alignment", fn);
        L2Args a;
        a.ctrl = ctrl;
        a.t = t;
        a.y = target;
        a.loss_part = loss_part;
        a.gctrl = grad_ctrl;
        a.gt = grad_t;
        a.n_curves = n_curves;
        a.n_t = n_t;
        a.plane = n_curves * n_t;
        a.inv_m = static_cast<float>(1.0 / static_cast<double>(n_curves * n_t));
        return launch_l2(degree, dim, a, as_stream(stream));
    });
}

int bz_fit_adam_step(float *ctrl, float *t, const float *y, int64_t n_curves, int degree, int dim, int64_t n_t,
                     float *m_ctrl, float *v_ctrl, float *m_t, float *v_t, int step, float lr, float beta1, float beta2,
                     float eps, float *loss_part, bz_stream stream) {
    return guarded("bz_fit_adam_step", [&]() -> int {
        int rc = check_fit("bz_fit_adam_step", ctrl, t, y, n_curves, degree, dim, n_t, m_ctrl, v_ctrl, m_t, v_t, lr,
                           beta1, beta2, eps);
        if (rc || n_curves == 0 || n_t == 0) return rc;
        if (step < 1) return fail(BZ_ERR_SHAPE, "bz_fit_adam_step: step counts from 1");
        const FitArgs a = make_fit_args(ctrl, t, y, n_curves, n_t, m_ctrl, v_ctrl, m_t, v_t, step, lr, beta1, beta2,
                                        eps, loss_part);
        return launch_fit(degree, dim, a, as_stream(stream));
    });
}

int bz_fit_adam_run(float *ctrl, float *t, const float *y, int64_t n_curves, int degree, int dim, int64_t n_t,
                    float *m_ctrl, float *v_ctrl, float *m_t, float *v_t, int first_step, int n_steps, float lr,
                    float beta1, float beta2, float eps, float *loss_part, bz_stream stream) {
    return guarded("bz_fit_adam_run", [&]() -> int {
        const char *fn = "bz_fit_adam_run";
        int rc = check_fit(fn, ctrl, t, y, n_curves, degree, dim, n_t, m_ctrl, v_ctrl, m_t, v_t, lr, beta1, beta2, eps);
        if (rc || n_curves == 0 || n_t == 0 || n_steps == 0) return rc;
        if (first_step < 1 || n_steps < 0) return fail(BZ_ERR_SHAPE, "%s: steps count from 1", fn);
        const hipStream_t s = as_stream(stream);
        const int64_t lanes_per_curve = dim * (degree + 1) <= 32 ? 32 : 64;
        if (n_t <= 4 * lanes_per_curve) {
            // all steps in one launch, per-curve state in registers
            std::vector<float> tab(2 * static_cast<size_t>(n_steps));
            for (int i = 0; i < n_steps; ++i) {
                const FitArgs ai = make_fit_args(ctrl, t, y, n_curves, n_t, m_ctrl, v_ctrl, m_t, v_t, first_step + i,
                                                 lr, beta1, beta2, eps, loss_part);
                tab[2 * i] = ai.ic1;
                tab[2 * i + 1] = ai.ic2;
            }
            float2 *bias = nullptr;
            hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&bias), tab.size() * sizeof(float), s);
            if (e == hipErrorOutOfMemory) return fail(BZ_ERR_NOMEM, "%s: bias table", fn);
            BZ_CHECK_HIP(e);
            e = hipMemcpyAsync(bias, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, s);
            const FitArgs a = make_fit_args(ctrl, t, y, n_curves, n_t, m_ctrl, v_ctrl, m_t, v_t, first_step, lr, beta1,
                                            beta2, eps, loss_part);
            if (e == hipSuccess) rc = launch_fit_run(degree, dim, a, bias, n_steps, s);
            else rc = hip_fail(e, "bias table copy");
            const hipError_t e2 = hipFreeAsync(bias, s);
            const hipError_t e3 = hipStreamSynchronize(s);
            if (rc == BZ_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipFreeAsync");
            if (rc == BZ_OK && e3 != hipSuccess) rc = hip_fail(e3, "hipStreamSynchronize");
            return rc;
        }
        // otherwise: capture the single steps on a private stream and replay the graph
        hipStream_t cap;
        BZ_CHECK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int i = 0; i < n_steps && rc == BZ_OK; ++i) {
                const FitArgs a = make_fit_args(ctrl, t, y, n_curves, n_t, m_ctrl, v_ctrl, m_t, v_t, first_step + i,
                                                lr, beta1, beta2, eps, loss_part);
                rc = launch_fit(degree, dim, a, cap);
            }
            const hipError_t e2 = hipStreamEndCapture(cap, &graph);
            if (rc == BZ_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
        } else {
            rc = hip_fail(e, "begin capture");
        }
        if (rc == BZ_OK) {
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e == hipSuccess) e = hipGraphLaunch(exec, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = hip_fail(e, "graph launch");
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        return rc;
    });
}

}  // extern "C"
