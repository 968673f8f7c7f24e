// C0 piecewise cubic chains as two zig-zag layers stacked front to back
// (Sec. 2.1: a cubic is the depth interpolation of two quadratics that share
// their end control points).  Random-access evaluator of the two-layer grid
// written by bz_encode_piecewise_cubic.
#include "common.h"

namespace bzi {
namespace {

// Cubic chain: grid[N+1][2 layers][2 rows][dim]; segment k reads columns k
// and k+1 (a contiguous 32*dim-byte window, 16-byte aligned), takes the
// bilinear diagonal read of each layer and lerps the two layers (the
// trilinear read of a 2x2x2 texture) with the same t.
template <int DIM, int QPT>
__global__ __launch_bounds__(kBlock) void k_piecewise_cubic_eval(const float *__restrict__ grid, uint32_t n_seg,
                                                                 const float *__restrict__ T, uint32_t nq,
                                                                 float *__restrict__ out, int64_t plane) {
    const uint32_t base = blockIdx.x * (kBlock * QPT) + threadIdx.x;
    const float nf = static_cast<float>(n_seg);
    const float nm1 = static_cast<float>(n_seg - 1);
    float tl[QPT];
    uint32_t kk[QPT];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
        const float Tq = ld_stream(T + q);
        float Tc = Tq < 0.0f ? 0.0f : Tq;
        Tc = Tc > nf ? nf : Tc;
        const float kf = __builtin_fminf(__builtin_floorf(Tc), nm1);
        const uint32_t k = min(static_cast<uint32_t>(kf), n_seg - 1);
        kk[i] = k;
        tl[i] = Tc - static_cast<float>(k);
    }
    float4 g[QPT][2 * DIM];
    const float4 *__restrict__ g4 = reinterpret_cast<const float4 *>(grid);
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) g[i][e] = g4[static_cast<size_t>(kk[i]) * DIM + e];
    float v[QPT][DIM];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        float f[8 * DIM];  // [column 0/1][layer 0/1][row 0/1][dim]
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) {
            f[4 * e] = g[i][e].x;
            f[4 * e + 1] = g[i][e].y;
            f[4 * e + 2] = g[i][e].z;
            f[4 * e + 3] = g[i][e].w;
        }
        const bool odd = kk[i] & 1;
        const float t = tl[i];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            float lv[2];
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const float c0r0 = f[(0 * 2 + l) * 2 * DIM + c], c0r1 = f[(0 * 2 + l) * 2 * DIM + DIM + c];
                const float c1r0 = f[(1 * 2 + l) * 2 * DIM + c], c1r1 = f[(1 * 2 + l) * 2 * DIM + DIM + c];
                const float A = odd ? c0r1 : c0r0, xk = odd ? c0r0 : c0r1;
                const float xk1 = odd ? c1r1 : c1r0, A1 = odd ? c1r0 : c1r1;
                lv[l] = lerp(lerp(A, xk1, t), lerp(xk, A1, t), t);
            }
            v[i][c] = lerp(lv[0], lv[1], t);
        }
    }
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) st_stream(out + c * plane + q, v[i][c]);
    }
}

template <int DIM>
int launch_cubic_eval(const float *grid, uint32_t n_seg, const float *T, uint32_t nq, float *out, int64_t plane,
                      hipStream_t s) {
    constexpr int Q = 4;
    const uint32_t blocks = (nq + kBlock * Q - 1) / (kBlock * Q);
    hipLaunchKernelGGL((k_piecewise_cubic_eval<DIM, Q>), dim3(blocks), dim3(kBlock), 0, s, grid, n_seg, T, nq, out,
                       plane);
    BZ_CHECK_LAUNCH("k_piecewise_cubic_eval");
    return BZ_OK;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

int bz_eval_piecewise_cubic(const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                            bz_stream stream) {
    return guarded("bz_eval_piecewise_cubic", [&]() -> int {
        const char *fn = "bz_eval_piecewise_cubic";
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_q < 0) return fail(BZ_ERR_SHAPE, "%s: n_q", fn);
        if (n_seg < 1 || n_seg > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_seg not in 1..2^31", fn);
        if (n_q == 0) return BZ_OK;
        if (!grid || !T || !out) return fail(BZ_ERR_NULL, "%s: grid, T and out are required", fn);
        if (!aligned(grid, 16) || !aligned(T, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "%s: grid needs 16-byte, T and out 4-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const int64_t per = int64_t(1) << 30;
        for (int64_t q0 = 0; q0 < n_q; q0 += per) {
            const uint32_t nq = static_cast<uint32_t>(std::min(per, n_q - q0));
            const uint32_t ns = static_cast<uint32_t>(n_seg);
            int rc;
            switch (dim) {
                case 1: rc = launch_cubic_eval<1>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
                case 2: rc = launch_cubic_eval<2>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
                case 3: rc = launch_cubic_eval<3>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
                default: rc = launch_cubic_eval<4>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
            }
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

}  // extern "C"
