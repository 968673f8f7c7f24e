// Seiler surfaces and volumes: per-axis Seiler terms (the curve conversion
// of Sec. 3 applied to every fibre of the tensor net of Sec. 2.2, the
// direction Sec. 6 leaves open).
//
//  k_tensor_to_seiler  one thread per (object, coordinate): the net in FP64
//                      registers, fibres converted along w, v, u, each term
//                      rounded once to FP32.
//  evaluation          the separable kernels of tensor_impl.h with the Seiler
//                      basis 1-t, t, st(1-t), st t, ... per axis: the nested
//                      Seiler recursion is linear in the terms, so the
//                      contraction over the net is unchanged.
#include "tensor_impl.h"

namespace bzi {
namespace {

template <int D, int NF>
__device__ __forceinline__ void convert_fibre(double (&a)[NF], int base, int stride) {
    if constexpr (D >= 1) {
        double b[D + 1], sc[D + 1];
#pragma unroll
        for (int i = 0; i <= D; ++i) b[i] = a[base + i * stride];
        seiler_terms<D, double, double, double>(b, sc);
#pragma unroll
        for (int i = 0; i <= D; ++i) a[base + i * stride] = sc[i];
    }
}

template <int DU, int DV, int DW>
__global__ __launch_bounds__(kBlock) void k_tensor_to_seiler(const float *__restrict__ ctrl, float *__restrict__ sc,
                                                              uint32_t n_rows) {
    constexpr int NV = DV + 1, NW = DW + 1, NCP = (DU + 1) * NV * NW;
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_rows) return;
    double a[NCP];
#pragma unroll
    for (int e = 0; e < NCP; ++e) a[e] = static_cast<double>(ctrl[static_cast<size_t>(r) * NCP + e]);
#pragma unroll
    for (int i = 0; i <= DU; ++i)
#pragma unroll
        for (int j = 0; j <= DV; ++j) convert_fibre<DW>(a, (i * NV + j) * NW, 1);
#pragma unroll
    for (int i = 0; i <= DU; ++i)
#pragma unroll
        for (int k = 0; k <= DW; ++k) convert_fibre<DV>(a, i * NV * NW + k, NW);
#pragma unroll
    for (int j = 0; j <= DV; ++j)
#pragma unroll
        for (int k = 0; k <= DW; ++k) convert_fibre<DU>(a, j * NW + k, NV * NW);
#pragma unroll
    for (int e = 0; e < NCP; ++e) sc[static_cast<size_t>(r) * NCP + e] = static_cast<float>(a[e]);
}

template <int DU, int DV>
int launch_to_seiler2(int dw, const float *ctrl, float *sc, uint32_t rows, hipStream_t s) {
    const uint32_t blocks = (rows + kBlock - 1) / kBlock;
    switch (dw) {
        case 0: hipLaunchKernelGGL((k_tensor_to_seiler<DU, DV, 0>), dim3(blocks), dim3(kBlock), 0, s, ctrl, sc, rows); break;
        case 1: hipLaunchKernelGGL((k_tensor_to_seiler<DU, DV, 1>), dim3(blocks), dim3(kBlock), 0, s, ctrl, sc, rows); break;
        case 2: hipLaunchKernelGGL((k_tensor_to_seiler<DU, DV, 2>), dim3(blocks), dim3(kBlock), 0, s, ctrl, sc, rows); break;
        case 3: hipLaunchKernelGGL((k_tensor_to_seiler<DU, DV, 3>), dim3(blocks), dim3(kBlock), 0, s, ctrl, sc, rows); break;
        default: hipLaunchKernelGGL((k_tensor_to_seiler<DU, DV, 4>), dim3(blocks), dim3(kBlock), 0, s, ctrl, sc, rows); break;
    }
    BZ_CHECK_LAUNCH("k_tensor_to_seiler");
    return BZ_OK;
}

template <int DU>
int launch_to_seiler1(int dv, int dw, const float *ctrl, float *sc, uint32_t rows, hipStream_t s) {
    switch (dv) {
        case 1: return launch_to_seiler2<DU, 1>(dw, ctrl, sc, rows, s);
        case 2: return launch_to_seiler2<DU, 2>(dw, ctrl, sc, rows, s);
        case 3: return launch_to_seiler2<DU, 3>(dw, ctrl, sc, rows, s);
        default: return launch_to_seiler2<DU, 4>(dw, ctrl, sc, rows, s);
    }
}

int check_degrees(const char *fn, int du, int dv, int dw, int dim, int64_t n_obj) {
    if (du < 1 || du > 4 || dv < 1 || dv > 4 || dw < 0 || dw > 4)
        return fail(BZ_ERR_SHAPE, "%s: degrees (%d,%d,%d) outside 1..4 (dw 0..4)", fn, du, dv, dw);
    if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
    if (n_obj < 0) return fail(BZ_ERR_SHAPE, "%s: n_obj %lld", fn, (long long)n_obj);
    return BZ_OK;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

int bz_tensor_to_seiler(const float *ctrl, int64_t n_obj, int du, int dv, int dw, int dim, float *sc,
                        bz_stream stream) {
    return guarded("bz_tensor_to_seiler", [&]() -> int {
        const char *fn = "bz_tensor_to_seiler";
        int rc = check_degrees(fn, du, dv, dw, dim, n_obj);
        if (rc) return rc;
        if (n_obj == 0) return BZ_OK;
        if (!ctrl || !sc) return fail(BZ_ERR_NULL, "%s: ctrl and sc are required", fn);
        if (!aligned(ctrl, 4) || !aligned(sc, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
        const int ncp = (du + 1) * (dv + 1) * (dw + 1);
        const hipStream_t s = as_stream(stream);
        const int64_t rows = n_obj * dim;
        const int64_t per = int64_t(1) << 30;
        for (int64_t r0 = 0; r0 < rows; r0 += per) {
            const uint32_t nr = static_cast<uint32_t>(std::min(per, rows - r0));
            const float *c0 = ctrl + r0 * ncp;
            float *s0 = sc + r0 * ncp;
            switch (du) {
                case 1: rc = launch_to_seiler1<1>(dv, dw, c0, s0, nr, s); break;
                case 2: rc = launch_to_seiler1<2>(dv, dw, c0, s0, nr, s); break;
                case 3: rc = launch_to_seiler1<3>(dv, dw, c0, s0, nr, s); break;
                default: rc = launch_to_seiler1<4>(dv, dw, c0, s0, nr, s); break;
            }
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

int bz_eval_tensor_seiler(const float *sc, int64_t n_obj, int du, int dv, int dw, int dim, const float *uvw,
                          int64_t n_per, int nu, int nv, float *out, bz_stream stream) {
    return guarded("bz_eval_tensor_seiler", [&]() -> int {
        const char *fn = "bz_eval_tensor_seiler";
        int rc = check_degrees(fn, du, dv, dw, dim, n_obj);
        if (rc) return rc;
        const int ncp = (du + 1) * (dv + 1) * (dw + 1);
        const hipStream_t s = as_stream(stream);
        const int64_t per = int64_t(1) << 22;
        if (uvw == nullptr) {  // grid mode
            if (dw != 0) return fail(BZ_ERR_UNSUPPORTED, "%s: grid mode is for surfaces (dw = 0)", fn);
            if (nu < 1 || nv < 1 || static_cast<int64_t>(nu) * nv > (1 << 24))
                return fail(BZ_ERR_SHAPE, "%s: grid %d x %d", fn, nu, nv);
            if (n_obj == 0) return BZ_OK;
            if (!sc || !out) return fail(BZ_ERR_NULL, "%s: sc and out are required", fn);
            if (!aligned(sc, 4) || !aligned(out, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
            const int64_t plane = n_obj * static_cast<int64_t>(nu) * nv;
            for (int64_t o0 = 0; o0 < n_obj; o0 += per) {
                const uint32_t blocks = static_cast<uint32_t>(std::min(per, n_obj - o0));
                launch_grid<float, kBasisSeiler>(du, dv, dim, sc + o0 * dim * ncp, nu, nv, out, plane, o0, blocks, s);
                BZ_CHECK_LAUNCH("k_tensor_grid");
            }
            return BZ_OK;
        }
        if (n_per < 0) return fail(BZ_ERR_SHAPE, "%s: n_per %lld", fn, (long long)n_per);
        if (n_obj == 0 || n_per == 0) return BZ_OK;
        if (!sc || !out) return fail(BZ_ERR_NULL, "%s: sc and out are required", fn);
        if (!aligned(sc, 4) || !aligned(uvw, 4) || !aligned(out, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
        const int64_t plane = n_obj * n_per;
        for (int64_t o0 = 0; o0 < n_obj; o0 += per) {
            const uint32_t blocks = static_cast<uint32_t>(std::min(per, n_obj - o0));
            launch_pts<float, kBasisSeiler>(du, dv, dw, dim, sc + o0 * dim * ncp, uvw, n_per, out, plane, o0, blocks,
                                            s);
            BZ_CHECK_LAUNCH("k_tensor_points");
        }
        return BZ_OK;
    });
}

}  // extern "C"
