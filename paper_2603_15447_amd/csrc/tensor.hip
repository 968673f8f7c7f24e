// Tensor-product Bezier surfaces and volumes (Sec. 2.2: the order splits
// over the parameter axes) for gfx950.
//
//  k_tensor_grid   one patch per workgroup, nu x nv uniform grid.  When the
//                  block size is a multiple of nv every thread keeps one grid
//                  column b, contracts the control net with the v basis once
//                  (isoline control points R_i(v_b)) and then needs only the
//                  u basis and du+1 FMAs per coordinate for each of its points.
//  k_tensor_points one object per wavefront, random (u,v[,w]) per query,
//                  4 queries per lane, separable contraction w -> v -> u.
//  k_tensor_mfma   bicubic 32x32 grids as a dense contraction on the matrix
//                  cores: D[(patch,coord)][grid pt] = P[(patch,coord)][16] x
//                  K[16][grid pt] with K the Kronecker product of the u and v
//                  Bernstein bases, one 32x32 output tile per MFMA group.
//                  FP16x3 splits both operands into FP16 high and low parts
//                  (each control-point row first scaled by a power of two so
//                  that its largest entry lies in [0.5, 1)) and sums the
//                  products hi*hi + hi*lo + lo*hi in the FP32 accumulator,
//                  which recovers FP32-class accuracy from FP16 MFMAs.
#include "tensor_impl.h"

namespace bzi {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

enum { MF_F32 = 0, MF_BF16 = 1, MF_F16 = 2, MF_F16X3 = 3 };

// Bicubic patches on a 32 x 32 grid.  Rows of the contraction are the
// (patch, coordinate) pairs of the control-point array read as
// [n_obj*dim][16]; each workgroup owns the 32 rows of one coordinate c of 32
// consecutive patches, so its whole output is one contiguous 128 KB block of
// plane c, addressed from a wave-uniform base with a 32-bit lane offset.  The
// 32 grid rows a go to kMfmaGridSplit<ENG> workgroups in equal ranges, whose
// four waves take them in turn (wave w: a = first + w, first + w + 4, ...), so
// the block is written front to back, four consecutive lines per row at a
// time.  The cubic basis at the 32 grid parameters comes from a 512-byte LDS
// table filled once per workgroup.
// Per grid row a wave issues the MFMA(s) of a 32 x 32 x 16 product (FP32: the
// u contraction on the vector ALU, then a 32 x 32 x 4 product) and stores the
// 32 x 32 result tile (each half-wave writes 128 contiguous bytes).
// Output-tile layout of the 32x32 MFMAs: lane l holds column l%32 and, in
// accumulator register r, row 8*(r/4) + 4*(l/32) + r%4.
// Workgroups per (32 patches, coordinate): the grid rows are split over
// kMfmaGridSplit workgroups of short waves (measured faster for every engine
// once the FP32 engine contracts u on the vector ALU; with the 16-term
// Kronecker basis, eight FP32 MFMAs per grid row drew enough power that more
// parallel work only lowered the sustained clock).
template <int ENG>
constexpr int kMfmaGridSplit = 4;

template <int ENG>
__global__ __launch_bounds__(kBlock) void k_tensor_mfma(const float *__restrict__ ctrl, uint32_t n_patches, uint32_t dim,
                                                        float *__restrict__ out, int64_t plane, int64_t o0) {
    const int lane = threadIdx.x & 63;
    constexpr int kWaves = kBlock / 64;
    constexpr int kSplit = kMfmaGridSplit<ENG>;
    constexpr int kRowsPerBlock = 32 / kSplit;
    // Workgroups are dealt to the 8 XCDs in turn; the kSplit parts of a row
    // block are numbered 8 apart so that they run on one XCD and fetch the
    // block's control points into one L2.  Numbers past the last block exit.
    const uint32_t xcd = blockIdx.x % 8, rest = blockIdx.x / 8;
    const uint32_t part = kSplit > 1 ? rest % kSplit : 0;
    const uint32_t bi = kSplit > 1 ? (rest / kSplit) * 8 + xcd : blockIdx.x;
    if (bi >= (n_patches + 31) / 32 * dim) return;
    const int a_begin = part * kRowsPerBlock + (threadIdx.x >> 6);  // then + kWaves, ...
    const int a_end = (part + 1) * kRowsPerBlock;
    const uint32_t g = bi / dim;     // block of 32 patches
    const uint32_t c = bi - g * dim;  // coordinate
    const uint32_t p0 = g * 32;
    const uint32_t n_valid = min(32u, n_patches - p0);
    const int col = lane & 31, kh = lane >> 5;
    const uint32_t prow = p0 + min(static_cast<uint32_t>(col), n_valid - 1);
    float A[16];
    const float4 *__restrict__ a4 =
        reinterpret_cast<const float4 *>(ctrl + (static_cast<size_t>(prow) * dim + c) * 16);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float4 v = a4[e];
        A[4 * e] = v.x;
        A[4 * e + 1] = v.y;
        A[4 * e + 2] = v.z;
        A[4 * e + 3] = v.w;
    }
    // cubic Bernstein basis at the 32 grid parameters j/31, once per workgroup
    __shared__ __align__(16) float tab[32 * 4];
    if (threadIdx.x < 32) {
        float B[4];
        bernstein_basis<3>(static_cast<float>(threadIdx.x) / 31.0f, B);
        *reinterpret_cast<float4 *>(tab + 4 * threadIdx.x) = make_float4(B[0], B[1], B[2], B[3]);
    }
    __syncthreads();
    float Bv[4];
    {
        const float4 v = *reinterpret_cast<const float4 *>(tab + 4 * col);
        Bv[0] = v.x;
        Bv[1] = v.y;
        Bv[2] = v.z;
        Bv[3] = v.w;
    }
    // accumulator row r of this lane is patch p0 + 8*(r/4) + 4*kh + r%4; its
    // points start (8*(r/4) + r%4) * 1024 floats after the lane's own base
    float *__restrict__ wb = out + static_cast<int64_t>(c) * plane + (o0 + p0) * 1024;
    const uint32_t lane_off = 4 * kh * 1024 + col;
    v8bf Ab;
    v8h Ah, Al;
    float unscale[16];
    if constexpr (ENG == MF_BF16) {
#pragma unroll
        for (int e = 0; e < 8; ++e) Ab[e] = static_cast<__bf16>(A[8 * kh + e]);
    } else if constexpr (ENG == MF_F16) {
#pragma unroll
        for (int e = 0; e < 8; ++e) Ah[e] = static_cast<_Float16>(A[8 * kh + e]);
    } else if constexpr (ENG == MF_F16X3) {
        float m = 0.0f;
#pragma unroll
        for (int e = 0; e < 16; ++e) m = __builtin_fmaxf(m, __builtin_fabsf(A[e]));
        int ex = 0;
        (void)__builtin_frexpf(m, &ex);  // m = f * 2^ex, f in [0.5, 1); m = 0 gives ex = 0
        const float sc = __builtin_ldexpf(1.0f, -ex);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float a = A[8 * kh + e] * sc;  // exact: power-of-two scale
            Ah[e] = static_cast<_Float16>(a);
            Al[e] = static_cast<_Float16>(a - static_cast<float>(Ah[e]));
        }
        // The scale of accumulator row j belongs to A row j, held by lane j.
        const float inv = __builtin_ldexpf(1.0f, ex);
#pragma unroll
        for (int r = 0; r < 16; ++r) unscale[r] = __shfl(inv, 8 * (r / 4) + 4 * kh + (r % 4));
    }
    for (int a = a_begin; a < a_end; a += kWaves) {
        float Bu[4];
        {
            const float4 v = *reinterpret_cast<const float4 *>(tab + 4 * a);
            Bu[0] = v.x;
            Bu[1] = v.y;
            Bu[2] = v.z;
            Bu[3] = v.w;
        }
        v16f acc = {};
        if constexpr (ENG == MF_F32) {
            // contract u on the vector ALU first: Q[p][j] = sum_i P[p][4i+j] Bu[a][i]
            // (lane: row p = col, j = 2s + kh), then the K = 4 product with the
            // v basis on the matrix cores -- two MFMAs per grid row, where the
            // Kronecker basis of u and v would take eight
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int j = 2 * s + kh;
                const float qa = __builtin_fmaf(A[12 + j], Bu[3], __builtin_fmaf(A[8 + j], Bu[2],
                                                __builtin_fmaf(A[4 + j], Bu[1], A[j] * Bu[0])));
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(qa, Bv[j], acc, 0, 0, 0);
            }
        } else if constexpr (ENG == MF_BF16) {
            v8bf Bb;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * kh + e;
                Bb[e] = static_cast<__bf16>(Bu[k >> 2] * Bv[k & 3]);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ab, Bb, acc, 0, 0, 0);
        } else if constexpr (ENG == MF_F16X3) {
            v8h Bh, Bl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * kh + e;
                const float b = Bu[k >> 2] * Bv[k & 3];
                Bh[e] = static_cast<_Float16>(b);
                Bl[e] = static_cast<_Float16>(b - static_cast<float>(Bh[e]));
            }
            // small terms first, so the high product is added last
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al, Bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, Bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, Bh, acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] *= unscale[r];
        } else {
            v8h Bh;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * kh + e;
                Bh[e] = static_cast<_Float16>(Bu[k >> 2] * Bv[k & 3]);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, Bh, acc, 0, 0, 0);
        }
        const uint32_t off = lane_off + a * 32;
        if (n_valid == 32) {
#pragma unroll
            for (int r = 0; r < 16; ++r) st_stream(wb + off + (8 * (r / 4) + r % 4) * 1024, acc[r]);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (8 * (r / 4) + 4 * kh + r % 4 < static_cast<int>(n_valid))
                    st_stream(wb + off + (8 * (r / 4) + r % 4) * 1024, acc[r]);
        }
    }
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" int bz_eval_tensor_patch(const void *ctrl, int dtype, int64_t n_obj, int du, int dv, int dw, int dim,
                                    const float *uvw, int64_t n_per, int nu, int nv, int engine, float *out,
                                    bz_stream stream) {
    return guarded("bz_eval_tensor_patch", [&]() -> int {
        const char *fn = "bz_eval_tensor_patch";
        if (du < 1 || du > 4 || dv < 1 || dv > 4 || dw < 0 || dw > 4)
            return fail(BZ_ERR_SHAPE, "%s: degrees (%d,%d,%d) outside 1..4 (dw 0..4)", fn, du, dv, dw);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_obj < 0) return fail(BZ_ERR_SHAPE, "%s: n_obj %lld", fn, (long long)n_obj);
        const int es = dtype_size(dtype);
        if (es == 0) return fail(BZ_ERR_DTYPE, "%s: dtype %d", fn, dtype);
        if (engine < BZ_TP_VALU || engine > BZ_TP_MFMA_F16X3) return fail(BZ_ERR_UNSUPPORTED, "%s: engine %d", fn, engine);
        const int ncp = (du + 1) * (dv + 1) * (dw + 1);
        const hipStream_t s = as_stream(stream);
        if (uvw == nullptr) {  // grid mode
            if (dw != 0) return fail(BZ_ERR_UNSUPPORTED, "%s: grid mode is for surfaces (dw = 0)", fn);
            if (nu < 1 || nv < 1 || static_cast<int64_t>(nu) * nv > (1 << 24))
                return fail(BZ_ERR_SHAPE, "%s: grid %d x %d", fn, nu, nv);
            if (engine != BZ_TP_VALU && (du != 3 || dv != 3 || nu != 32 || nv != 32 || dtype != BZ_F32))
                return fail(BZ_ERR_UNSUPPORTED, "%s: MFMA engines need bicubic FP32 patches on a 32x32 grid", fn);
            if (n_obj == 0) return BZ_OK;
            if (!ctrl || !out) return fail(BZ_ERR_NULL, "%s: ctrl and out are required", fn);
            if (!aligned(ctrl, engine == BZ_TP_VALU ? es : 16) || !aligned(out, 4))
                return fail(BZ_ERR_ALIGN, "%s: misaligned pointer (MFMA engines read ctrl as 16-byte rows)", fn);
            const int64_t npts = static_cast<int64_t>(nu) * nv;
            const int64_t plane = n_obj * npts;
            if (engine == BZ_TP_VALU) {
                const int64_t per = int64_t(1) << 22;
                for (int64_t o0 = 0; o0 < n_obj; o0 += per) {
                    const uint32_t blocks = static_cast<uint32_t>(std::min(per, n_obj - o0));
                    const char *c0 = static_cast<const char *>(ctrl) + o0 * dim * ncp * es;
                    if (dtype == BZ_F32) launch_grid<float, kBasisBernstein>(du, dv, dim, c0, nu, nv, out, plane, o0, blocks, s);
                    else if (dtype == BZ_F16) launch_grid<_Float16, kBasisBernstein>(du, dv, dim, c0, nu, nv, out, plane, o0, blocks, s);
                    else launch_grid<bf16_t, kBasisBernstein>(du, dv, dim, c0, nu, nv, out, plane, o0, blocks, s);
                    BZ_CHECK_LAUNCH("k_tensor_grid");
                }
            } else {
                const int64_t per = int64_t(1) << 22;  // patches per launch
                const uint32_t ud = static_cast<uint32_t>(dim);
                for (int64_t o0 = 0; o0 < n_obj; o0 += per) {
                    const uint32_t np = static_cast<uint32_t>(std::min(per, n_obj - o0));
                    // row blocks, rounded up to whole rounds of the 8 XCDs, times the engine's grid split
                    const uint32_t blocks = ((np + 31) / 32 * ud + 7) / 8 * 8;
                    const float *c0 = static_cast<const float *>(ctrl) + o0 * dim * 16;
                    if (engine == BZ_TP_MFMA_F32)
                        hipLaunchKernelGGL((k_tensor_mfma<MF_F32>), dim3(blocks * kMfmaGridSplit<MF_F32>), dim3(kBlock), 0, s,
                                           c0, np, ud, out, plane, o0);
                    else if (engine == BZ_TP_MFMA_BF16)
                        hipLaunchKernelGGL((k_tensor_mfma<MF_BF16>), dim3(blocks * kMfmaGridSplit<MF_BF16>), dim3(kBlock), 0,
                                           s, c0, np, ud, out, plane, o0);
                    else if (engine == BZ_TP_MFMA_F16)
                        hipLaunchKernelGGL((k_tensor_mfma<MF_F16>), dim3(blocks * kMfmaGridSplit<MF_F16>), dim3(kBlock), 0, s,
                                           c0, np, ud, out, plane, o0);
                    else
                        hipLaunchKernelGGL((k_tensor_mfma<MF_F16X3>), dim3(blocks * kMfmaGridSplit<MF_F16X3>), dim3(kBlock), 0,
                                           s, c0, np, ud, out, plane, o0);
                    BZ_CHECK_LAUNCH("k_tensor_mfma");
                }
            }
            return BZ_OK;
        }
        // points mode
        if (engine != BZ_TP_VALU) return fail(BZ_ERR_UNSUPPORTED, "%s: points mode runs on the VALU engine", fn);
        if (n_per < 0) return fail(BZ_ERR_SHAPE, "%s: n_per %lld", fn, (long long)n_per);
        if (n_obj == 0 || n_per == 0) return BZ_OK;
        if (!ctrl || !out) return fail(BZ_ERR_NULL, "%s: ctrl and out are required", fn);
        if (!aligned(ctrl, es) || !aligned(uvw, 4) || !aligned(out, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
        const int64_t plane = n_obj * n_per;
        const int64_t per = int64_t(1) << 22;
        for (int64_t o0 = 0; o0 < n_obj; o0 += per) {
            const uint32_t blocks = static_cast<uint32_t>(std::min(per, n_obj - o0));
            const char *c0 = static_cast<const char *>(ctrl) + o0 * dim * ncp * es;
            if (dtype == BZ_F32) launch_pts<float, kBasisBernstein>(du, dv, dw, dim, c0, uvw, n_per, out, plane, o0, blocks, s);
            else if (dtype == BZ_F16) launch_pts<_Float16, kBasisBernstein>(du, dv, dw, dim, c0, uvw, n_per, out, plane, o0, blocks, s);
            else launch_pts<bf16_t, kBasisBernstein>(du, dv, dw, dim, c0, uvw, n_per, out, plane, o0, blocks, s);
            BZ_CHECK_LAUNCH("k_tensor_points");
        }
        return BZ_OK;
    });
}
