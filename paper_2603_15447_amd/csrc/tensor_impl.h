// Separable tensor-product kernels shared by the Bernstein (tensor.hip) and
// per-axis Seiler (tensor_seiler.hip) evaluators of surfaces and volumes
// (Sec. 2.2: the order splits over the parameter axes).  The contraction is
// the same for both; only the per-axis basis differs.
//
//  k_tensor_grid   one patch per workgroup, nu x nv uniform grid.  When the
//                  block size is a multiple of nv every thread keeps one grid
//                  column b, contracts the net with the v basis once
//                  (isoline coefficients R_i(v_b)) and then needs only the u
//                  basis and du+1 FMAs per coordinate for each of its points;
//                  the u basis of each row (nu <= block size) comes from a
//                  table in LDS filled once per workgroup.
//  k_tensor_points one object per wavefront, random (u,v[,w]) per query,
//                  4 queries per lane, separable contraction w -> v -> u.
#pragma once
#include "curves_impl.h"

namespace bzi {
namespace {

// Per-axis basis: Bernstein for control points, or the Seiler basis for
// per-axis Seiler terms stored [b0, bd, d1, d_{d-1}, d2, ...] (Sec. 3): the
// Seiler recursion L(b0,bd,t) + st (L(d1,d_{d-1},t) + st (...)) is linear in
// the terms with coefficients 1-t, t, st(1-t), st t, (st)^2(1-t), ...,
// and (st)^(d/2) for the middle term of even degree.
enum { kBasisBernstein = 0, kBasisSeiler = 1 };

template <int D>
__device__ __forceinline__ void seiler_basis(float t, float (&B)[D + 1]) {
    const float s = 1.0f - t, st = s * t;
    B[0] = s;
    if constexpr (D >= 1) B[1] = t;
    float p = 1.0f;
#pragma unroll
    for (int i = 1; 2 * i + 1 <= D; ++i) {
        p *= st;
        B[2 * i] = p * s;
        B[2 * i + 1] = p * t;
    }
    if constexpr (D >= 2 && D % 2 == 0) {
        float m = 1.0f;
#pragma unroll
        for (int i = 0; i < D / 2; ++i) m *= st;
        B[D] = m;
    }
}

template <int D, int BASIS>
__device__ __forceinline__ void basis_at(float x, float (&B)[D + 1]) {
    if constexpr (BASIS == kBasisSeiler) seiler_basis<D>(x, B);
    else bernstein_basis<D>(x, B);
}

// ------------------------------------------------------------------ VALU grid
// Column-per-thread body of k_tensor_grid (nv divides the block size): each
// thread keeps grid column b, contracts the net with the v basis once and
// evaluates its points of that column with the u basis of their rows.  When nu <= block size the u
// basis of every row is computed once per workgroup into the LDS table tab_u
// (the divide and the basis cost more instructions than a row's FMAs and
// stores).  NU, NV > 0 fix the grid size at compile time: the row loop
// unrolls, with du = dv the column basis is a row of the same table, and each
// column is contracted once, by one thread, and shared with the other threads
// of that column through LDS; 0 takes nu, nv at run time.  Every variant evaluates the
// same basis at the same parameters a/(nu-1), b/(nv-1).
template <int DU, int DV, int DIM, typename T, int BASIS, int NU, int NV>
__device__ __forceinline__ void grid_columns(const T *__restrict__ P, int nu_rt, int nv_rt, float du_den, float dv_den,
                                             float *__restrict__ ob, int64_t plane, float *tab_u) {
    constexpr int NCP = (DU + 1) * (DV + 1);
    const int nu = NU > 0 ? NU : nu_rt;
    const int nv = NV > 0 ? NV : nv_rt;
    const int b = threadIdx.x % nv;
    const int a0 = threadIdx.x / nv;
    const int astep = kBlock / nv;
    const bool table = nu <= kBlock;
    if (table) {
        if (static_cast<int>(threadIdx.x) < nu) {
            float Bu[DU + 1];
            basis_at<DU, BASIS>(static_cast<float>(threadIdx.x) / du_den, Bu);
#pragma unroll
            for (int i = 0; i <= DU; ++i) tab_u[threadIdx.x * (DU + 1) + i] = Bu[i];
        }
        __syncthreads();
    }
    // isoline coefficients of column b: R[c][i] = sum_j Bv_j(b) P[c][i][j]
    auto contract = [&](float (&R)[DIM][DU + 1]) {
        float Bv[DV + 1];
        if constexpr (NU > 0 && NU == NV && DU == DV) {
#pragma unroll
            for (int j = 0; j <= DV; ++j) Bv[j] = tab_u[b * (DU + 1) + j];
        } else {
            basis_at<DV, BASIS>(static_cast<float>(b) / dv_den, Bv);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int i = 0; i <= DU; ++i) {
                float acc = Bv[0] * to_f32<T>(P[c * NCP + i * (DV + 1)]);
#pragma unroll
                for (int j = 1; j <= DV; ++j)
                    acc = __builtin_fmaf(Bv[j], to_f32<T>(P[c * NCP + i * (DV + 1) + j]), acc);
                R[c][i] = acc;
            }
    };
    float R[DIM][DU + 1];
    if constexpr (NU > 0) {
        static_assert(NU <= kBlock && NU % (kBlock / NV) == 0, "fixed grids fill whole row steps");
        // the first NV threads contract one column each; the kBlock / NV
        // threads of a column share it through LDS
        __shared__ __align__(16) float tab_r[NV * DIM * (DU + 1)];
        if (static_cast<int>(threadIdx.x) < NV) {
            float Rc[DIM][DU + 1];
            contract(Rc);
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int i = 0; i <= DU; ++i) tab_r[(b * DIM + c) * (DU + 1) + i] = Rc[c][i];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int i = 0; i <= DU; ++i) R[c][i] = tab_r[(b * DIM + c) * (DU + 1) + i];
        const uint32_t lo = static_cast<uint32_t>(a0 * NV + b);
#pragma unroll
        for (int k = 0; k < NU / (kBlock / NV); ++k) {
            const int a = a0 + k * (kBlock / NV);
            float Bu[DU + 1];
#pragma unroll
            for (int i = 0; i <= DU; ++i) Bu[i] = tab_u[a * (DU + 1) + i];
#pragma unroll
            for (int c = 0; c < DIM; ++c) st_stream(ob + c * plane + (lo + k * kBlock), dot_basis<DU>(Bu, R[c]));
        }
        return;
    }
    contract(R);
    float *__restrict__ oc = ob + a0 * nv + b;
    if (table) {
        for (int a = a0; a < nu; a += astep, oc += kBlock) {
            float Bu[DU + 1];
#pragma unroll
            for (int i = 0; i <= DU; ++i) Bu[i] = tab_u[a * (DU + 1) + i];
#pragma unroll
            for (int c = 0; c < DIM; ++c) st_stream(oc + c * plane, dot_basis<DU>(Bu, R[c]));
        }
    } else {
        for (int a = a0; a < nu; a += astep, oc += kBlock) {
            float Bu[DU + 1];
            basis_at<DU, BASIS>(static_cast<float>(a) / du_den, Bu);
#pragma unroll
            for (int c = 0; c < DIM; ++c) st_stream(oc + c * plane, dot_basis<DU>(Bu, R[c]));
        }
    }
}

template <int DU, int DV, int DIM, typename T, int BASIS>
__global__ __launch_bounds__(kBlock) void k_tensor_grid(const T *__restrict__ ctrl, int nu, int nv,
                                                        float *__restrict__ out, int64_t plane, int64_t o0) {
    constexpr int NCP = (DU + 1) * (DV + 1);
    const uint32_t o = blockIdx.x;
    const T *__restrict__ P = ctrl + static_cast<size_t>(o) * DIM * NCP;
    const int npts = nu * nv;
    float *__restrict__ ob = out + (o0 + o) * static_cast<int64_t>(npts);
    const float du_den = nu > 1 ? static_cast<float>(nu - 1) : 1.0f;
    const float dv_den = nv > 1 ? static_cast<float>(nv - 1) : 1.0f;
    __shared__ __align__(16) float tab_u[kBlock * (DU + 1)];
    if (kBlock % nv == 0) {
        if (nu == 32 && nv == 32) grid_columns<DU, DV, DIM, T, BASIS, 32, 32>(P, nu, nv, du_den, dv_den, ob, plane, tab_u);
        else grid_columns<DU, DV, DIM, T, BASIS, 0, 0>(P, nu, nv, du_den, dv_den, ob, plane, tab_u);
    } else {
        for (int p = threadIdx.x; p < npts; p += kBlock) {
            const int a = p / nv, b = p - (p / nv) * nv;
            float Bu[DU + 1], Bv[DV + 1];
            basis_at<DU, BASIS>(static_cast<float>(a) / du_den, Bu);
            basis_at<DV, BASIS>(static_cast<float>(b) / dv_den, Bv);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                float Ri[DU + 1];
#pragma unroll
                for (int i = 0; i <= DU; ++i) {
                    float acc = Bv[0] * to_f32<T>(P[c * NCP + i * (DV + 1)]);
#pragma unroll
                    for (int j = 1; j <= DV; ++j)
                        acc = __builtin_fmaf(Bv[j], to_f32<T>(P[c * NCP + i * (DV + 1) + j]), acc);
                    Ri[i] = acc;
                }
                st_stream(ob + c * plane + p, dot_basis<DU>(Bu, Ri));
            }
        }
    }
}

// ------------------------------------------------------------------ VALU points
// One wavefront per object, 4 queries per lane at a time: the object's
// control points are wave-uniform (scalar loads into SGPRs) and each one
// feeds the FMAs of 4 queries.  Separable contraction w -> v -> u.
constexpr int kPtsQ = 4;

template <int DU, int DV, int DW, int DIM, typename T, int BASIS>
__global__ __launch_bounds__(kBlock) void k_tensor_points(const T *__restrict__ ctrl, const float *__restrict__ uvw,
                                                          int64_t n_per, uint32_t n_obj, float *__restrict__ out,
                                                          int64_t plane, int64_t o0) {
    constexpr int NCP = (DU + 1) * (DV + 1) * (DW + 1);
    constexpr int NPAR = DW > 0 ? 3 : 2;
    const uint32_t o = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (o >= n_obj) return;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ P = ctrl + static_cast<size_t>(o) * DIM * NCP;
    for (int64_t j0 = 0; j0 < n_per; j0 += 64 * kPtsQ) {
        float Bu[kPtsQ][DU + 1], Bv[kPtsQ][DV + 1], Bw[kPtsQ][DW + 1];
        int64_t q[kPtsQ];
        bool ok[kPtsQ];
#pragma unroll
        for (int s = 0; s < kPtsQ; ++s) {
            const int64_t j = j0 + s * 64 + lane;
            ok[s] = j < n_per;
            q[s] = (o0 + o) * n_per + (ok[s] ? j : n_per - 1);
            const float *__restrict__ p = uvw + q[s] * NPAR;
            basis_at<DU, BASIS>(p[0], Bu[s]);
            basis_at<DV, BASIS>(p[1], Bv[s]);
            if constexpr (DW > 0) basis_at<DW, BASIS>(p[2], Bw[s]);
            else Bw[s][0] = 1.0f;
        }
        // One (coordinate, i) slab of (DV+1)(DW+1) coefficients at a time: the
        // slab loop is not unrolled, so the scalar loads of one slab are in
        // flight while the previous slab's FMAs run, and the coefficients never
        // outnumber the scalar registers (a fully unrolled nest would hoist all
        // DIM * NCP loads and spill them into vector-register lanes).
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            float acc[kPtsQ] = {};
#pragma unroll 1
            for (int i = 0; i <= DU; ++i) {
                float Ri[kPtsQ] = {};
#pragma unroll
                for (int jj = 0; jj <= DV; ++jj) {
                    float Qj[kPtsQ] = {};
#pragma unroll
                    for (int k = 0; k <= DW; ++k) {
                        const float pv = to_f32<T>(P[c * NCP + (i * (DV + 1) + jj) * (DW + 1) + k]);
#pragma unroll
                        for (int s = 0; s < kPtsQ; ++s) Qj[s] = __builtin_fmaf(Bw[s][k], pv, Qj[s]);
                    }
#pragma unroll
                    for (int s = 0; s < kPtsQ; ++s) Ri[s] = __builtin_fmaf(Bv[s][jj], Qj[s], Ri[s]);
                }
#pragma unroll
                for (int s = 0; s < kPtsQ; ++s) acc[s] = __builtin_fmaf(Bu[s][i], Ri[s], acc[s]);
            }
#pragma unroll
            for (int s = 0; s < kPtsQ; ++s)
                if (ok[s]) st_stream(out + c * plane + q[s], acc[s]);
        }
    }
}

// ------------------------------------------------------------------ MFMA grid

// ------------------------------------------------------------------ dispatch (over degrees and dim)
template <typename T, int BASIS, int DU, int DV, int DIM>
void launch_grid3(const void *ctrl, int nu, int nv, float *out, int64_t plane, int64_t o0, uint32_t blocks,
                  hipStream_t s) {
    hipLaunchKernelGGL((k_tensor_grid<DU, DV, DIM, T, BASIS>), dim3(blocks), dim3(kBlock), 0, s,
                       static_cast<const T *>(ctrl), nu, nv, out, plane, o0);
}

template <typename T, int BASIS, int DU, int DV>
int launch_grid2(int dim, const void *ctrl, int nu, int nv, float *out, int64_t plane, int64_t o0, uint32_t blocks,
                 hipStream_t s) {
    switch (dim) {
        case 1: launch_grid3<T, BASIS, DU, DV, 1>(ctrl, nu, nv, out, plane, o0, blocks, s); break;
        case 2: launch_grid3<T, BASIS, DU, DV, 2>(ctrl, nu, nv, out, plane, o0, blocks, s); break;
        case 3: launch_grid3<T, BASIS, DU, DV, 3>(ctrl, nu, nv, out, plane, o0, blocks, s); break;
        default: launch_grid3<T, BASIS, DU, DV, 4>(ctrl, nu, nv, out, plane, o0, blocks, s); break;
    }
    return BZ_OK;
}

template <typename T, int BASIS, int DU>
int launch_grid1(int dv, int dim, const void *ctrl, int nu, int nv, float *out, int64_t plane, int64_t o0,
                 uint32_t blocks, hipStream_t s) {
    switch (dv) {
        case 1: return launch_grid2<T, BASIS, DU, 1>(dim, ctrl, nu, nv, out, plane, o0, blocks, s);
        case 2: return launch_grid2<T, BASIS, DU, 2>(dim, ctrl, nu, nv, out, plane, o0, blocks, s);
        case 3: return launch_grid2<T, BASIS, DU, 3>(dim, ctrl, nu, nv, out, plane, o0, blocks, s);
        default: return launch_grid2<T, BASIS, DU, 4>(dim, ctrl, nu, nv, out, plane, o0, blocks, s);
    }
}

template <typename T, int BASIS>
int launch_grid(int du, int dv, int dim, const void *ctrl, int nu, int nv, float *out, int64_t plane, int64_t o0,
                uint32_t blocks, hipStream_t s) {
    switch (du) {
        case 1: return launch_grid1<T, BASIS, 1>(dv, dim, ctrl, nu, nv, out, plane, o0, blocks, s);
        case 2: return launch_grid1<T, BASIS, 2>(dv, dim, ctrl, nu, nv, out, plane, o0, blocks, s);
        case 3: return launch_grid1<T, BASIS, 3>(dv, dim, ctrl, nu, nv, out, plane, o0, blocks, s);
        default: return launch_grid1<T, BASIS, 4>(dv, dim, ctrl, nu, nv, out, plane, o0, blocks, s);
    }
}

template <typename T, int BASIS, int DU, int DV, int DW>
int launch_pts3(int dim, const void *ctrl, const float *uvw, int64_t n_per, float *out, int64_t plane, int64_t o0,
                uint32_t n_obj, hipStream_t s) {
    const T *p = static_cast<const T *>(ctrl);
    const uint32_t blocks = (n_obj + kBlock / 64 - 1) / (kBlock / 64);
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_tensor_points<DU, DV, DW, 1, T, BASIS>), dim3(blocks), dim3(kBlock), 0, s, p, uvw, n_per, n_obj, out, plane, o0); break;
        case 2: hipLaunchKernelGGL((k_tensor_points<DU, DV, DW, 2, T, BASIS>), dim3(blocks), dim3(kBlock), 0, s, p, uvw, n_per, n_obj, out, plane, o0); break;
        case 3: hipLaunchKernelGGL((k_tensor_points<DU, DV, DW, 3, T, BASIS>), dim3(blocks), dim3(kBlock), 0, s, p, uvw, n_per, n_obj, out, plane, o0); break;
        default: hipLaunchKernelGGL((k_tensor_points<DU, DV, DW, 4, T, BASIS>), dim3(blocks), dim3(kBlock), 0, s, p, uvw, n_per, n_obj, out, plane, o0); break;
    }
    return BZ_OK;
}

template <typename T, int BASIS, int DU, int DV>
int launch_pts2(int dw, int dim, const void *ctrl, const float *uvw, int64_t n_per, float *out, int64_t plane,
                int64_t o0, uint32_t blocks, hipStream_t s) {
    switch (dw) {
        case 0: return launch_pts3<T, BASIS, DU, DV, 0>(dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 1: return launch_pts3<T, BASIS, DU, DV, 1>(dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 2: return launch_pts3<T, BASIS, DU, DV, 2>(dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 3: return launch_pts3<T, BASIS, DU, DV, 3>(dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        default: return launch_pts3<T, BASIS, DU, DV, 4>(dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
    }
}

template <typename T, int BASIS, int DU>
int launch_pts1(int dv, int dw, int dim, const void *ctrl, const float *uvw, int64_t n_per, float *out, int64_t plane,
                int64_t o0, uint32_t blocks, hipStream_t s) {
    switch (dv) {
        case 1: return launch_pts2<T, BASIS, DU, 1>(dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 2: return launch_pts2<T, BASIS, DU, 2>(dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 3: return launch_pts2<T, BASIS, DU, 3>(dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        default: return launch_pts2<T, BASIS, DU, 4>(dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
    }
}

template <typename T, int BASIS>
int launch_pts(int du, int dv, int dw, int dim, const void *ctrl, const float *uvw, int64_t n_per, float *out,
               int64_t plane, int64_t o0, uint32_t blocks, hipStream_t s) {
    switch (du) {
        case 1: return launch_pts1<T, BASIS, 1>(dv, dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 2: return launch_pts1<T, BASIS, 2>(dv, dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        case 3: return launch_pts1<T, BASIS, 3>(dv, dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
        default: return launch_pts1<T, BASIS, 4>(dv, dw, dim, ctrl, uvw, n_per, out, plane, o0, blocks, s);
    }
}

}  // namespace
}  // namespace bzi
