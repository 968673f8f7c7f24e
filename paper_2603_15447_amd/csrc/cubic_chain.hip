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

// ------------------------------------------------------------------ tiled
// Cache-line tiles of the cubic chain.  Both layers share the on-path texel
// A_k, so a column is stored once as [A_k, x0_k, x1_k] (3*dim floats: the
// endpoint and the two layers' free texels; the row parity is implied by k
// and the diagonal read A s^2 + (x_k + x_k+1) s t + A' t^2 is symmetric in
// the two free texels).  A 128-byte tile holds C = 32/(3*dim) consecutive
// columns, consecutive tiles overlapping by one, so tile j holds segments
// [jS, jS+S) with S = C-1 and a segment's window is one line: 3D gives two
// segments per 128-byte tile (64 MB for 2^20 segments, one line per query,
// against 1.6 lines per query in the two-layer grid).
template <int DIM>
struct CubicTileGeom {
    static constexpr int W = 3 * DIM;    // floats per column
    static constexpr int C = 32 / W;     // columns per tile
    static constexpr int S = C - 1;      // segments per tile
};

int cubic_tile_segs(int dim) { return 32 / (3 * dim) - 1; }

__global__ __launch_bounds__(kBlock) void k_tile_cubic(const float *__restrict__ grid, int64_t n_seg, int dim,
                                                       int segs, int64_t n_tiles, float *__restrict__ tiles) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_tiles * 32) return;
    const int64_t j = i >> 5;
    const int f = static_cast<int>(i & 31);
    const int w = 3 * dim;
    const int c = f / w, within = f - c * w;
    const int part = within / dim, ch = within - part * dim;  // part 0: A, 1: x0, 2: x1
    const int64_t col = j * segs + c;
    float v = 0.0f;
    if (c <= segs && col <= n_seg) {
        const int r = static_cast<int>(col & 1);
        const int layer = part == 2 ? 1 : 0;
        const int row = part == 0 ? r : 1 - r;
        v = grid[((col * 2 + layer) * 2 + row) * dim + ch];
    }
    tiles[i] = v;
}

template <int DIM, int QPT>
__global__ __launch_bounds__(kBlock) void k_piecewise_cubic_eval_tiled(const float *__restrict__ tiles, uint32_t n_seg,
                                                                       const float *__restrict__ T, uint32_t nq,
                                                                       float *__restrict__ out, int64_t plane) {
    typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
    constexpr int W = CubicTileGeom<DIM>::W, S = CubicTileGeom<DIM>::S;
    constexpr int NW = 2 * W;  // floats in a segment's window
    const uint32_t base = blockIdx.x * (kBlock * QPT) + threadIdx.x;
    const float nf = static_cast<float>(n_seg);
    const float nm1 = static_cast<float>(n_seg - 1);
    float tl[QPT];
    uint32_t off[QPT];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
        const float Tq = ld_stream(T + q);
        float Tc = Tq < 0.0f ? 0.0f : Tq;
        Tc = Tc > nf ? nf : Tc;
        const float kf = __builtin_fminf(__builtin_floorf(Tc), nm1);
        const uint32_t k = min(static_cast<uint32_t>(kf), n_seg - 1);
        const uint32_t j = k / S, r = k - j * S;
        off[i] = j * 32 + r * W;
        tl[i] = Tc - static_cast<float>(k);
    }
    float f[QPT][NW];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const float *__restrict__ p = tiles + off[i];
#pragma unroll
        for (int e = 0; e < NW / 4; ++e) {
            const f4u x = *reinterpret_cast<const f4u *>(p + 4 * e);
            f[i][4 * e] = x[0], f[i][4 * e + 1] = x[1], f[i][4 * e + 2] = x[2], f[i][4 * e + 3] = x[3];
        }
#pragma unroll
        for (int e = 4 * (NW / 4); e < NW; ++e) f[i][e] = p[e];
    }
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const float t = tl[i];
        const uint32_t q = min(base + i * kBlock, nq - 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float A = f[i][c], A1 = f[i][W + c];
            const float v0 = lerp(lerp(A, f[i][W + DIM + c], t), lerp(f[i][DIM + c], A1, t), t);
            const float v1 = lerp(lerp(A, f[i][W + 2 * DIM + c], t), lerp(f[i][2 * DIM + c], A1, t), t);
            st_stream(out + c * plane + q, lerp(v0, v1, t));
        }
    }
}

template <int DIM>
int launch_cubic_eval_tiled(const float *tiles, uint32_t n_seg, const float *T, uint32_t nq, float *out,
                            int64_t plane, hipStream_t s) {
    constexpr int Q = 4;
    const uint32_t blocks = (nq + kBlock * Q - 1) / (kBlock * Q);
    hipLaunchKernelGGL((k_piecewise_cubic_eval_tiled<DIM, Q>), dim3(blocks), dim3(kBlock), 0, s, tiles, n_seg, T, nq,
                       out, plane);
    BZ_CHECK_LAUNCH("k_piecewise_cubic_eval_tiled");
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

int64_t bz_piecewise_cubic_tiled_floats(int64_t n_seg, int dim) {
    if (n_seg < 1 || dim < 1 || dim > kMaxDim) return 0;
    const int64_t segs = cubic_tile_segs(dim);
    return (n_seg + segs - 1) / segs * 32;
}

int bz_tile_piecewise_cubic(const float *grid, int64_t n_seg, int dim, float *tiles, bz_stream stream) {
    return guarded("bz_tile_piecewise_cubic", [&]() -> int {
        const char *fn = "bz_tile_piecewise_cubic";
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_seg < 1 || n_seg > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_seg not in 1..2^31", fn);
        if (!grid || !tiles) return fail(BZ_ERR_NULL, "%s: grid and tiles are required", fn);
        if (!aligned(grid, 4) || !aligned(tiles, 16)) return fail(BZ_ERR_ALIGN, "%s: tiles need 16-byte alignment", fn);
        const int segs = cubic_tile_segs(dim);
        const int64_t n_tiles = (n_seg + segs - 1) / segs;
        const int64_t total = n_tiles * 32;
        const uint32_t blocks = static_cast<uint32_t>((total + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_tile_cubic, dim3(blocks), dim3(kBlock), 0, as_stream(stream), grid, n_seg, dim, segs,
                           n_tiles, tiles);
        BZ_CHECK_LAUNCH("k_tile_cubic");
        return BZ_OK;
    });
}

int bz_eval_piecewise_cubic_tiled(const float *tiles, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                                  bz_stream stream) {
    return guarded("bz_eval_piecewise_cubic_tiled", [&]() -> int {
        const char *fn = "bz_eval_piecewise_cubic_tiled";
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_q < 0) return fail(BZ_ERR_SHAPE, "%s: n_q", fn);
        if (n_seg < 1 || n_seg > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_seg not in 1..2^31", fn);
        if (n_q == 0) return BZ_OK;
        if (!tiles || !T || !out) return fail(BZ_ERR_NULL, "%s: tiles, T and out are required", fn);
        if (!aligned(tiles, 16) || !aligned(T, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "%s: tiles need 16-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const int64_t per = int64_t(1) << 30;
        for (int64_t q0 = 0; q0 < n_q; q0 += per) {
            const uint32_t nq = static_cast<uint32_t>(std::min(per, n_q - q0));
            const uint32_t ns = static_cast<uint32_t>(n_seg);
            int rc;
            switch (dim) {
                case 1: rc = launch_cubic_eval_tiled<1>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
                case 2: rc = launch_cubic_eval_tiled<2>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
                case 3: rc = launch_cubic_eval_tiled<3>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
                default: rc = launch_cubic_eval_tiled<4>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
            }
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

}  // extern "C"
