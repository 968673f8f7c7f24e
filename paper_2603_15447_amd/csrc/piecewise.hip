// C0 piecewise quadratic chains in the shared-diagonal ("zig-zag") encoding
// (Sec. 2.1, Eq. 1-2, Fig. 2): random-access evaluators of the grid and of
// its cache-line-tiled placement.  The encoder is in chain_encode.hip.
//
// Grid layout in HBM: grid[n_seg+1][2][dim] FP32, one 2*dim*4-byte column per
// chain vertex, so segment k reads one contiguous 16*dim-byte window (columns
// k and k+1).  The evaluator is a gather: each thread takes QPT queries, issues
// all their parameter loads, then all their window loads (8-byte vector loads,
// cached: the grid is re-read by many queries), then evaluates and streams the
// results out with non-temporal stores so they do not evict the grid from the
// L2 and the Infinity Cache.
#include <cstdlib>

#include "common.h"

namespace bzi {
namespace {

template <int DIM, int QPT>
__global__ __launch_bounds__(kBlock) void k_piecewise_eval(const float *__restrict__ grid, uint32_t n_seg,
                                                           const float *__restrict__ T, uint32_t nq,
                                                           float *__restrict__ out, int64_t plane) {
    const uint32_t base = blockIdx.x * (kBlock * QPT) + threadIdx.x;
    const float nf = static_cast<float>(n_seg);
    const float nm1 = static_cast<float>(n_seg - 1);
    // No branches: tail lanes (q >= nq) redo query nq-1 and store the same
    // value to the same place, so every query's gather stays in flight at once.
    float tl[QPT];
    uint32_t kk[QPT];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
        const float Tq = ld_stream(T + q);
        float Tc = Tq < 0.0f ? 0.0f : Tq;  // NaN passes both clamps
        Tc = Tc > nf ? nf : Tc;
        const float kf = __builtin_fminf(__builtin_floorf(Tc), nm1);  // NaN -> n_seg-1
        const uint32_t k = min(static_cast<uint32_t>(kf), n_seg - 1);
        kk[i] = k;
        tl[i] = Tc - static_cast<float>(k);
    }
    // Window of segment k: columns k and k+1, 4*DIM floats, 8-byte aligned.
    float2 g[QPT][2 * DIM];
    const float2 *__restrict__ g2 = reinterpret_cast<const float2 *>(grid);
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
        for (int j = 0; j < 2 * DIM; ++j) g[i][j] = g2[static_cast<size_t>(kk[i]) * DIM + j];
    float v[QPT][DIM];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        float f[4 * DIM];
#pragma unroll
        for (int j = 0; j < 2 * DIM; ++j) {
            f[2 * j] = g[i][j].x;
            f[2 * j + 1] = g[i][j].y;
        }
        const bool odd = kk[i] & 1;
        const float t = tl[i];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float c0r0 = f[c], c0r1 = f[DIM + c], c1r0 = f[2 * DIM + c], c1r1 = f[3 * DIM + c];
            // on-path texels A_k (row k mod 2 of column k) and A_{k+1}; off-path x_k, x_{k+1}
            const float A = odd ? c0r1 : c0r0, xk = odd ? c0r0 : c0r1;
            const float xk1 = odd ? c1r1 : c1r0, A1 = odd ? c1r0 : c1r1;
            // bilinear read along the diagonal: L(L(A, x_{k+1}), L(x_k, A_{k+1})) (Eq. 1)
            v[i][c] = lerp(lerp(A, xk1, t), lerp(xk, A1, t), t);
        }
    }
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) st_stream(out + c * plane + q, v[i][c]);
    }
}

// ------------------------------------------------------------------ tiled
// Cache-line tiling of the zig-zag grid: 128-byte tiles of C = 128/(8*dim)
// consecutive columns, consecutive tiles overlapping by one column, so tile j
// holds the S = C-1 segments [jS, jS+S) and every segment's 2x2 window lies in
// one 128-byte line (as a texture is stored in cache-line tiles).  The texels
// are those of the zig-zag grid; only their placement differs.
template <int DIM>
struct TileGeom {
    static constexpr int C = 128 / (8 * DIM);  // columns per tile
    static constexpr int S = C - 1;            // segments per tile
};

__global__ __launch_bounds__(kBlock) void k_tile_grid(const float *__restrict__ grid, int64_t n_seg, int dim, int cols,
                                                      int segs, int64_t n_tiles, float *__restrict__ tiles) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_tiles * 32) return;
    const int64_t j = i >> 5;
    const int f = static_cast<int>(i & 31);
    const int c = f / (2 * dim), within = f - c * 2 * dim;
    const int64_t col = j * segs + c;
    tiles[i] = (c < cols && col <= n_seg) ? grid[col * 2 * dim + within] : 0.0f;
}

template <int DIM, int QPT>
__global__ __launch_bounds__(kBlock) void k_piecewise_eval_tiled(const float *__restrict__ tiles, uint32_t n_seg,
                                                                 const float *__restrict__ T, uint32_t nq,
                                                                 float *__restrict__ out, int64_t plane) {
    constexpr int S = TileGeom<DIM>::S;
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
    float2 g[QPT][2 * DIM];
    const float2 *__restrict__ g2 = reinterpret_cast<const float2 *>(tiles);
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t j = kk[i] / S, r = kk[i] - j * S;
        const size_t off = static_cast<size_t>(j) * 16 + r * DIM;  // in float2 units
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) g[i][e] = g2[off + e];
    }
    float v[QPT][DIM];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        float f[4 * DIM];
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) {
            f[2 * e] = g[i][e].x;
            f[2 * e + 1] = g[i][e].y;
        }
        const bool odd = kk[i] & 1;
        const float t = tl[i];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float c0r0 = f[c], c0r1 = f[DIM + c], c1r0 = f[2 * DIM + c], c1r1 = f[3 * DIM + c];
            const float A = odd ? c0r1 : c0r0, xk = odd ? c0r0 : c0r1;
            const float xk1 = odd ? c1r1 : c1r0, A1 = odd ? c1r0 : c1r1;
            v[i][c] = lerp(lerp(A, xk1, t), lerp(xk, A1, t), t);
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
int launch_eval_tiled(const float *tiles, uint32_t n_seg, const float *T, uint32_t nq, float *out, int64_t plane,
                      hipStream_t s) {
    constexpr int Q = 4;
    const uint32_t per_block = kBlock * Q;
    const uint32_t blocks = (nq + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_piecewise_eval_tiled<DIM, Q>), dim3(blocks), dim3(kBlock), 0, s, tiles, n_seg, T, nq, out,
                       plane);
    BZ_CHECK_LAUNCH("k_piecewise_eval_tiled");
    return BZ_OK;
}

int tile_segs(int dim) { return 128 / (8 * dim) - 1; }

// ------------------------------------------------- 16-bit texel tiles
// The same cache-line tiling with FP16 or BF16 texels: 128-byte tiles of
// C = 32/dim columns (32, 16, 10, 8 for dim 1..4), S = C-1 segments each, so
// the tiled chain takes 2-2.25x fewer bytes and every query still reads one
// line.  Texels are the FP32 grid's, rounded to nearest even once.
int tile_segs16(int dim) { return 32 / dim - 1; }

template <typename T>
__device__ __forceinline__ uint16_t f32_to_bits16(float x);
template <>
__device__ __forceinline__ uint16_t f32_to_bits16<_Float16>(float x) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
}
template <>
__device__ __forceinline__ uint16_t f32_to_bits16<bf16_t>(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);  // NaN stays NaN
    return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);                // round to nearest even
}

template <typename T>
__device__ __forceinline__ float bits16_to_f32(uint32_t b) {
    if constexpr (std::is_same<T, _Float16>::value)
        return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(b)));
    else
        return __uint_as_float(b << 16);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_grid16(const float *__restrict__ grid, int64_t n_seg, int dim, int cols,
                                                        int segs, int64_t n_tiles, uint16_t *__restrict__ tiles) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_tiles * 64) return;
    const int64_t j = i >> 6;
    const int f = static_cast<int>(i & 63);
    const int c = f / (2 * dim), within = f - c * 2 * dim;
    const int64_t col = j * segs + c;
    tiles[i] = (c < cols && col <= n_seg) ? f32_to_bits16<T>(grid[col * 2 * dim + within]) : uint16_t(0);
}

// As k_piecewise_eval_tiled; a segment's window (two columns of 2*DIM
// texels, 8*DIM bytes at a 4-byte aligned offset) comes in 2*DIM 4-byte loads.
template <int DIM, typename H, int QPT>
__global__ __launch_bounds__(kBlock) void k_piecewise_eval_tiled16(const uint16_t *__restrict__ tiles, uint32_t n_seg,
                                                                   const float *__restrict__ T, uint32_t nq,
                                                                   float *__restrict__ out, int64_t plane) {
    constexpr int S = 32 / DIM - 1;
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
    uint32_t g[QPT][2 * DIM];
    const uint32_t *__restrict__ g32 = reinterpret_cast<const uint32_t *>(tiles);
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t j = kk[i] / S, r = kk[i] - j * S;
        const size_t off = static_cast<size_t>(j) * 32 + r * DIM;  // in 4-byte units
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) g[i][e] = g32[off + e];
    }
    float v[QPT][DIM];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        float f[4 * DIM];
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) {
            f[2 * e] = bits16_to_f32<H>(g[i][e] & 0xffffu);
            f[2 * e + 1] = bits16_to_f32<H>(g[i][e] >> 16);
        }
        const bool odd = kk[i] & 1;
        const float t = tl[i];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float c0r0 = f[c], c0r1 = f[DIM + c], c1r0 = f[2 * DIM + c], c1r1 = f[3 * DIM + c];
            const float A = odd ? c0r1 : c0r0, xk = odd ? c0r0 : c0r1;
            const float xk1 = odd ? c1r1 : c1r0, A1 = odd ? c1r0 : c1r1;
            v[i][c] = lerp(lerp(A, xk1, t), lerp(xk, A1, t), t);
        }
    }
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) st_stream(out + c * plane + q, v[i][c]);
    }
}

template <int DIM, typename H>
int launch_eval_tiled16(const uint16_t *tiles, uint32_t n_seg, const float *Tp, uint32_t nq, float *out, int64_t plane,
                        hipStream_t s) {
    constexpr int Q = 4;
    const uint32_t per_block = kBlock * Q;
    const uint32_t blocks = (nq + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_piecewise_eval_tiled16<DIM, H, Q>), dim3(blocks), dim3(kBlock), 0, s, tiles, n_seg, Tp, nq,
                       out, plane);
    BZ_CHECK_LAUNCH("k_piecewise_eval_tiled16");
    return BZ_OK;
}

template <typename T>
int eval_tiled16_dim(int dim, const uint16_t *tiles, uint32_t ns, const float *Tp, uint32_t nq, float *out,
                     int64_t plane, hipStream_t s) {
    switch (dim) {
        case 1: return launch_eval_tiled16<1, T>(tiles, ns, Tp, nq, out, plane, s);
        case 2: return launch_eval_tiled16<2, T>(tiles, ns, Tp, nq, out, plane, s);
        case 3: return launch_eval_tiled16<3, T>(tiles, ns, Tp, nq, out, plane, s);
        default: return launch_eval_tiled16<4, T>(tiles, ns, Tp, nq, out, plane, s);
    }
}

// Queries per thread; BZ_PIECEWISE_QPT (1, 2, 4 or 8) overrides the default.
int piecewise_qpt() {
    static const int q = [] {
        const char *e = getenv("BZ_PIECEWISE_QPT");
        const int v = e ? atoi(e) : 4;
        return (v == 1 || v == 2 || v == 4 || v == 8) ? v : 4;
    }();
    return q;
}

template <int DIM, int QPT>
int launch_eval_q(const float *grid, uint32_t n_seg, const float *T, uint32_t nq, float *out, int64_t plane,
                  hipStream_t s) {
    const uint32_t per_block = kBlock * QPT;
    const uint32_t blocks = (nq + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_piecewise_eval<DIM, QPT>), dim3(blocks), dim3(kBlock), 0, s, grid, n_seg, T, nq, out, plane);
    BZ_CHECK_LAUNCH("k_piecewise_eval");
    return BZ_OK;
}

template <int DIM>
int launch_eval(const float *grid, uint32_t n_seg, const float *T, uint32_t nq, float *out, int64_t plane,
                hipStream_t s) {
    switch (piecewise_qpt()) {
        case 1: return launch_eval_q<DIM, 1>(grid, n_seg, T, nq, out, plane, s);
        case 2: return launch_eval_q<DIM, 2>(grid, n_seg, T, nq, out, plane, s);
        case 8: return launch_eval_q<DIM, 8>(grid, n_seg, T, nq, out, plane, s);
        default: return launch_eval_q<DIM, 4>(grid, n_seg, T, nq, out, plane, s);
    }
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

int bz_eval_piecewise(const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                      bz_stream stream) {
    return guarded("bz_eval_piecewise", [&]() -> int {
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "bz_eval_piecewise: dim %d", dim);
        if (n_q < 0) return fail(BZ_ERR_SHAPE, "bz_eval_piecewise: n_q %lld", (long long)n_q);
        if (n_seg < 1 || n_seg > (int64_t(1) << 31))
            return fail(BZ_ERR_SHAPE, "bz_eval_piecewise: n_seg %lld not in 1..2^31", (long long)n_seg);
        if (n_q == 0) return BZ_OK;
        if (!grid || !T || !out) return fail(BZ_ERR_NULL, "bz_eval_piecewise: grid, T and out are required");
        if (!aligned(grid, 8) || !aligned(T, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "bz_eval_piecewise: grid needs 8-byte, T and out 4-byte alignment");
        const hipStream_t s = as_stream(stream);
        const int64_t per = int64_t(1) << 30;
        for (int64_t q0 = 0; q0 < n_q; q0 += per) {
            const uint32_t nq = static_cast<uint32_t>(std::min(per, n_q - q0));
            const uint32_t ns = static_cast<uint32_t>(n_seg);
            int rc;
            switch (dim) {
                case 1: rc = launch_eval<1>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
                case 2: rc = launch_eval<2>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
                case 3: rc = launch_eval<3>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
                default: rc = launch_eval<4>(grid, ns, T + q0, nq, out + q0, n_q, s); break;
            }
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

int64_t bz_piecewise_tiled_floats(int64_t n_seg, int dim) {
    if (dim < 1 || dim > kMaxDim || n_seg < 1) return 0;
    const int64_t S = tile_segs(dim);
    return (n_seg + S - 1) / S * 32;
}

int bz_tile_piecewise(const float *grid, int64_t n_seg, int dim, float *tiles, bz_stream stream) {
    return guarded("bz_tile_piecewise", [&]() -> int {
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "bz_tile_piecewise: dim %d", dim);
        if (n_seg < 0 || n_seg > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "bz_tile_piecewise: n_seg");
        if (n_seg == 0) return BZ_OK;
        if (!grid || !tiles) return fail(BZ_ERR_NULL, "bz_tile_piecewise: grid and tiles are required");
        if (!aligned(grid, 4) || !aligned(tiles, 128)) return fail(BZ_ERR_ALIGN, "bz_tile_piecewise: tiles need 128-byte alignment");
        const int S = tile_segs(dim);
        const int64_t n_tiles = (n_seg + S - 1) / S;
        const int64_t n = n_tiles * 32;
        const uint32_t blocks = static_cast<uint32_t>((n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_tile_grid, dim3(blocks), dim3(kBlock), 0, as_stream(stream), grid, n_seg, dim, S + 1, S,
                           n_tiles, tiles);
        BZ_CHECK_LAUNCH("k_tile_grid");
        return BZ_OK;
    });
}

int64_t bz_piecewise_tiled16_halfs(int64_t n_seg, int dim) {
    if (dim < 1 || dim > kMaxDim || n_seg < 1) return 0;
    const int64_t S = tile_segs16(dim);
    return (n_seg + S - 1) / S * 64;
}

int bz_tile_piecewise16(const float *grid, int64_t n_seg, int dim, int dtype, void *tiles, bz_stream stream) {
    return guarded("bz_tile_piecewise16", [&]() -> int {
        const char *fn = "bz_tile_piecewise16";
        if (dtype != BZ_F16 && dtype != BZ_BF16) return fail(BZ_ERR_DTYPE, "%s: dtype %d (F16 or BF16)", fn, dtype);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_seg < 0 || n_seg > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_seg", fn);
        if (n_seg == 0) return BZ_OK;
        if (!grid || !tiles) return fail(BZ_ERR_NULL, "%s: grid and tiles are required", fn);
        if (!aligned(grid, 4) || !aligned(tiles, 128)) return fail(BZ_ERR_ALIGN, "%s: tiles need 128-byte alignment", fn);
        const int S = tile_segs16(dim);
        const int64_t n_tiles = (n_seg + S - 1) / S;
        const int64_t n = n_tiles * 64;
        const uint32_t blocks = static_cast<uint32_t>((n + kBlock - 1) / kBlock);
        uint16_t *t16 = static_cast<uint16_t *>(tiles);
        if (dtype == BZ_F16)
            hipLaunchKernelGGL(k_tile_grid16<_Float16>, dim3(blocks), dim3(kBlock), 0, as_stream(stream), grid, n_seg,
                               dim, S + 1, S, n_tiles, t16);
        else
            hipLaunchKernelGGL(k_tile_grid16<bf16_t>, dim3(blocks), dim3(kBlock), 0, as_stream(stream), grid, n_seg, dim,
                               S + 1, S, n_tiles, t16);
        BZ_CHECK_LAUNCH("k_tile_grid16");
        return BZ_OK;
    });
}

int bz_eval_piecewise_tiled16(const void *tiles, int dtype, int64_t n_seg, int dim, const float *T, int64_t n_q,
                              float *out, bz_stream stream) {
    return guarded("bz_eval_piecewise_tiled16", [&]() -> int {
        const char *fn = "bz_eval_piecewise_tiled16";
        if (dtype != BZ_F16 && dtype != BZ_BF16) return fail(BZ_ERR_DTYPE, "%s: dtype %d (F16 or BF16)", fn, dtype);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_q < 0) return fail(BZ_ERR_SHAPE, "%s: n_q", fn);
        if (n_seg < 1 || n_seg > (int64_t(1) << 31))
            return fail(BZ_ERR_SHAPE, "%s: n_seg %lld not in 1..2^31", fn, (long long)n_seg);
        if (n_q == 0) return BZ_OK;
        if (!tiles || !T || !out) return fail(BZ_ERR_NULL, "%s: tiles, T and out are required", fn);
        if (!aligned(tiles, 128) || !aligned(T, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "%s: tiles need 128-byte, T and out 4-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const uint16_t *t16 = static_cast<const uint16_t *>(tiles);
        const int64_t per = int64_t(1) << 30;
        for (int64_t q0 = 0; q0 < n_q; q0 += per) {
            const uint32_t nq = static_cast<uint32_t>(std::min(per, n_q - q0));
            const uint32_t ns = static_cast<uint32_t>(n_seg);
            const int rc = dtype == BZ_F16 ? eval_tiled16_dim<_Float16>(dim, t16, ns, T + q0, nq, out + q0, n_q, s)
                                           : eval_tiled16_dim<bf16_t>(dim, t16, ns, T + q0, nq, out + q0, n_q, s);
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

int bz_eval_piecewise_tiled(const float *tiles, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                            bz_stream stream) {
    return guarded("bz_eval_piecewise_tiled", [&]() -> int {
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "bz_eval_piecewise_tiled: dim %d", dim);
        if (n_q < 0) return fail(BZ_ERR_SHAPE, "bz_eval_piecewise_tiled: n_q");
        if (n_seg < 1 || n_seg > (int64_t(1) << 31))
            return fail(BZ_ERR_SHAPE, "bz_eval_piecewise_tiled: n_seg %lld not in 1..2^31", (long long)n_seg);
        if (n_q == 0) return BZ_OK;
        if (!tiles || !T || !out) return fail(BZ_ERR_NULL, "bz_eval_piecewise_tiled: tiles, T and out are required");
        if (!aligned(tiles, 128) || !aligned(T, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "bz_eval_piecewise_tiled: tiles need 128-byte, T and out 4-byte alignment");
        const hipStream_t s = as_stream(stream);
        const int64_t per = int64_t(1) << 30;
        for (int64_t q0 = 0; q0 < n_q; q0 += per) {
            const uint32_t nq = static_cast<uint32_t>(std::min(per, n_q - q0));
            const uint32_t ns = static_cast<uint32_t>(n_seg);
            int rc;
            switch (dim) {
                case 1: rc = launch_eval_tiled<1>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
                case 2: rc = launch_eval_tiled<2>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
                case 3: rc = launch_eval_tiled<3>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
                default: rc = launch_eval_tiled<4>(tiles, ns, T + q0, nq, out + q0, n_q, s); break;
            }
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

}  // extern "C"
