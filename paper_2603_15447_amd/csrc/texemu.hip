// Texture-filter emulation on the vector ALUs.  gfx950 exposes no texture
// filtering to HIP, so the filter the paper relies on -- texel values at
// texel centres (Sec. 2), weights held in fixed point with 8 fractional bits
// (Sec. 2.3), bilinear / trilinear blends -- runs in registers:
//
//  k_tex_build       control points -> curve textures: de Casteljau layers
//                    [[b_i, b_i+1], [b_i+1, b_i+2]] (Sec. 2) or the Seiler
//                    layouts of Table 1 (Sec. 4), extended to degrees 6 and 7
//                    in one 2x2x2 texture (the case Sec. 6 anticipates),
//                    texels formed in FP64.
//  k_texemu          one query per thread: clamp t, per-axis weight (remap
//                    1/4 + t/2, texel-space 2x - 1/2, F-bit rounding), then
//                    the mode's reads (Fig. 3): one trilinear read (de
//                    Casteljau), bilinear reads + FP32 lerps (hybrid), or
//                    the Seiler read at (t, st), (t, st, st) or, for degrees
//                    6 and 7, (t, st, (st)^2).
//  k_piecewise_texemu  the zig-zag chain (Sec. 2.1) read through the same
//                    emulated bilinear filter in texel space.
//  k_tex_patch_build / k_texemu_patch  surfaces (Sec. 2.2): per v-index a
//                    u-curve texture; de Casteljau isoline reads + v in FP32,
//                    or per-axis Seiler u-textures paired into 2x2x2 reads at
//                    (u, su, v) (Seiler surfaces in the filter, Sec. 6).
//
// The weight decisions are FP32 with every operation rounded as written (no
// contraction), so they match any other FP32 evaluation of the same rule.
#include "texfilter.h"

namespace bzi {
namespace {

enum { TX_DC = 0, TX_HYBRID = 1, TX_SEILER = 2 };
constexpr int kTexMaxDegree = 8;

template <int D, int MODE>
constexpr int tex_texels() {
    return MODE == TX_SEILER ? (D <= 3 ? 4 : 8) : 4 * (D - 1);
}

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_tex_build(const float *__restrict__ ctrl, float *__restrict__ tex,
                                                       uint32_t n_rows) {
    constexpr int NT = tex_texels<D, MODE>();
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_rows) return;
    float b[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) b[i] = ctrl[static_cast<size_t>(r) * (D + 1) + i];
    float T[NT];
    if constexpr (MODE != TX_SEILER) {
#pragma unroll
        for (int i = 0; i < D - 1; ++i) {
            T[4 * i] = b[i];
            T[4 * i + 1] = b[i + 1];
            T[4 * i + 2] = b[i + 1];
            T[4 * i + 3] = b[i + 2];
        }
    } else {
        double sc[D + 1];  // [b0, bd, d1, d_{d-1}, d2, ...]
        seiler_terms<D, double, double>(b, sc);
        const double b0 = sc[0], bd = sc[1];
        if constexpr (D == 2) {
            T[0] = b[0], T[1] = b[2];
            T[2] = static_cast<float>(b0 + sc[2]), T[3] = static_cast<float>(bd + sc[2]);
        } else if constexpr (D == 3) {
            T[0] = b[0], T[1] = b[3];
            T[2] = static_cast<float>(b0 + sc[2]), T[3] = static_cast<float>(bd + sc[3]);
        } else if constexpr (D >= 6) {
            // Read at (t, st, (st)^2), where the eight trilinear products have
            // the distinct degrees 0..7 in t: matching L(b0,bd) + st L(d1,
            // d_{d-1}) + (st)^2 L(d2, d_{d-2}) + (st)^3 L(d3, d_{d-3}) term by
            // term (d_{d-3} = d3 at degree 6).
            const double d1 = sc[2], dl1 = sc[3], d2 = sc[4], dl2 = sc[5], d3 = sc[6];
            const double dl3 = D == 6 ? sc[6] : sc[7];
            T[0] = b[0], T[1] = b[D];
            T[2] = static_cast<float>(b0 + d1), T[3] = static_cast<float>(bd + dl1);
            T[4] = static_cast<float>(b0 + d2), T[5] = static_cast<float>(bd + dl2);
            T[6] = static_cast<float>(b0 + d1 + d2 + d3), T[7] = static_cast<float>(bd + dl1 + dl2 + dl3);
        } else {
            // degree 4: d1, d3, d2; degree 5: d1, d4, d2, d3
            const double d1 = sc[2], dl = sc[3], d2 = sc[4];
            const double dm = sc[D == 4 ? 4 : 5];
            T[0] = b[0], T[1] = b[D], T[2] = b[0], T[3] = b[D];
            T[4] = static_cast<float>(b0 + d1), T[5] = static_cast<float>(bd + dl);
            T[6] = static_cast<float>(b0 + d1 + d2), T[7] = static_cast<float>(bd + dl + dm);
        }
    }
    float4 *__restrict__ o = reinterpret_cast<float4 *>(tex + static_cast<size_t>(r) * NT);
#pragma unroll
    for (int e = 0; e < NT / 4; ++e) o[e] = make_float4(T[4 * e], T[4 * e + 1], T[4 * e + 2], T[4 * e + 3]);
}

struct TexArgs {
    const float *tex;  // textures of curves [c0, c0+n)
    const float *t;    // base of the full parameter array
    float *out;        // base of the full output array
    int64_t plane;     // total queries of the call
    int64_t q0;        // first query of this launch
    uint32_t nq;
    FastDiv div_nt;
    int per_object;
    int frac_bits;
    int rounding;
};

// UNI: n_t is a multiple of 64, so each wavefront reads one curve's texture;
// its index is made wave-uniform and the texels come in through scalar loads.
template <int D, int DIM, int MODE, bool UNI>
__global__ __launch_bounds__(kBlock) void k_texemu(TexArgs a) {
    constexpr int NT = tex_texels<D, MODE>();
    const uint32_t ql = blockIdx.x * kBlock + threadIdx.x;
    if (ql >= a.nq) return;
    uint32_t cl = fdiv(ql, a.div_nt);
    if constexpr (UNI) cl = __builtin_amdgcn_readfirstlane(cl);
    const uint32_t j = ql - cl * a.div_nt.d;
    const int64_t qg = a.q0 + ql;
    float p = a.per_object ? a.t[qg] : a.t[j];
    p = p < 0.0f ? 0.0f : p;  // clamp-to-edge; NaN passes
    p = p > 1.0f ? 1.0f : p;
    const float w = tx_axis_weight(p, a.frac_bits, a.rounding);
    float wst = 0.0f, wz = 0.0f;
    if constexpr (MODE == TX_SEILER) {
#pragma clang fp contract(off)
        const float st = (1.0f - p) * p;
        wst = tx_axis_weight(st, a.frac_bits, a.rounding);
        wz = D >= 6 ? tx_axis_weight(st * st, a.frac_bits, a.rounding) : wst;
    }
    const float4 *__restrict__ src = reinterpret_cast<const float4 *>(a.tex + static_cast<size_t>(cl) * DIM * NT);
    // every coordinate is read before any result is stored (the stores could
    // alias the texels for the compiler, which would then serialise the reads)
    float res[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        float L[NT];
#pragma unroll
        for (int e = 0; e < NT / 4; ++e) {
            const float4 v = src[k * (NT / 4) + e];
            L[4 * e] = v.x, L[4 * e + 1] = v.y, L[4 * e + 2] = v.z, L[4 * e + 3] = v.w;
        }
        float v;
        if constexpr (MODE == TX_SEILER) {
            v = D <= 3 ? tx_bilinear(L, w, wst) : lerp(tx_bilinear(L, w, wst), tx_bilinear(L + 4, w, wst), wz);
        } else {
            // texture reads: level-3 points (trilinear) in de Casteljau mode
            // from degree 3, level-2 points (bilinear) otherwise; the
            // remaining de Casteljau levels run in FP32 with the exact t
            constexpr int M = (MODE == TX_DC && D >= 3) ? D - 2 : D - 1;
            float lv[M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if constexpr (MODE == TX_DC && D >= 3)
                    lv[i] = lerp(tx_bilinear(L + 4 * i, w, w), tx_bilinear(L + 4 * i + 4, w, w), w);
                else
                    lv[i] = tx_bilinear(L + 4 * i, w, w);
            }
#pragma unroll
            for (int lvl = 1; lvl < M; ++lvl)
#pragma unroll
                for (int i = 0; i < M - lvl; ++i) lv[i] = lerp(lv[i], lv[i + 1], p);
            v = lv[0];
        }
        res[k] = v;
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) st_stream(a.out + k * a.plane + qg, res[k]);
}

// TILED: the texels in the 128-byte cache-line tiles of bz_tile_piecewise
// (C = 128/(8*DIM) columns per tile, consecutive tiles sharing a column, so
// segment k's window is columns r, r+1 of tile k/(C-1)); otherwise the
// column-major grid.
template <int DIM, int QPT, bool TILED>
__global__ __launch_bounds__(kBlock) void k_piecewise_texemu(const float *__restrict__ grid, uint32_t n_seg,
                                                             const float *__restrict__ T, uint32_t nq,
                                                             float *__restrict__ out, int64_t plane, int F,
                                                             int rnd) {
#pragma clang fp contract(off)
    const uint32_t base = blockIdx.x * (kBlock * QPT) + threadIdx.x;
    const float nf = static_cast<float>(n_seg);
    const float nm1 = static_cast<float>(n_seg - 1);
    float wx[QPT], wy[QPT];
    uint32_t kk[QPT];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t q = min(base + i * kBlock, nq - 1);
        float Tc = ld_stream(T + q);
        Tc = Tc < 0.0f ? 0.0f : Tc;
        Tc = Tc > nf ? nf : Tc;
        const float x = Tc + 0.5f;  // texel-space coordinate, centres at c + 1/2
        const float xb = x - 0.5f;
        const float kf = __builtin_fminf(__builtin_floorf(xb), nm1);  // NaN -> n_seg-1, in bounds
        const uint32_t k = min(static_cast<uint32_t>(kf), n_seg - 1);
        const float fx = xb - static_cast<float>(k);
        const float y = (k & 1) ? 1.5f - fx : fx + 0.5f;
        float yb = y - 0.5f;
        yb = yb < 0.0f ? 0.0f : yb;
        yb = yb > 1.0f ? 1.0f : yb;
        kk[i] = k;
        wx[i] = tx_round(fx, F, rnd);
        wy[i] = tx_round(yb, F, rnd);
    }
    float2 g[QPT][2 * DIM];
    const float2 *__restrict__ g2 = reinterpret_cast<const float2 *>(grid);
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        size_t off = static_cast<size_t>(kk[i]) * DIM;  // in float2 units
        if constexpr (TILED) {
            constexpr uint32_t S = 128 / (8 * DIM) - 1;  // segments per tile
            const uint32_t j = kk[i] / S, r = kk[i] - j * S;
            off = static_cast<size_t>(j) * 16 + r * DIM;
        }
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) g[i][e] = g2[off + e];
    }
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        float f[4 * DIM];  // [column k, k+1][row 0, 1][dim]
#pragma unroll
        for (int e = 0; e < 2 * DIM; ++e) f[2 * e] = g[i][e].x, f[2 * e + 1] = g[i][e].y;
        const uint32_t q = min(base + i * kBlock, nq - 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const float L[4] = {f[c], f[2 * DIM + c], f[DIM + c], f[3 * DIM + c]};
            st_stream(out + c * plane + q, tx_bilinear(L, wx[i], wy[i]));
        }
    }
}

// ------------------------------------------------------------------ host
template <int MODE>
int launch_build_m(int degree, const float *ctrl, float *tex, uint32_t rows, hipStream_t s) {
    const uint32_t blocks = (rows + kBlock - 1) / kBlock;
#define BZI_TB(D)                                                                                   \
    case D:                                                                                         \
        if constexpr (MODE != TX_SEILER || D <= 7)                                                  \
            hipLaunchKernelGGL((k_tex_build<D, MODE>), dim3(blocks), dim3(kBlock), 0, s, ctrl, tex, rows); \
        break;
    switch (degree) {
        BZI_TB(2) BZI_TB(3) BZI_TB(4) BZI_TB(5) BZI_TB(6) BZI_TB(7) BZI_TB(8)
        default: return fail(BZ_ERR_SHAPE, "degree %d", degree);
    }
#undef BZI_TB
    BZ_CHECK_LAUNCH("k_tex_build");
    return BZ_OK;
}

template <int D, int MODE, bool UNI>
void launch_texemu_dmu(int dim, const TexArgs &a, hipStream_t s) {
    const uint32_t blocks = (a.nq + kBlock - 1) / kBlock;
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_texemu<D, 1, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_texemu<D, 2, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_texemu<D, 3, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_texemu<D, 4, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
    }
}

template <int D, int MODE>
int launch_texemu_dm(int dim, const TexArgs &a, hipStream_t s) {
    if (a.div_nt.d % 64 == 0) launch_texemu_dmu<D, MODE, true>(dim, a, s);
    else launch_texemu_dmu<D, MODE, false>(dim, a, s);
    BZ_CHECK_LAUNCH("k_texemu");
    return BZ_OK;
}

template <int MODE>
int launch_texemu_m(int degree, int dim, const TexArgs &a, hipStream_t s) {
    switch (degree) {
        case 2: return launch_texemu_dm<2, MODE>(dim, a, s);
        case 3: return launch_texemu_dm<3, MODE>(dim, a, s);
        case 4: return launch_texemu_dm<4, MODE>(dim, a, s);
        case 5: return launch_texemu_dm<5, MODE>(dim, a, s);
        case 6: return launch_texemu_dm<6, MODE>(dim, a, s);
        case 7: return launch_texemu_dm<7, MODE>(dim, a, s);
        default: break;
    }
    if constexpr (MODE != TX_SEILER) {
        if (degree == 8) return launch_texemu_dm<8, MODE>(dim, a, s);
    }
    return fail(BZ_ERR_SHAPE, "degree %d", degree);
}

int tex_texels_rt(int degree, int mode) {
    if (mode == TX_SEILER) return degree >= 2 && degree <= 7 ? (degree <= 3 ? 4 : 8) : 0;
    if (mode == TX_DC || mode == TX_HYBRID) return degree >= 2 && degree <= kTexMaxDegree ? 4 * (degree - 1) : 0;
    return 0;
}

template <int DIM, bool TILED>
int launch_chain_texemu(const float *grid, uint32_t n_seg, const float *T, uint32_t nq, float *out, int64_t plane,
                        int F, int rnd, hipStream_t s) {
    constexpr int Q = 4;
    const uint32_t blocks = (nq + kBlock * Q - 1) / (kBlock * Q);
    hipLaunchKernelGGL((k_piecewise_texemu<DIM, Q, TILED>), dim3(blocks), dim3(kBlock), 0, s, grid, n_seg, T, nq, out,
                       plane, F, rnd);
    BZ_CHECK_LAUNCH("k_piecewise_texemu");
    return BZ_OK;
}

constexpr int kMaxFracBits = 20;

// Validation and chunked launches of the chain read through the filter, for
// the column-major grid or its cache-line tiles.
template <bool TILED>
int chain_texemu_entry(const char *fn, const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q,
                       int frac_bits, int rounding, float *out, bz_stream stream) {
    if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
    if (n_q < 0) return fail(BZ_ERR_SHAPE, "%s: n_q", fn);
    if (n_seg < 1 || n_seg > (int64_t(1) << 24))
        return fail(BZ_ERR_SHAPE, "%s: n_seg not in 1..2^24 (FP32 texel-space coordinates)", fn);
    if (frac_bits < 0 || frac_bits > kMaxFracBits)
        return fail(BZ_ERR_SHAPE, "%s: frac_bits %d not in 0..%d", fn, frac_bits, kMaxFracBits);
    if (rounding != BZ_TEXW_NEAREST && rounding != BZ_TEXW_TRUNCATE)
        return fail(BZ_ERR_SHAPE, "%s: rounding %d", fn, rounding);
    if (n_q == 0) return BZ_OK;
    if (!grid || !T || !out) return fail(BZ_ERR_NULL, "%s: texels, T and out are required", fn);
    if (!aligned(grid, TILED ? 128 : 8) || !aligned(T, 4) || !aligned(out, 4))
        return fail(BZ_ERR_ALIGN, "%s: texels need %d-byte alignment", fn, TILED ? 128 : 8);
    const hipStream_t s = as_stream(stream);
    const int64_t per = int64_t(1) << 30;
    for (int64_t q0 = 0; q0 < n_q; q0 += per) {
        const uint32_t nq = static_cast<uint32_t>(std::min(per, n_q - q0));
        const uint32_t ns = static_cast<uint32_t>(n_seg);
        int rc;
        switch (dim) {
            case 1: rc = launch_chain_texemu<1, TILED>(grid, ns, T + q0, nq, out + q0, n_q, frac_bits, rounding, s); break;
            case 2: rc = launch_chain_texemu<2, TILED>(grid, ns, T + q0, nq, out + q0, n_q, frac_bits, rounding, s); break;
            case 3: rc = launch_chain_texemu<3, TILED>(grid, ns, T + q0, nq, out + q0, n_q, frac_bits, rounding, s); break;
            default: rc = launch_chain_texemu<4, TILED>(grid, ns, T + q0, nq, out + q0, n_q, frac_bits, rounding, s); break;
        }
        if (rc) return rc;
    }
    return BZ_OK;
}

// ------------------------------------------------------------------ surfaces
// Patch ctrl[n][dim][(DU+1)(DV+1)] (u major), DU in {2, 3}, DV in 1..4.  Every
// v-index j gets the u-curve texture of its fibre: de Casteljau layers of
// (P_0j..P_DUj), or -- Seiler mode -- the Table 1 texture of the fibre of the
// per-axis Seiler terms (converted along v, then u, in FP64).
template <int DU, int MODE>
constexpr int patch_fibre_texels() {
    return MODE == TX_SEILER ? 4 : 4 * (DU - 1);
}

template <int DU, int DV, int MODE>
__global__ __launch_bounds__(kBlock) void k_tex_patch_build(const float *__restrict__ ctrl, float *__restrict__ tex,
                                                             uint32_t n_rows) {
    constexpr int NV = DV + 1, NCP = (DU + 1) * NV, PER = patch_fibre_texels<DU, MODE>();
    const uint32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_rows) return;
    double a[NCP];
#pragma unroll
    for (int e = 0; e < NCP; ++e) a[e] = static_cast<double>(ctrl[static_cast<size_t>(r) * NCP + e]);
    if constexpr (MODE == TX_SEILER) {
#pragma unroll
        for (int i = 0; i <= DU; ++i) {  // v fibres
            double b[DV + 1], sc[DV + 1];
#pragma unroll
            for (int j = 0; j <= DV; ++j) b[j] = a[i * NV + j];
            seiler_terms<DV, double, double, double>(b, sc);
#pragma unroll
            for (int j = 0; j <= DV; ++j) a[i * NV + j] = sc[j];
        }
#pragma unroll
        for (int j = 0; j <= DV; ++j) {  // u fibres
            double b[DU + 1], sc[DU + 1];
#pragma unroll
            for (int i = 0; i <= DU; ++i) b[i] = a[i * NV + j];
            seiler_terms<DU, double, double, double>(b, sc);
#pragma unroll
            for (int i = 0; i <= DU; ++i) a[i * NV + j] = sc[i];
        }
    }
    float *__restrict__ o = tex + static_cast<size_t>(r) * NV * PER;
#pragma unroll
    for (int j = 0; j <= DV; ++j) {
        float T[PER];
        if constexpr (MODE != TX_SEILER) {
#pragma unroll
            for (int i = 0; i < DU - 1; ++i) {
                T[4 * i] = static_cast<float>(a[i * NV + j]);
                T[4 * i + 1] = static_cast<float>(a[(i + 1) * NV + j]);
                T[4 * i + 2] = static_cast<float>(a[(i + 1) * NV + j]);
                T[4 * i + 3] = static_cast<float>(a[(i + 2) * NV + j]);
            }
        } else {
            // fibre terms [b0, bd, d1(, d2)]: degree 2 [[b0, b2], [b0+d1, b2+d1]],
            // degree 3 [[b0, b3], [b0+d1, b3+d2]]
            const double b0 = a[j], bd = a[NV + j], d1 = a[2 * NV + j];
            const double dl = DU == 2 ? d1 : a[3 * NV + j];
            T[0] = static_cast<float>(b0), T[1] = static_cast<float>(bd);
            T[2] = static_cast<float>(b0 + d1), T[3] = static_cast<float>(bd + dl);
        }
#pragma unroll
        for (int e = 0; e < PER / 4; ++e)
            reinterpret_cast<float4 *>(o + j * PER)[e] = make_float4(T[4 * e], T[4 * e + 1], T[4 * e + 2], T[4 * e + 3]);
    }
}

struct TexPatchArgs {
    const float *tex;  // textures of patches [o0, o0+n)
    const float *uv;   // base of the full parameter array [n_obj][n_per][2]
    float *out;
    int64_t plane;
    int64_t q0;        // first query of this launch
    uint32_t nq;
    FastDiv div_per;
    int frac_bits;
    int rounding;
};

// UNI: n_per is a multiple of 64, so each wavefront reads one patch's
// textures, through scalar loads of a wave-uniform address.
template <int DU, int DV, int DIM, int MODE, bool UNI>
__global__ __launch_bounds__(kBlock) void k_texemu_patch(TexPatchArgs a) {
    constexpr int PER = patch_fibre_texels<DU, MODE>(), NT = (DV + 1) * PER;
    const uint32_t ql = blockIdx.x * kBlock + threadIdx.x;
    if (ql >= a.nq) return;
    uint32_t ol = fdiv(ql, a.div_per);
    if constexpr (UNI) ol = __builtin_amdgcn_readfirstlane(ol);
    const int64_t qg = a.q0 + ql;
    const float2 p2 = reinterpret_cast<const float2 *>(a.uv)[qg];
    float u = p2.x < 0.0f ? 0.0f : p2.x, v = p2.y < 0.0f ? 0.0f : p2.y;  // clamp-to-edge; NaN passes
    u = u > 1.0f ? 1.0f : u;
    v = v > 1.0f ? 1.0f : v;
    const float wu = tx_axis_weight(u, a.frac_bits, a.rounding);
    float wsu = 0.0f, wv = 0.0f;
    if constexpr (MODE == TX_SEILER) {
#pragma clang fp contract(off)
        wsu = tx_axis_weight((1.0f - u) * u, a.frac_bits, a.rounding);
        wv = tx_axis_weight(v, a.frac_bits, a.rounding);
    }
    const float4 *__restrict__ src = reinterpret_cast<const float4 *>(a.tex + static_cast<size_t>(ol) * DIM * NT);
    float res[DIM];  // all coordinates read before any store
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        float L[NT];
#pragma unroll
        for (int e = 0; e < NT / 4; ++e) {
            const float4 x = src[c * (NT / 4) + e];
            L[4 * e] = x.x, L[4 * e + 1] = x.y, L[4 * e + 2] = x.z, L[4 * e + 3] = x.w;
        }
        float val;
        if constexpr (MODE != TX_SEILER) {
            float R[DV + 1];  // isoline control points R_j(u), then de Casteljau in v
#pragma unroll
            for (int j = 0; j <= DV; ++j)
                R[j] = DU == 3 ? lerp(tx_bilinear(L + j * PER, wu, wu), tx_bilinear(L + j * PER + 4, wu, wu), wu)
                               : tx_bilinear(L + j * PER, wu, wu);
#pragma unroll
            for (int lvl = 1; lvl <= DV; ++lvl)
#pragma unroll
                for (int j = 0; j <= DV - lvl; ++j) R[j] = lerp(R[j], R[j + 1], v);
            val = R[0];
        } else {
            // v-Seiler terms in storage order [b0, bd, d1, d_{d-1}, d2]: pairs
            // (0,1) and (2,3) by trilinear reads at (u, su, v), the middle
            // term of even DV by a bilinear read at (u, su)
            const float sv = (1.0f - v) * v;
            const float r0 = lerp(tx_bilinear(L, wu, wsu), tx_bilinear(L + 4, wu, wsu), wv);
            float acc = 0.0f;
            if constexpr (DV == 2) acc = tx_bilinear(L + 8, wu, wsu);
            if constexpr (DV >= 3) {
                acc = lerp(tx_bilinear(L + 8, wu, wsu), tx_bilinear(L + 12, wu, wsu), wv);
                if constexpr (DV == 4) acc = __builtin_fmaf(sv, tx_bilinear(L + 16, wu, wsu), acc);
            }
            val = __builtin_fmaf(sv, acc, r0);
        }
        res[c] = val;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) st_stream(a.out + c * a.plane + qg, res[c]);
}

template <int MODE>
int launch_patch_build(int du, int dv, const float *ctrl, float *tex, uint32_t rows, hipStream_t s) {
    const uint32_t blocks = (rows + kBlock - 1) / kBlock;
#define BZI_PB(U, V)                                                                                        \
    if (du == U && dv == V) {                                                                               \
        hipLaunchKernelGGL((k_tex_patch_build<U, V, MODE>), dim3(blocks), dim3(kBlock), 0, s, ctrl, tex, rows); \
        BZ_CHECK_LAUNCH("k_tex_patch_build");                                                               \
        return BZ_OK;                                                                                       \
    }
    BZI_PB(2, 1) BZI_PB(2, 2) BZI_PB(2, 3) BZI_PB(2, 4) BZI_PB(3, 1) BZI_PB(3, 2) BZI_PB(3, 3) BZI_PB(3, 4)
#undef BZI_PB
    return fail(BZ_ERR_SHAPE, "degrees (%d, %d)", du, dv);
}

template <int DU, int DV, int MODE, bool UNI>
void launch_patch_eval_du(int dim, const TexPatchArgs &a, hipStream_t s) {
    const uint32_t blocks = (a.nq + kBlock - 1) / kBlock;
    switch (dim) {
        case 1: hipLaunchKernelGGL((k_texemu_patch<DU, DV, 1, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_texemu_patch<DU, DV, 2, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_texemu_patch<DU, DV, 3, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_texemu_patch<DU, DV, 4, MODE, UNI>), dim3(blocks), dim3(kBlock), 0, s, a); break;
    }
}

template <int DU, int DV, int MODE>
int launch_patch_eval_d(int dim, const TexPatchArgs &a, hipStream_t s) {
    if (a.div_per.d % 64 == 0) launch_patch_eval_du<DU, DV, MODE, true>(dim, a, s);
    else launch_patch_eval_du<DU, DV, MODE, false>(dim, a, s);
    BZ_CHECK_LAUNCH("k_texemu_patch");
    return BZ_OK;
}

template <int MODE>
int launch_patch_eval(int du, int dv, int dim, const TexPatchArgs &a, hipStream_t s) {
#define BZI_PE(U, V) \
    if (du == U && dv == V) return launch_patch_eval_d<U, V, MODE>(dim, a, s);
    BZI_PE(2, 1) BZI_PE(2, 2) BZI_PE(2, 3) BZI_PE(2, 4) BZI_PE(3, 1) BZI_PE(3, 2) BZI_PE(3, 3) BZI_PE(3, 4)
#undef BZI_PE
    return fail(BZ_ERR_SHAPE, "degrees (%d, %d)", du, dv);
}

int patch_texels_rt(int du, int dv, int mode) {
    if (du < 2 || du > 3 || dv < 1 || dv > 4) return 0;
    if (mode == TX_SEILER) return (dv + 1) * 4;
    if (mode == TX_DC) return (dv + 1) * 4 * (du - 1);
    return 0;
}


}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

int bz_texture_texels(int degree, int mode) { return tex_texels_rt(degree, mode); }

int bz_build_texture(const float *ctrl, int64_t n_curves, int degree, int dim, int mode, float *tex,
                     bz_stream stream) {
    return guarded("bz_build_texture", [&]() -> int {
        const char *fn = "bz_build_texture";
        if (tex_texels_rt(degree, mode) == 0)
            return fail(BZ_ERR_UNSUPPORTED, "%s: mode %d at degree %d (de Casteljau / hybrid 2..%d, Seiler 2..7)", fn,
                        mode, degree, kTexMaxDegree);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_curves < 0 || n_curves * dim > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_curves", fn);
        if (n_curves == 0) return BZ_OK;
        if (!ctrl || !tex) return fail(BZ_ERR_NULL, "%s: ctrl and tex are required", fn);
        if (!aligned(ctrl, 4) || !aligned(tex, 16)) return fail(BZ_ERR_ALIGN, "%s: tex needs 16-byte alignment", fn);
        const uint32_t rows = static_cast<uint32_t>(n_curves * dim);
        const hipStream_t s = as_stream(stream);
        if (mode == TX_SEILER) return launch_build_m<TX_SEILER>(degree, ctrl, tex, rows, s);
        return launch_build_m<TX_DC>(degree, ctrl, tex, rows, s);  // hybrid shares the texels
    });
}

int bz_eval_texture(const float *tex, int64_t n_curves, int degree, int dim, int mode, const float *t, int64_t n_t,
                    int t_mode, int frac_bits, int rounding, float *out, bz_stream stream) {
    return guarded("bz_eval_texture", [&]() -> int {
        const char *fn = "bz_eval_texture";
        const int ntx = tex_texels_rt(degree, mode);
        if (ntx == 0)
            return fail(BZ_ERR_UNSUPPORTED, "%s: mode %d at degree %d (de Casteljau / hybrid 2..%d, Seiler 2..7)", fn,
                        mode, degree, kTexMaxDegree);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_curves < 0 || n_t < 0 || n_t > (int64_t(1) << 30)) return fail(BZ_ERR_SHAPE, "%s: counts", fn);
        if (n_curves > 0 && n_t > 0 && n_curves > (int64_t(1) << 62) / n_t)
            return fail(BZ_ERR_SHAPE, "%s: n_curves*n_t overflows", fn);
        if (t_mode != BZ_T_SHARED && t_mode != BZ_T_PER_OBJECT) return fail(BZ_ERR_SHAPE, "%s: t_mode %d", fn, t_mode);
        if (frac_bits < 0 || frac_bits > kMaxFracBits)
            return fail(BZ_ERR_SHAPE, "%s: frac_bits %d not in 0..%d", fn, frac_bits, kMaxFracBits);
        if (rounding != BZ_TEXW_NEAREST && rounding != BZ_TEXW_TRUNCATE)
            return fail(BZ_ERR_SHAPE, "%s: rounding %d", fn, rounding);
        if (n_curves == 0 || n_t == 0) return BZ_OK;
        if (!tex || !t || !out) return fail(BZ_ERR_NULL, "%s: tex, t and out are required", fn);
        if (!aligned(tex, 16) || !aligned(t, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "%s: tex needs 16-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const int64_t nq = n_curves * n_t;
        const int64_t per = std::max<int64_t>(1, (int64_t(1) << 30) / n_t);
        for (int64_t c0 = 0; c0 < n_curves; c0 += per) {
            const int64_t nc = std::min(per, n_curves - c0);
            TexArgs a;
            a.tex = tex + c0 * dim * ntx;
            a.t = t;
            a.out = out;
            a.plane = nq;
            a.q0 = c0 * n_t;
            a.nq = static_cast<uint32_t>(nc * n_t);
            a.div_nt = make_fastdiv(static_cast<uint32_t>(n_t));
            a.per_object = t_mode == BZ_T_PER_OBJECT;
            a.frac_bits = frac_bits;
            a.rounding = rounding;
            int rc;
            if (mode == TX_DC) rc = launch_texemu_m<TX_DC>(degree, dim, a, s);
            else if (mode == TX_HYBRID) rc = launch_texemu_m<TX_HYBRID>(degree, dim, a, s);
            else rc = launch_texemu_m<TX_SEILER>(degree, dim, a, s);
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

int bz_eval_piecewise_texemu(const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q, int frac_bits,
                             int rounding, float *out, bz_stream stream) {
    return guarded("bz_eval_piecewise_texemu", [&]() -> int {
        return chain_texemu_entry<false>("bz_eval_piecewise_texemu", grid, n_seg, dim, T, n_q, frac_bits, rounding,
                                         out, stream);
    });
}

int bz_eval_piecewise_texemu_tiled(const float *tiles, int64_t n_seg, int dim, const float *T, int64_t n_q,
                                   int frac_bits, int rounding, float *out, bz_stream stream) {
    return guarded("bz_eval_piecewise_texemu_tiled", [&]() -> int {
        return chain_texemu_entry<true>("bz_eval_piecewise_texemu_tiled", tiles, n_seg, dim, T, n_q, frac_bits,
                                        rounding, out, stream);
    });
}

int bz_texture_patch_texels(int du, int dv, int mode) { return patch_texels_rt(du, dv, mode); }

int bz_build_texture_patch(const float *ctrl, int64_t n_obj, int du, int dv, int dim, int mode, float *tex,
                           bz_stream stream) {
    return guarded("bz_build_texture_patch", [&]() -> int {
        const char *fn = "bz_build_texture_patch";
        if (patch_texels_rt(du, dv, mode) == 0)
            return fail(BZ_ERR_UNSUPPORTED, "%s: mode %d at degrees (%d, %d) (du 2..3, dv 1..4, de Casteljau or Seiler)",
                        fn, mode, du, dv);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_obj < 0 || n_obj * dim > (int64_t(1) << 31)) return fail(BZ_ERR_SHAPE, "%s: n_obj", fn);
        if (n_obj == 0) return BZ_OK;
        if (!ctrl || !tex) return fail(BZ_ERR_NULL, "%s: ctrl and tex are required", fn);
        if (!aligned(ctrl, 4) || !aligned(tex, 16)) return fail(BZ_ERR_ALIGN, "%s: tex needs 16-byte alignment", fn);
        const uint32_t rows = static_cast<uint32_t>(n_obj * dim);
        const hipStream_t s = as_stream(stream);
        if (mode == TX_SEILER) return launch_patch_build<TX_SEILER>(du, dv, ctrl, tex, rows, s);
        return launch_patch_build<TX_DC>(du, dv, ctrl, tex, rows, s);
    });
}

int bz_eval_texture_patch(const float *tex, int64_t n_obj, int du, int dv, int dim, int mode, const float *uv,
                          int64_t n_per, int frac_bits, int rounding, float *out, bz_stream stream) {
    return guarded("bz_eval_texture_patch", [&]() -> int {
        const char *fn = "bz_eval_texture_patch";
        const int ntx = patch_texels_rt(du, dv, mode);
        if (ntx == 0)
            return fail(BZ_ERR_UNSUPPORTED, "%s: mode %d at degrees (%d, %d) (du 2..3, dv 1..4, de Casteljau or Seiler)",
                        fn, mode, du, dv);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_obj < 0 || n_per < 0 || n_per > (int64_t(1) << 30)) return fail(BZ_ERR_SHAPE, "%s: counts", fn);
        if (n_obj > 0 && n_per > 0 && n_obj > (int64_t(1) << 62) / n_per)
            return fail(BZ_ERR_SHAPE, "%s: n_obj*n_per overflows", fn);
        if (frac_bits < 0 || frac_bits > kMaxFracBits)
            return fail(BZ_ERR_SHAPE, "%s: frac_bits %d not in 0..%d", fn, frac_bits, kMaxFracBits);
        if (rounding != BZ_TEXW_NEAREST && rounding != BZ_TEXW_TRUNCATE)
            return fail(BZ_ERR_SHAPE, "%s: rounding %d", fn, rounding);
        if (n_obj == 0 || n_per == 0) return BZ_OK;
        if (!tex || !uv || !out) return fail(BZ_ERR_NULL, "%s: tex, uv and out are required", fn);
        if (!aligned(tex, 16) || !aligned(uv, 8) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "%s: tex needs 16-byte, uv 8-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const int64_t nq = n_obj * n_per;
        const int64_t per = std::max<int64_t>(1, (int64_t(1) << 30) / n_per);
        for (int64_t o0 = 0; o0 < n_obj; o0 += per) {
            const int64_t no = std::min(per, n_obj - o0);
            TexPatchArgs a;
            a.tex = tex + o0 * dim * ntx;
            a.uv = uv;
            a.out = out;
            a.plane = nq;
            a.q0 = o0 * n_per;
            a.nq = static_cast<uint32_t>(no * n_per);
            a.div_per = make_fastdiv(static_cast<uint32_t>(n_per));
            a.frac_bits = frac_bits;
            a.rounding = rounding;
            const int rc = mode == TX_SEILER ? launch_patch_eval<TX_SEILER>(du, dv, dim, a, s)
                                             : launch_patch_eval<TX_DC>(du, dv, dim, a, s);
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

}  // extern "C"
