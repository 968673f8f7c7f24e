/*
 * bz.h -- C ABI of the MI355X (gfx950) Bezier-family evaluation library.
 *
 * Evaluates Bezier curves, surfaces and volumes (integral and rational),
 * C0 piecewise quadratic chains in the shared-diagonal encoding and cubic
 * NURBS at many parameter values, following Anas & Wolfe, "A Texture Lookup
 * Approach to Bezier Curve Evaluation on the GPU" (arXiv 2603.15447), with
 * hand-written HIP kernels instead of texture filtering.
 *
 * General conventions (apply to every entry point below):
 *  - Every array argument is a DEVICE pointer owned by the caller.  The
 *    library never frees it and keeps no reference to it after the call
 *    returns (a batch plan keeps its own copies).
 *  - Every call is asynchronous on `stream` (a hipStream_t, NULL = the null
 *    stream) and never synchronises the device, except bz_batch_plan_create.
 *  - Every entry point returns a bz_status.  Arguments are validated before
 *    anything is launched, so an error leaves no partial work behind.  A
 *    zero-size call returns BZ_OK without launching.  No C++ exception
 *    crosses the ABI.  bz_last_error() gives a thread-local message for the
 *    most recent failure on the calling thread.
 *  - Parameters outside [0,1] extrapolate the polynomial.  NaN in gives NaN
 *    out.  Results are FP32.
 *  - Curve layout: ctrl[n][dim][degree+1] (coordinate-major per curve).
 *    Parameters t[n_t] (BZ_T_SHARED: the same n_t values for every curve) or
 *    t[n][n_t] (BZ_T_PER_OBJECT).  Results are planar, out[dim][n*n_t], with
 *    query q = c*n_t + j.
 *  - Limits: 1 <= degree <= 15, 1 <= dim <= 4, counts >= 0.  Pointers to
 *    FP32 data need 4-byte alignment, FP16/BF16 data 2-byte alignment.
 */
#ifndef BZ_H
#define BZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *bz_stream; /* hipStream_t */

typedef enum {
    BZ_OK = 0,
    BZ_ERR_NULL = 1,        /* a required pointer is NULL */
    BZ_ERR_SHAPE = 2,       /* degree, dim or a count is out of range */
    BZ_ERR_DTYPE = 3,       /* unknown storage type */
    BZ_ERR_UNSUPPORTED = 4, /* valid but not implemented combination */
    BZ_ERR_ALIGN = 5,       /* pointer misaligned for its element type */
    BZ_ERR_HIP = 6,         /* the HIP runtime reported an error */
    BZ_ERR_NOMEM = 7,       /* a device allocation failed */
    BZ_ERR_INTERNAL = 8     /* unexpected internal failure */
} bz_status;

typedef enum { BZ_F32 = 0, BZ_F16 = 1, BZ_BF16 = 2 } bz_dtype; /* control-point / weight storage */

/* BZ_AUTO lets the library pick the form: the Bernstein form, the fastest of
 * the three measured at degree 3 (or within the run-to-run spread) and O(d)
 * per coordinate against de Casteljau's O(d^2) at higher degrees, at the same
 * accuracy. */
typedef enum { BZ_DECASTELJAU = 0, BZ_BERNSTEIN = 1, BZ_SEILER = 2, BZ_AUTO = 3 } bz_method;

typedef enum { BZ_T_SHARED = 0, BZ_T_PER_OBJECT = 1 } bz_tmode;

typedef enum { BZ_TEX_DECASTELJAU = 0, BZ_TEX_HYBRID = 1, BZ_TEX_SEILER = 2 } bz_tex_mode;

typedef enum { BZ_TEXW_NEAREST = 0, BZ_TEXW_TRUNCATE = 1 } bz_tex_rounding;

typedef enum {
    BZ_TP_VALU = 0,      /* separable FP32 vector evaluation */
    BZ_TP_MFMA_F32 = 1,  /* basis-matrix contraction on FP32 matrix cores */
    BZ_TP_MFMA_BF16 = 2, /* BF16 operands, FP32 accumulation */
    BZ_TP_MFMA_F16 = 3,  /* FP16 operands, FP32 accumulation */
    BZ_TP_MFMA_F16X3 = 4 /* FP16 high/low operand split, three products, FP32 accumulation */
} bz_tp_engine;

int bz_version(void);
const char *bz_status_string(int code);
const char *bz_last_error(void);

/*
 * Bezier curves (Sec. 2: de Casteljau recursive lerps; Sec. 3: Seiler
 * interpolation; Sec. 5: the Bernstein polynomial form).
 * ctrl: [n_curves][dim][degree+1] in ctrl_dtype.  t: see t_mode.
 * method: BZ_DECASTELJAU (d(d+1)/2 lerps), BZ_BERNSTEIN (basis + d+1 FMAs per
 * coordinate), BZ_SEILER (difference terms derived per evaluation, then
 * d lerps) or BZ_AUTO.  out: [dim][n_curves*n_t] FP32.
 */
int bz_eval_bezier(const void *ctrl, int ctrl_dtype, int64_t n_curves, int degree, int dim, const float *t,
                   int64_t n_t, int t_mode, int method, float *out, bz_stream stream);

/*
 * Seiler difference terms (Sec. 3.1: C = L(b0,bd,t) + (1-t)t D_1 with the
 * recursive D_i).  Writes, per curve and coordinate, d+1 FP32 values
 * [b0, bd, d1, d_{d-1}, d2, d_{d-2}, ...] (the middle term d_{d/2} once for
 * even d) to seiler[n_curves][dim][degree+1].
 */
int bz_bezier_to_seiler(const void *ctrl, int ctrl_dtype, int64_t n_curves, int degree, int dim, float *seiler,
                        bz_stream stream);

/* Evaluate curves given by Seiler terms (layout as produced above). */
int bz_eval_seiler(const float *seiler, int64_t n_curves, int degree, int dim, const float *t, int64_t n_t,
                   int t_mode, float *out, bz_stream stream);

/*
 * Rational Bezier curves (Sec. 2.2: one integral spline divided by
 * another): the chosen method is applied to the homogeneous points
 * (w_i b_i, w_i) and the result divided by the weight.
 * w: [n_curves][degree+1] in the same dtype as ctrl.
 * A point whose conditioning number sum|w_i|B_i / |sum w_i B_i| exceeds
 * kappa (or whose weight sum is 0 or not finite) is recomputed in FP64 by de
 * Casteljau.  With all weights positive the number is 1 and no point is
 * recomputed.  kappa <= 0 disables the recomputation.  n_fixed (nullable,
 * device, one uint32) is incremented by the number of recomputed points.
 */
int bz_eval_rational(const void *ctrl, const void *w, int dtype, int64_t n_curves, int degree, int dim,
                     const float *t, int64_t n_t, int t_mode, int method, float kappa, float *out,
                     uint32_t *n_fixed, bz_stream stream);

/*
 * C0 piecewise quadratic chain, shared-diagonal ("zig-zag") encoding
 * (Sec. 2.1, Eq. 1-2, Fig. 2).
 * chain: [2*n_seg+1][dim], A_k = chain[2k] the shared endpoints and
 *        M_k = chain[2k+1] the middle control point of segment k.
 * grid:  [n_seg+1][2][dim], 2(n_seg+1) texels.  Column k holds A_k in row
 *        k mod 2 and a free texel x_k in the other row, with x_0 = M_0 and
 *        (x_k + x_{k+1})/2 = M_k (the diagonal texels of segment k average
 *        to its middle control point).  The free texels are formed by an
 *        FP64 alternating prefix sum and rounded once to FP32.
 * Uses a small stream-ordered device workspace (hipMallocAsync).
 */
int bz_encode_piecewise(const float *chain, int64_t n_seg, int dim, float *grid, bz_stream stream);

/*
 * Allocation-free variant of bz_encode_piecewise, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, same results bit for
 * bit; it allocates nothing (no hipMalloc, hipMallocAsync or hipFree): the
 * encoder's block partials live in a fixed 2 MiB device array of the library
 * (a copy per device, held until the process ends), whose address is looked
 * up once per device on the first call with that device current.  Limit: the
 * partials of ceil((n_seg+1)/2048) blocks x dim coordinates must fit 2^18
 * doubles, i.e. n_seg <= floor(2^18/dim)*2048 - 1 (536870911, 268435455,
 * 178956287, 134217727 for dim 1..4); larger n_seg returns BZ_ERR_SHAPE.
 * Every call on one device uses that device's one array: calls that overlap
 * in time on one device (different streams or threads) race and must be
 * serialised by the caller.  The array needs no clearing between calls.
 */
int bz_encode_piecewise_noalloc(const float *chain, int64_t n_seg, int dim, float *grid, bz_stream stream);

/*
 * Evaluate the chain at global parameters T[n_q]: T is clamped to
 * [0, n_seg], segment k = min(floor(T), n_seg-1), local t = T - k, and the
 * point is the bilinear read of the 2x2 window [A_k x_{k+1}; x_k A_{k+1}]
 * along its diagonal.  out: [dim][n_q].
 */
int bz_eval_piecewise(const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                      bz_stream stream);

/*
 * C0 piecewise cubic chain as two zig-zag layers stacked front to back (Sec.
 * 2.1: two C0 quadratic textures, interpolated in depth).  chain:
 * [3*n_seg+1][dim], segment k the cubic Bezier (P_3k, P_3k+1, P_3k+2,
 * P_3k+3).  grid: [n_seg+1][2 layers][2 rows][dim], 4(n_seg+1) texels.  Both
 * layers hold the shared endpoints A_k = P_3k in row k mod 2; their free
 * texels are the zig-zag encodings of the middle points E0_k = (3 P_3k+1 -
 * P_3k)/2 (layer 0) and E1_k = (3 P_3k+2 - P_3k+3)/2 (layer 1), formed in
 * FP64.  Evaluation: T is decoded as in bz_eval_piecewise; the point is the
 * lerp with weight t of the two layers' bilinear diagonal reads, which is the
 * cubic segment.  grid needs 16-byte alignment.  out: [dim][n_q].
 */
int bz_encode_piecewise_cubic(const float *chain, int64_t n_seg, int dim, float *grid, bz_stream stream);
int bz_eval_piecewise_cubic(const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                            bz_stream stream);

/*
 * Cache-line-tiled placement of the cubic chain (same texel values, same
 * results bit for bit).  The two layers share their on-path texel, so a
 * column is stored once as [A_k, x0_k, x1_k] (3*dim floats: the endpoint and
 * the free texels of layers 0 and 1).  A 128-byte tile holds C = 32/(3*dim)
 * consecutive columns (zero-padded), consecutive tiles overlapping by one
 * column, so tile j holds segments [jS, jS+S) with S = C-1 (3D: 2) and each
 * segment's window lies in one line.  bz_piecewise_cubic_tiled_floats: size
 * of the tiled array in floats (0 for invalid arguments).
 * bz_tile_piecewise_cubic: grid (as bz_encode_piecewise_cubic writes it) ->
 * tiles (16-byte aligned).  bz_eval_piecewise_cubic_tiled: as
 * bz_eval_piecewise_cubic on the tiles.
 */
int64_t bz_piecewise_cubic_tiled_floats(int64_t n_seg, int dim);
int bz_tile_piecewise_cubic(const float *grid, int64_t n_seg, int dim, float *tiles, bz_stream stream);
int bz_eval_piecewise_cubic_tiled(const float *tiles, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                                  bz_stream stream);

/*
 * Cache-line-tiled placement of the same zig-zag texels: 128-byte tiles of
 * C = 128/(8*dim) consecutive grid columns (16, 8, 5, 4 for dim 1..4),
 * consecutive tiles overlapping by one column, so tile j holds segments
 * [j*(C-1), (j+1)*(C-1)) and each segment's 2x2 window lies in one 128-byte
 * line.  Unused tile bytes are zero.  bz_piecewise_tiled_floats gives the
 * buffer size in floats (0 for invalid arguments; host function, no device
 * access).  tiles must be 128-byte aligned.  bz_eval_piecewise_tiled has the
 * semantics of bz_eval_piecewise.
 */
int64_t bz_piecewise_tiled_floats(int64_t n_seg, int dim);
int bz_tile_piecewise(const float *grid, int64_t n_seg, int dim, float *tiles, bz_stream stream);
int bz_eval_piecewise_tiled(const float *tiles, int64_t n_seg, int dim, const float *T, int64_t n_q, float *out,
                            bz_stream stream);

/*
 * The same tiles with 16-bit texels (dtype BZ_F16 or BZ_BF16; a storage
 * choice, not the paper's): 128-byte tiles of C = 32/dim columns (32, 16, 10,
 * 8 for dim 1..4), tile j holding segments [j*(C-1), (j+1)*(C-1)), unused
 * bytes zero, so the tiled chain takes about 2.2x fewer bytes and every query
 * still reads one line.  bz_piecewise_tiled16_halfs: buffer size in 16-bit
 * elements (0 for invalid arguments; host function).  bz_tile_piecewise16:
 * grid (FP32, as bz_encode_piecewise writes it) -> tiles, each texel rounded
 * to nearest even once (NaN stays NaN); tiles 128-byte aligned, device.
 * bz_eval_piecewise_tiled16: as bz_eval_piecewise (same parameter decode, FP32
 * arithmetic on the widened texels).  Error: the bilinear read weighs the four
 * texels of a window by (1-t)^2, t(1-t), t(1-t), t^2 (sum 1), so a result
 * differs from the FP32 tiles' by at most the largest texel rounding, 2^-11
 * (F16) or 2^-8 (BF16) of the largest |texel| of its window, plus FP32
 * rounding; the zig-zag's free texels drift like the chain's alternating sums
 * (Eq. 2), so for long chains far from the origin this can be large against a
 * segment's own size.  BZ_ERR_DTYPE for another dtype; otherwise the errors of
 * the FP32 functions.
 */
int64_t bz_piecewise_tiled16_halfs(int64_t n_seg, int dim);
int bz_tile_piecewise16(const float *grid, int64_t n_seg, int dim, int dtype, void *tiles, bz_stream stream);
int bz_eval_piecewise_tiled16(const void *tiles, int dtype, int64_t n_seg, int dim, const float *T, int64_t n_q,
                              float *out, bz_stream stream);

/*
 * Texture-filter emulation (Sec. 2: texel values at texel centres, 2x2 and
 * 2x2x2 textures holding de Casteljau levels; Sec. 2.3: filter weights in
 * fixed point with 8 fractional bits; Sec. 4 with Table 1: Seiler textures;
 * Fig. 3: the three ways of reading a cubic).  No texture unit is used: the
 * filter runs on the vector ALUs.
 *
 * Weight rule (per axis, decided in FP32 with every operation rounded as
 * written): a curve parameter p is clamped to [0,1] (clamp-to-edge), placed
 * on a two-texel axis at x = 1/4 + p/2, turned back into the texel-space
 * position xb = 2x - 1/2, and the fraction xb in [0,1] is held with
 * frac_bits fractional bits: BZ_TEXW_NEAREST rounds to nearest with halves
 * up, BZ_TEXW_TRUNCATE truncates; frac_bits = 0 leaves it unrounded
 * (0..20).  Blends are FP32 lerps.
 *
 * bz_texture_texels: texels per curve and coordinate for (degree, mode), 0
 * if unsupported.  De Casteljau and hybrid: 4(degree-1), degree 2..8;
 * Seiler: 4 (degree 2, 3) or 8 (degree 4..7).
 * bz_build_texture: ctrl[n][dim][degree+1] FP32 -> tex[n][dim][texels],
 * 2x2 layers stored [layer][row][column] (tex 16-byte aligned).
 *   de Casteljau / hybrid: layer i = [[b_i, b_i+1], [b_i+1, b_i+2]];
 *   Seiler (Table 1, d_j the difference terms, sums formed in FP64):
 *     2: [[b0, b2], [b0+d1, b2+d1]]   3: [[b0, b3], [b0+d1, b3+d2]]
 *     4: [[b0, b4], [b0, b4]], [[b0+d1, b4+d3], [b0+d1+d2, b4+d3+d2]]
 *     5: [[b0, b5], [b0, b5]], [[b0+d1, b5+d4], [b0+d1+d2, b5+d4+d3]]
 *     6, 7 (one 2x2x2 texture, the case Sec. 6 anticipates; e_j = d_{d-j}):
 *       [[b0, bd], [b0+d1, bd+e1]], [[b0+d2, bd+e2], [b0+d1+d2+d3, bd+e1+e2+e3]]
 * bz_eval_texture: tex as built, t / t_mode / out as bz_eval_bezier.
 *   BZ_TEX_DECASTELJAU: degree 2 one bilinear read at (t,t); degree >= 3 a
 *     trilinear read of layers i, i+1 at (t,t,t) per cubic sub-curve, then
 *     the remaining degree-3 de Casteljau levels as FP32 lerps with t.
 *   BZ_TEX_HYBRID: a bilinear read of every layer, then degree-2 FP32 levels.
 *   BZ_TEX_SEILER: one bilinear read at (t, st) (degree 2, 3) or trilinear at
 *     (t, st, st) (degree 4, 5) or (t, st, (st)^2) (degree 6, 7), st = (1-t)t
 *     and (st)^2 formed in FP32 before the remap.
 * bz_eval_piecewise_texemu: the zig-zag grid of bz_encode_piecewise read by
 *   the emulated bilinear filter in texel space: T is clamped to [0,N] and
 *   placed at x = T + 1/2 (texel centres at column + 1/2), k = min(floor(x -
 *   1/2), N-1), the column weight is the rounded fraction x - 1/2 - k, the
 *   row coordinate runs from the centre of row k mod 2 to the other row.
 *   n_seg 1..2^24 (FP32 texel-space coordinates); grid 8-byte aligned.
 * bz_eval_piecewise_texemu_tiled: the same reads of the same texels placed
 *   in the cache-line tiles of bz_tile_piecewise (128-byte aligned); results
 *   identical to bz_eval_piecewise_texemu on the grid the tiles came from.
 * Errors: BZ_ERR_UNSUPPORTED for a (degree, mode) pair outside the above,
 * BZ_ERR_SHAPE for counts, dim, frac_bits or rounding out of range.
 */
int bz_texture_texels(int degree, int mode);
int bz_build_texture(const float *ctrl, int64_t n_curves, int degree, int dim, int mode, float *tex, bz_stream stream);
int bz_eval_texture(const float *tex, int64_t n_curves, int degree, int dim, int mode, const float *t, int64_t n_t,
                    int t_mode, int frac_bits, int rounding, float *out, bz_stream stream);
int bz_eval_piecewise_texemu(const float *grid, int64_t n_seg, int dim, const float *T, int64_t n_q, int frac_bits,
                             int rounding, float *out, bz_stream stream);
int bz_eval_piecewise_texemu_tiled(const float *tiles, int64_t n_seg, int dim, const float *T, int64_t n_q,
                                   int frac_bits, int rounding, float *out, bz_stream stream);

/*
 * Surfaces through the emulated filter (Sec. 2.2: the surface's order splits
 * between texture reads in u and shader lerps in v; Sec. 6: Seiler surfaces
 * in the interpolator).  ctrl[n_obj][dim][(du+1)(dv+1)] FP32 (u major), du
 * 2..3, dv 1..4; tex[n_obj][dim][texels], one u-curve texture per v-index j
 * (16-byte aligned); uv[n_obj][n_per][2] (8-byte aligned), out[dim][n_obj*n_per];
 * weight rule, frac_bits and rounding as bz_eval_texture, u and v clamped to
 * [0,1].
 *   BZ_TEX_DECASTELJAU: texture j = the de Casteljau layers of the u-fibre
 *     P_0j..P_duj (4(du-1) texels), read at (u,u[,u]) -> isoline control point
 *     R_j(u); then de Casteljau over R_0..R_dv at the exact v in FP32.
 *   BZ_TEX_SEILER: the net converted to per-axis Seiler terms s (as
 *     bz_tensor_to_seiler, FP64, sums rounded once); texture j = the 2x2
 *     Seiler texture of the u-fibre of s (4 texels, Table 1).  Textures j,
 *     j+1 form a 2x2x2 texture read at (u, su, v) = L(c_j, c_j+1, v), c the
 *     isoline's v-direction Seiler terms; pairs (0,1), (2,3) by trilinear
 *     reads, the middle term of even dv by a bilinear read, then
 *     c = r0 + sv (r1 + sv c_mid) in FP32.
 * bz_texture_patch_texels: texels per patch and coordinate, 0 if unsupported.
 */
int bz_texture_patch_texels(int du, int dv, int mode);
int bz_build_texture_patch(const float *ctrl, int64_t n_obj, int du, int dv, int dim, int mode, float *tex,
                           bz_stream stream);
int bz_eval_texture_patch(const float *tex, int64_t n_obj, int du, int dv, int dim, int mode, const float *uv,
                          int64_t n_per, int frac_bits, int rounding, float *out, bz_stream stream);

/*
 * Tensor-product surfaces and volumes (Sec. 2.2: per-axis order split).
 * ctrl: [n_obj][dim][(du+1)(dv+1)(dw+1)] in dtype, index (i*(dv+1)+j)*(dw+1)+k
 * (u major).  dw = 0 for surfaces.  Degrees 1..4 per axis (dw 0..4).
 * Grid mode (uvw == NULL, surfaces only): nu x nv inclusive uniform grid,
 *   u_a = a/(nu-1), v_b = b/(nv-1); out[dim][n_obj*nu*nv], point o*nu*nv +
 *   a*nv + b.  engine selects VALU or an MFMA contraction (the MFMA engines
 *   require du = dv = 3, nu = nv = 32 and FP32 storage).  BF16 and FP16 round
 *   both operands once (error up to a few 2^-9 resp. 2^-11 of max|P|);
 *   FP16x3 scales each control-point row by a power of two, splits both
 *   operands into FP16 high + low parts and drops only the low*low product
 *   (error of order 2^-21 of the row's max|P|).
 * Points mode (uvw != NULL): uvw[n_obj][n_per][2 or 3], out[dim][n_obj*n_per];
 *   engine must be BZ_TP_VALU.
 */
int bz_eval_tensor_patch(const void *ctrl, int dtype, int64_t n_obj, int du, int dv, int dw, int dim,
                         const float *uvw, int64_t n_per, int nu, int nv, int engine, float *out,
                         bz_stream stream);

/*
 * Seiler surfaces and volumes (Sec. 3's Seiler form applied per axis of the
 * Sec. 2.2 tensor product; Sec. 6 leaves Seiler surfaces and volumes open).
 * bz_tensor_to_seiler: FP32 ctrl[n_obj][dim][(du+1)(dv+1)(dw+1)] (u major)
 *   -> sc of the same shape: every fibre of the net converted to Seiler terms
 *   [b0, bd, d1, d_{d-1}, d2, ...] along w, then v, then u, in FP64, each
 *   term rounded once.  Degrees 1..4 per axis (dw 0..4).
 * bz_eval_tensor_seiler: sc as above; grid mode (uvw == NULL, surfaces) and
 *   points mode exactly as bz_eval_tensor_patch; evaluates the nested
 *   per-axis Seiler recursion L(b0,bd,t) + st (L(d1,d_{d-1},t) + st ...) as a
 *   separable contraction with the per-axis Seiler basis (1-t, t, st(1-t),
 *   st t, ..., (st)^(d/2) for even d).  FP32 throughout.
 */
int bz_tensor_to_seiler(const float *ctrl, int64_t n_obj, int du, int dv, int dw, int dim, float *sc,
                        bz_stream stream);
int bz_eval_tensor_seiler(const float *sc, int64_t n_obj, int du, int dv, int dw, int dim, const float *uvw,
                          int64_t n_per, int nu, int nv, float *out, bz_stream stream);

/*
 * Mixed batches in one persistent launch: integral and rational Bezier
 * curves of degree 1..15, cubic NURBS (Sec. 2.2: B-splines are converted to
 * rational Bezier segments by knot insertion) and tensor-product surface
 * patches (Sec. 2.2).  All descriptor arrays are device pointers:
 *   kind_degree[n_obj]   kind << 8 | degree; kind 0 Bezier, 1 rational,
 *                        2 NURBS (degree must be 3), 3 surface patch with
 *                        degree du << 4 | dv, du and dv in 1..3
 *   cp_offset[n_obj+1]   first control point of each object; object o's
 *                        points are ctrl[cp_offset[o]*dim ...] as [dim][ncp]
 *                        (a patch's (du+1)(dv+1) points indexed i*(dv+1)+j)
 *   ctrl, w              in dtype; w aligned with control points (ignored
 *                        for kinds 0 and 3; may be NULL if no object is
 *                        rational or NURBS)
 *   knot_offset[n_obj+1], knots (FP32): NURBS knot vectors, clamped, of
 *                        length ncp+4; may be NULL if there is no NURBS
 *   n_t                  parameters per object
 * The plan reads the descriptor (synchronously), sorts objects into
 * uniform classes (kind, degree), copies the control points and weights of
 * the Bezier objects into class-sorted contiguous order, extracts the
 * rational Bezier segments of every NURBS on the GPU and keeps all of that in
 * its own device memory: none of the descriptor arrays, ctrl or w is used
 * after bz_batch_plan_create returns (changed control points need a new
 * plan).  Parameters t[n_obj][n_t] (NURBS parameters are clamped to the knot
 * range; a patch's u) and out[dim][n_obj*n_t] are passed per evaluation (out
 * must not overlap t); a plan with patches is evaluated by bz_batch_eval_uv,
 * whose v[n_obj][n_t] holds the patches' second parameters (only the rows of
 * patch objects are read), and bz_batch_eval returns BZ_ERR_NULL for it.
 * method:
 * BZ_DECASTELJAU, BZ_BERNSTEIN or BZ_AUTO.  Rational objects whose weights are all
 * positive are evaluated in FP32 (their conditioning number is 1).  Rational
 * objects with a weight that is zero, negative or NaN form classes of their
 * own whose every query takes the conditioning test of bz_eval_rational with
 * kappa = 64: sum|w_i|B_i > 64 |sum w_i B_i| (or a zero weight sum) sends the
 * point to FP64 de Casteljau on the homogeneous points.  NURBS weights must
 * be positive (BZ_ERR_UNSUPPORTED otherwise).  n_obj*n_t must stay below 2^32.
 */
typedef struct bz_plan_s *bz_plan;
int bz_batch_plan_create(int64_t n_obj, const uint16_t *kind_degree, const int64_t *cp_offset, const void *ctrl,
                         const void *w, int dtype, int dim, const int64_t *knot_offset, const float *knots,
                         int64_t n_t, int method, bz_stream stream, bz_plan *plan);
int bz_batch_eval(bz_plan plan, const float *t, float *out, bz_stream stream);
int bz_batch_eval_uv(bz_plan plan, const float *t, const float *v, float *out, bz_stream stream);
/*
 * Autotuner: times the persistent launch on (t, out) for 4 tile orders
 * (class-major, or window-major over blocks of 2^15, 2^17 or 2^18 consecutive
 * objects with every class's tiles for a window together, heaviest class
 * first: neighbouring objects' parameter rows and points, which share cache
 * lines, are then read and written closer in time, and heavy and light
 * classes alternate through the launch; for FP32 storage, in either order,
 * the NURBS tiles are spread evenly among the others) x 2 lane mappings (one query per lane, or --
 * when n_t is a multiple of 4 -- four consecutive parameters of one object per
 * lane) x 3 tile sizes (1, 2 or 4 sub-tiles of 256 lanes per tile) x 2
 * schedules (atomic tile counter, static round robin) x 4 grid sizes (4, 8,
 * 12, 16 workgroups per CU) and keeps the fastest in the plan.
 * (The timing launches of a plan with patches read the patches' v from t.)  Without
 * autotuning a plan launches 8 workgroups per CU, 4 sub-tiles per tile, the
 * static schedule, windows of 2^17 objects and four parameters per lane when
 * n_t is a multiple of 4.  Synchronises the stream.  best6 (nullable, host, 6
 * values): workgroups, sub-tiles per tile, microseconds per launch, schedule
 * (1 dynamic, 0 static), queries per lane, window (0: class-major).
 */
int bz_batch_plan_autotune(bz_plan plan, const float *t, float *out, bz_stream stream, int64_t *best6);
/*
 * Set the launch configuration by hand (what the autotuner chooses among):
 * workgroups (1..2^20), sub_tiles (1, 2, 4), schedule (1 atomic counter, 0
 * static round robin), queries_per_lane (1, or 4 when n_t is a multiple of
 * 4), window (0 for class-major tile order, else the objects per window,
 * below 2^31).  Synchronises the stream.  BZ_ERR_UNSUPPORTED for 4 queries
 * per lane with n_t not a multiple of 4.
 */
int bz_batch_plan_configure(bz_plan plan, int64_t workgroups, int sub_tiles, int schedule, int queries_per_lane,
                            int64_t window, bz_stream stream);
/* Plan statistics: n_classes, n_tiles, n_segments (NURBS), workgroups. */
int bz_batch_plan_info(bz_plan plan, int64_t *info4);
int bz_plan_destroy(bz_plan plan);

/*
 * One frame of the particle ring (Sec. 5's particle test: particles moving
 * along cubic Bezier curves chained into a closed ring, evaluated per
 * particle per frame next to other shader work).  Per particle p:
 *   T[p] <- T[p] + speed[p]*dt wrapped into [0, n_seg) (FP32, no contraction;
 *   T in [0, n_seg) and |speed*dt| < n_seg), k = min(floor T, n_seg-1),
 *   t = T - k; position pos[3][n_particles] from `ring` by method
 *     0 polynomial: ring = control points [n_seg][3][4] (Bernstein form);
 *     1 Seiler: ring = Seiler terms [n_seg][3][4] (bz_bezier_to_seiler);
 *     2 Seiler texture: ring = Seiler textures [n_seg][3][4]
 *       (bz_build_texture, BZ_TEX_SEILER) read through the emulated filter
 *       with 8-bit nearest weights at (t, st);
 *     3 sampled table: ring = [3][n_seg*samples] curve samples, entry
 *       k*samples + j the point of segment k at t = j/samples
 *       (bz_particle_ring_table); x = T*samples, i = min(floor x,
 *       n_seg*samples-1), lerp of samples i and i+1 (wrapping to sample 0)
 *       with x - i;
 *   then shade[p] = v_K of v_0 = 0, v_{i+1} = fma(23/32, v_i, x/4 - y/8 + z/16)
 *   (iters = K >= 0), a stand-in for the shader's other work.
 * ring 16-byte aligned; T is updated in place.
 */
int bz_particles_step(int method, const float *ring, int64_t n_seg, int samples, float *T, const float *speed,
                      float dt, int64_t n_particles, int iters, float *pos, float *shade, bz_stream stream);

/*
 * The sampled table of the particle ring (method 3 above; the memory-lookup
 * end of Sec. 5's comparison): ring control points [n_seg][3][4] (FP32) ->
 * table[3][n_seg*samples], entry k*samples + j the point of segment k at
 * t = j/samples (FP32 division), evaluated by de Casteljau.  n_seg 1..2^20,
 * n_seg*samples at most 2^24.
 */
int bz_particle_ring_table(const float *ring, int64_t n_seg, int samples, float *table, bz_stream stream);

/*
 * Adjoint of curve evaluation (the derivative of Sec. 2's curves): given
 * grad_out[dim][n_curves*n_t] = dL/dC, writes (overwrites)
 *   grad_ctrl[n_curves][dim][degree+1]  dL/db_i = sum_j g_j w_i B_i(t_j)/W
 *   grad_w[n_curves][degree+1]          dL/dw_i = sum_j g_j.(b_i - C_j) B_i(t_j)/W
 *   grad_t[n_curves][n_t]               dL/dt_j = g_j . C'(t_j) (hodograph)
 * w NULL means integral curves (grad_w must then be NULL).  Any gradient
 * pointer may be NULL to skip it.  grad_t requires t_mode BZ_T_PER_OBJECT.
 * The per-curve sums over j are wave reductions: no atomics, deterministic.
 */
int bz_adjoint_bezier(const float *ctrl, const float *w, int64_t n_curves, int degree, int dim, const float *t,
                      int64_t n_t, int t_mode, const float *grad_out, float *grad_ctrl, float *grad_w,
                      float *grad_t, bz_stream stream);

/*
 * Gradient of the least-squares fitting loss without an optimiser step (the
 * derivative of Sec. 2's curves with respect to their control points and
 * parameters), for callers that run their own optimiser.  Integral curves,
 * per-curve parameters:
 *   L = (1/M) sum_q |C(t_q) - y_q|^2,  M = n_curves*n_t,
 *   ctrl[n_curves][dim][degree+1], t[n_curves][n_t], target y[dim][n_curves*n_t].
 * Writes (overwrites), each output nullable to skip it:
 *   loss_part[n_curves]                   curve c's contribution to L (their sum is L)
 *   grad_ctrl[n_curves][dim][degree+1]    dL/db_i = (2/M) sum_j (C(t_j) - y_j) B_i(t_j)
 *   grad_t[n_curves][n_t]                 dL/dt_j = (2/M) (C(t_j) - y_j) . C'(t_j), C' the hodograph
 * The per-curve sums are wave reductions: no atomics, deterministic.  Inputs
 * are not modified.  Every array is FP32 with 4-byte alignment
 * (BZ_ERR_ALIGN otherwise); ctrl, t and target are required (BZ_ERR_NULL).
 */
int bz_l2_fit_adjoint(const float *ctrl, int64_t n_curves, int degree, int dim, const float *t, int64_t n_t,
                      const float *target, float *loss_part, float *grad_ctrl, float *grad_t, bz_stream stream);

/*
 * One fused least-squares fitting step for integral curves with per-curve
 * parameters: loss L = (1/M) sum_q |C(t_q) - y_q|^2 (M = n_curves*n_t), its
 * gradients by the adjoint above, and an Adam update (bias-corrected, step
 * counted from 1; bias corrections applied as FP64-computed reciprocals, the
 * square root and the final reciprocal by the hardware approximations, about
 * 1 ulp) of ctrl and t in place, t clamped to [0,1].
 * y: [dim][n_curves*n_t].  m_*, v_*: Adam moments, same shapes as ctrl / t.
 * loss_part (nullable): [n_curves] per-curve contributions to L before the
 * update.  Requires n_t <= 1024.
 */
int bz_fit_adam_step(float *ctrl, float *t, const float *y, int64_t n_curves, int degree, int dim, int64_t n_t,
                     float *m_ctrl, float *v_ctrl, float *m_t, float *v_t, int step, float lr, float beta1,
                     float beta2, float eps, float *loss_part, bz_stream stream);

/*
 * n_steps consecutive fitting steps (steps first_step .. first_step+n_steps-1),
 * with exactly the results of n_steps calls of bz_fit_adam_step.  Curves are
 * optimised independently, so when n_t <= 128 (<= 256 if dim*(degree+1) > 32)
 * all steps run in one launch with each curve's samples, parameters and Adam
 * moments held in registers; otherwise the single steps are captured once into
 * a HIP graph and replayed.  loss_part receives the last step's loss.
 * Synchronises the stream.
 */
int bz_fit_adam_run(float *ctrl, float *t, const float *y, int64_t n_curves, int degree, int dim, int64_t n_t,
                    float *m_ctrl, float *v_ctrl, float *m_t, float *v_t, int first_step, int n_steps, float lr,
                    float beta1, float beta2, float eps, float *loss_part, bz_stream stream);

/*
 * Measurement utilities.  These are not part of the method: they measure the
 * memory system the evaluators run on, so that each kernel's rate can be set
 * against a ceiling measured on the same GPU (beside the published 8 TB/s of
 * MI355X HBM).
 *
 * bz_device_cu_count: number of compute units of the current device (0 on
 * failure).
 *
 * bz_hbm_probe: a streaming kernel over n floats (n a multiple of 4, buffers
 * 16-byte aligned) with a persistent grid of blocks_per_cu x (CU count)
 * workgroups of 256 threads (blocks_per_cu 1..64), or with blocks_per_cu 0
 * one 16-byte vector per thread.  mode 0: read src (dst[0] is written only if
 * a thread's partial sum equals -1, which non-negative data never gives); 1:
 * write dst; 2: copy src to dst.  Timing is the caller's (events around the
 * call).
 *
 * bz_gather_probe: the ceiling of a random one-line-per-query gather, the
 * access pattern of a chain query in cache-line tiles (one window read per
 * query at an arbitrary position along the chain): n_reads reads, read r
 * loading vec16 (1..4) consecutive 16-byte vectors from the start of line
 * floor(h(r) * n_lines / 2^32) of src, h the lowbias32 hash of
 * r * 0x9e3779b9 + 12345 and n_lines = n / 32.  src: n floats (a multiple of
 * 32 below 2^37), 128-byte aligned, device.  sink: one device float, written
 * only if a thread's partial sum equals -1 (never for non-negative data).
 * n_reads 0..2^31-1; 0 launches nothing.  Timing is the caller's.
 */
int bz_device_cu_count(void);
int bz_hbm_probe(int mode, const float *src, float *dst, int64_t n, int blocks_per_cu, bz_stream stream);
int bz_gather_probe(const float *src, int64_t n, int64_t n_reads, int vec16, float *sink, bz_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BZ_H */
