// C ABI of the curve evaluators: bz_eval_bezier, bz_bezier_to_seiler,
// bz_eval_seiler, bz_eval_rational.  Validation, chunking (at most 2^30
// queries per launch so all in-kernel indices stay 32-bit) and dispatch.
#include "curves_impl.h"

namespace bzi {

extern template int launch_curves_t<FORM_DC, false, float>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_DC, false, _Float16>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_DC, false, bf16_t>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_DC, true, float>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_DC, true, _Float16>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_DC, true, bf16_t>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_BERN, false, float>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_BERN, false, _Float16>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_BERN, false, bf16_t>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_BERN, true, float>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_BERN, true, _Float16>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_BERN, true, bf16_t>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER, false, float>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER, false, _Float16>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER, false, bf16_t>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER, true, float>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER, true, _Float16>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER, true, bf16_t>(int, int, const CurveArgs &, hipStream_t);
extern template int launch_curves_t<FORM_SEILER_PRE, false, float>(int, int, const CurveArgs &, hipStream_t);

namespace {

constexpr int64_t kMaxLaunchQueries = int64_t(1) << 30;

template <typename T>
int dispatch_form(int form, bool rat, int degree, int dim, const CurveArgs &a, hipStream_t s) {
    switch (form) {
        case FORM_DC: return rat ? launch_curves_t<FORM_DC, true, T>(degree, dim, a, s)
                                 : launch_curves_t<FORM_DC, false, T>(degree, dim, a, s);
        case FORM_BERN: return rat ? launch_curves_t<FORM_BERN, true, T>(degree, dim, a, s)
                                   : launch_curves_t<FORM_BERN, false, T>(degree, dim, a, s);
        case FORM_SEILER: return rat ? launch_curves_t<FORM_SEILER, true, T>(degree, dim, a, s)
                                     : launch_curves_t<FORM_SEILER, false, T>(degree, dim, a, s);
        default: return fail(BZ_ERR_INTERNAL, "bad form %d", form);
    }
}

int check_common(const char *fn, int64_t n_curves, int degree, int dim, int64_t n_t, int t_mode) {
    if (degree < 1 || degree > kMaxDegree) return fail(BZ_ERR_SHAPE, "%s: degree %d not in 1..%d", fn, degree, kMaxDegree);
    if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d not in 1..%d", fn, dim, kMaxDim);
    if (n_curves < 0 || n_t < 0) return fail(BZ_ERR_SHAPE, "%s: negative count", fn);
    if (n_t > kMaxLaunchQueries) return fail(BZ_ERR_SHAPE, "%s: n_t %lld above 2^30", fn, (long long)n_t);
    if (n_curves > 0 && n_t > 0 && n_curves > (int64_t(1) << 62) / n_t)
        return fail(BZ_ERR_SHAPE, "%s: n_curves*n_t overflows", fn);
    if (t_mode != BZ_T_SHARED && t_mode != BZ_T_PER_OBJECT) return fail(BZ_ERR_SHAPE, "%s: bad t_mode %d", fn, t_mode);
    return BZ_OK;
}

// Split the call into launches of at most 2^30 queries (whole curves).
int run_chunks(int form, bool rat, int dt, const void *ctrl, const void *w, int64_t n_curves, int degree, int dim,
               const float *t, int64_t n_t, int t_mode, float kappa, float *out, uint32_t *n_fixed, hipStream_t s) {
    const int64_t nq = n_curves * n_t;
    const int64_t per = std::max<int64_t>(1, kMaxLaunchQueries / n_t);
    const int es = dtype_size(dt);
    for (int64_t c0 = 0; c0 < n_curves; c0 += per) {
        const int64_t nc = std::min(per, n_curves - c0);
        CurveArgs a;
        a.ctrl = static_cast<const char *>(ctrl) + c0 * dim * (degree + 1) * es;
        a.w = w ? static_cast<const char *>(w) + c0 * (degree + 1) * es : nullptr;
        a.t = t;
        a.out = out;
        a.plane = nq;
        a.q0 = c0 * n_t;
        a.c0 = c0;
        a.nq = static_cast<uint32_t>(nc * n_t);
        a.div_nt = make_fastdiv(static_cast<uint32_t>(n_t));
        a.per_object = t_mode == BZ_T_PER_OBJECT;
        a.kappa = kappa;
        a.n_fixed = n_fixed;
        int rc;
        if (form == FORM_SEILER_PRE) rc = launch_curves_t<FORM_SEILER_PRE, false, float>(degree, dim, a, s);
        else if (dt == BZ_F32) rc = dispatch_form<float>(form, rat, degree, dim, a, s);
        else if (dt == BZ_F16) rc = dispatch_form<_Float16>(form, rat, degree, dim, a, s);
        else rc = dispatch_form<bf16_t>(form, rat, degree, dim, a, s);
        if (rc != BZ_OK) return rc;
    }
    return BZ_OK;
}

template <typename T>
int launch_to_seiler(int degree, const void *ctrl, float *seiler, uint32_t rows, hipStream_t s) {
    const uint32_t blocks = (rows + kBlock - 1) / kBlock;
    const T *p = static_cast<const T *>(ctrl);
#define BZI_SEILER_CASE(D) \
    case D: hipLaunchKernelGGL((k_to_seiler<D, T>), dim3(blocks), dim3(kBlock), 0, s, p, seiler, rows); break;
    switch (degree) {
        BZI_SEILER_CASE(1) BZI_SEILER_CASE(2) BZI_SEILER_CASE(3) BZI_SEILER_CASE(4) BZI_SEILER_CASE(5)
        BZI_SEILER_CASE(6) BZI_SEILER_CASE(7) BZI_SEILER_CASE(8) BZI_SEILER_CASE(9) BZI_SEILER_CASE(10)
        BZI_SEILER_CASE(11) BZI_SEILER_CASE(12) BZI_SEILER_CASE(13) BZI_SEILER_CASE(14) BZI_SEILER_CASE(15)
        default: return fail(BZ_ERR_SHAPE, "degree %d", degree);
    }
#undef BZI_SEILER_CASE
    BZ_CHECK_LAUNCH("k_to_seiler");
    return BZ_OK;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

int bz_eval_bezier(const void *ctrl, int ctrl_dtype, int64_t n_curves, int degree, int dim, const float *t,
                   int64_t n_t, int t_mode, int method, float *out, bz_stream stream) {
    return guarded("bz_eval_bezier", [&]() -> int {
        int rc = check_common("bz_eval_bezier", n_curves, degree, dim, n_t, t_mode);
        if (rc) return rc;
        if (dtype_size(ctrl_dtype) == 0) return fail(BZ_ERR_DTYPE, "bz_eval_bezier: dtype %d", ctrl_dtype);
        if (method == BZ_AUTO) method = BZ_BERNSTEIN;
        if (method != BZ_DECASTELJAU && method != BZ_BERNSTEIN && method != BZ_SEILER)
            return fail(BZ_ERR_UNSUPPORTED, "bz_eval_bezier: method %d", method);
        if (n_curves == 0 || n_t == 0) return BZ_OK;
        if (!ctrl || !t || !out) return fail(BZ_ERR_NULL, "bz_eval_bezier: ctrl, t and out are required");
        if (!aligned(ctrl, dtype_size(ctrl_dtype)) || !aligned(t, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "bz_eval_bezier: misaligned pointer");
        return run_chunks(method, false, ctrl_dtype, ctrl, nullptr, n_curves, degree, dim, t, n_t, t_mode, 0.0f, out,
                          nullptr, as_stream(stream));
    });
}

int bz_eval_rational(const void *ctrl, const void *w, int dtype, int64_t n_curves, int degree, int dim,
                     const float *t, int64_t n_t, int t_mode, int method, float kappa, float *out,
                     uint32_t *n_fixed, bz_stream stream) {
    return guarded("bz_eval_rational", [&]() -> int {
        int rc = check_common("bz_eval_rational", n_curves, degree, dim, n_t, t_mode);
        if (rc) return rc;
        if (dtype_size(dtype) == 0) return fail(BZ_ERR_DTYPE, "bz_eval_rational: dtype %d", dtype);
        if (method == BZ_AUTO) method = BZ_BERNSTEIN;
        if (method != BZ_DECASTELJAU && method != BZ_BERNSTEIN && method != BZ_SEILER)
            return fail(BZ_ERR_UNSUPPORTED, "bz_eval_rational: method %d", method);
        if (n_curves == 0 || n_t == 0) return BZ_OK;
        if (!ctrl || !w || !t || !out) return fail(BZ_ERR_NULL, "bz_eval_rational: ctrl, w, t and out are required");
        if (!aligned(ctrl, dtype_size(dtype)) || !aligned(w, dtype_size(dtype)) || !aligned(t, 4) ||
            !aligned(out, 4) || !aligned(n_fixed, 4))
            return fail(BZ_ERR_ALIGN, "bz_eval_rational: misaligned pointer");
        return run_chunks(method, true, dtype, ctrl, w, n_curves, degree, dim, t, n_t, t_mode, kappa, out, n_fixed,
                          as_stream(stream));
    });
}

int bz_bezier_to_seiler(const void *ctrl, int ctrl_dtype, int64_t n_curves, int degree, int dim, float *seiler,
                        bz_stream stream) {
    return guarded("bz_bezier_to_seiler", [&]() -> int {
        int rc = check_common("bz_bezier_to_seiler", n_curves, degree, dim, 1, BZ_T_SHARED);
        if (rc) return rc;
        if (dtype_size(ctrl_dtype) == 0) return fail(BZ_ERR_DTYPE, "bz_bezier_to_seiler: dtype %d", ctrl_dtype);
        if (n_curves == 0) return BZ_OK;
        if (!ctrl || !seiler) return fail(BZ_ERR_NULL, "bz_bezier_to_seiler: ctrl and seiler are required");
        if (!aligned(ctrl, dtype_size(ctrl_dtype)) || !aligned(seiler, 4))
            return fail(BZ_ERR_ALIGN, "bz_bezier_to_seiler: misaligned pointer");
        const int es = dtype_size(ctrl_dtype);
        const int64_t rows = n_curves * dim;
        const int64_t per = kMaxLaunchQueries;
        for (int64_t r0 = 0; r0 < rows; r0 += per) {
            const uint32_t nr = static_cast<uint32_t>(std::min(per, rows - r0));
            const void *p = static_cast<const char *>(ctrl) + r0 * (degree + 1) * es;
            float *o = seiler + r0 * (degree + 1);
            const hipStream_t s = as_stream(stream);
            rc = ctrl_dtype == BZ_F32   ? launch_to_seiler<float>(degree, p, o, nr, s)
                 : ctrl_dtype == BZ_F16 ? launch_to_seiler<_Float16>(degree, p, o, nr, s)
                                        : launch_to_seiler<bf16_t>(degree, p, o, nr, s);
            if (rc) return rc;
        }
        return BZ_OK;
    });
}

int bz_eval_seiler(const float *seiler, int64_t n_curves, int degree, int dim, const float *t, int64_t n_t,
                   int t_mode, float *out, bz_stream stream) {
    return guarded("bz_eval_seiler", [&]() -> int {
        int rc = check_common("bz_eval_seiler", n_curves, degree, dim, n_t, t_mode);
        if (rc) return rc;
        if (n_curves == 0 || n_t == 0) return BZ_OK;
        if (!seiler || !t || !out) return fail(BZ_ERR_NULL, "bz_eval_seiler: seiler, t and out are required");
        if (!aligned(seiler, 4) || !aligned(t, 4) || !aligned(out, 4))
            return fail(BZ_ERR_ALIGN, "bz_eval_seiler: misaligned pointer");
        return run_chunks(FORM_SEILER_PRE, false, BZ_F32, seiler, nullptr, n_curves, degree, dim, t, n_t, t_mode, 0.0f,
                          out, nullptr, as_stream(stream));
    });
}

}  // extern "C"
