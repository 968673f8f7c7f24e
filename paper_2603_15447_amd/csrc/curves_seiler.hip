// Explicit instantiations of the curve kernels for the SEILER form.
#include "curves_impl.h"

namespace bzi {
template int launch_curves_t<FORM_SEILER, false, float>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_SEILER, false, _Float16>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_SEILER, false, bf16_t>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_SEILER, true, float>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_SEILER, true, _Float16>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_SEILER, true, bf16_t>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_SEILER_PRE, false, float>(int, int, const CurveArgs &, hipStream_t);
}  // namespace bzi
