// Explicit instantiations of the curve kernels for the DC form.
#include "curves_impl.h"

namespace bzi {
template int launch_curves_t<FORM_DC, false, float>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_DC, false, _Float16>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_DC, false, bf16_t>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_DC, true, float>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_DC, true, _Float16>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_DC, true, bf16_t>(int, int, const CurveArgs &, hipStream_t);
}  // namespace bzi
