// Explicit instantiations of the curve kernels for the BERN form.
#include "curves_impl.h"

namespace bzi {
template int launch_curves_t<FORM_BERN, false, float>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_BERN, false, _Float16>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_BERN, false, bf16_t>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_BERN, true, float>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_BERN, true, _Float16>(int, int, const CurveArgs &, hipStream_t);
template int launch_curves_t<FORM_BERN, true, bf16_t>(int, int, const CurveArgs &, hipStream_t);
}  // namespace bzi
