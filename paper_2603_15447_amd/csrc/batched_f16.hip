// Persistent mixed-batch kernel instantiated for _Float16 storage (both forms).
#include "batched_impl.h"

namespace bzi {

template int launch_batch_kernel<FORM_DC, _Float16>(uint32_t, const BatchArgs &, hipStream_t);
template int launch_batch_kernel<FORM_BERN, _Float16>(uint32_t, const BatchArgs &, hipStream_t);

}  // namespace bzi
