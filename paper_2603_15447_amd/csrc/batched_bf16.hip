// Persistent mixed-batch kernel instantiated for bf16_t storage (both forms).
#include "batched_impl.h"

namespace bzi {

template int launch_batch_kernel<FORM_DC, bf16_t>(uint32_t, const BatchArgs &, hipStream_t);
template int launch_batch_kernel<FORM_BERN, bf16_t>(uint32_t, const BatchArgs &, hipStream_t);

}  // namespace bzi
