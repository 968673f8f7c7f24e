// Persistent mixed-batch kernel instantiated for one (form, storage) pair,
// one translation unit each so they compile in parallel.
#include "batched_impl.h"

namespace bzi {

template int launch_batch_kernel<FORM_BERN, float>(uint32_t, const BatchArgs &, hipStream_t);

}  // namespace bzi
