// Persistent mixed-batch kernel instantiated for one (form, storage) pair,
// one translation unit each so they compile in parallel.
#include "batched_impl.h"

namespace bzi {

template int launch_batch_kernel<FORM_BERN, float>(uint32_t, const BatchArgs &, hipStream_t);

int batch_kernel_blocks_per_cu(int *blocks) {
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        blocks, batch_dev::k_batch_persistent<FORM_BERN, float, 1>, kBlock, 0);
    return e == hipSuccess ? BZ_OK : hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
}

}  // namespace bzi
