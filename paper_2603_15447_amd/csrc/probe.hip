// HBM bandwidth probe: streaming read, write and copy kernels that give the
// measured ceiling the evaluators' rooflines are compared with.  16-byte
// vector accesses, grid-stride loops over a persistent grid of 4 waves per
// CU times an occupancy factor; the read kernel folds what it loads into one
// value per thread, stored only when it equals a sentinel the data never
// holds, so the loads cannot be elided.
#include "common.h"

namespace bzi {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_probe_read(const v4f *__restrict__ src, int64_t n4,
                                                       float *__restrict__ sink) {
    float acc = 0.0f;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += stride) {
        const v4f v = __builtin_nontemporal_load(src + i);
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == -1.0f) sink[0] = acc;  // never true for the probe's data (all ones)
}

__global__ __launch_bounds__(kBlock) void k_probe_write(v4f *__restrict__ dst, int64_t n4) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    const v4f one = v4f{1.0f, 1.0f, 1.0f, 1.0f};
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(one, dst + i);
}

__global__ __launch_bounds__(kBlock) void k_probe_copy(const v4f *__restrict__ src, v4f *__restrict__ dst,
                                                       int64_t n4) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" int bz_hbm_probe(int mode, const float *src, float *dst, int64_t n, int blocks_per_cu, bz_stream stream) {
    return guarded("bz_hbm_probe", [&]() -> int {
        const char *fn = "bz_hbm_probe";
        if (mode < 0 || mode > 2) return fail(BZ_ERR_SHAPE, "%s: mode %d (0 read, 1 write, 2 copy)", fn, mode);
        if (n < 0 || n % 4 != 0) return fail(BZ_ERR_SHAPE, "%s: n %lld not a multiple of 4", fn, (long long)n);
        if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(BZ_ERR_SHAPE, "%s: blocks_per_cu", fn);
        if (n == 0) return BZ_OK;
        if ((mode != 1 && !src) || !dst) return fail(BZ_ERR_NULL, "%s: buffers are required", fn);
        if (!aligned(src, 16) || !aligned(dst, 16)) return fail(BZ_ERR_ALIGN, "%s: 16-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const uint32_t blocks = static_cast<uint32_t>(bz_device_cu_count() * blocks_per_cu);
        const int64_t n4 = n / 4;
        if (mode == 0)
            hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(kBlock), 0, s, reinterpret_cast<const v4f *>(src),
                               n4, dst);
        else if (mode == 1)
            hipLaunchKernelGGL(k_probe_write, dim3(blocks), dim3(kBlock), 0, s, reinterpret_cast<v4f *>(dst), n4);
        else
            hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(kBlock), 0, s, reinterpret_cast<const v4f *>(src),
                               reinterpret_cast<v4f *>(dst), n4);
        BZ_CHECK_LAUNCH("k_probe");
        return BZ_OK;
    });
}
