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

// lowbias32, a 32-bit integer finaliser published by C. Wellons (hash-prospector):
// two xorshift-multiply rounds and a final xorshift.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Read r (r < n_reads) loads NV consecutive 16-byte vectors from the start of
// line floor(h(r) * n_lines / 2^32); four reads per thread, all issued before
// any is consumed, as in the chain evaluator.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_probe_gather(const v4f *__restrict__ src, uint32_t n_lines,
                                                         uint32_t n_reads, float *__restrict__ sink) {
    constexpr int QPT = 4;
    const uint32_t base = blockIdx.x * (kBlock * QPT) + threadIdx.x;
    v4f v[QPT][NV];
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
        const uint32_t r = min(base + i * kBlock, n_reads - 1);
        const uint32_t h = lowbias32(r * 0x9e3779b9u + 0x3039u);
        const uint32_t line = static_cast<uint32_t>((static_cast<uint64_t>(h) * n_lines) >> 32);
        const v4f *p = src + static_cast<size_t>(line) * 8;
#pragma unroll
        for (int e = 0; e < NV; ++e) v[i][e] = p[e];
    }
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
        for (int e = 0; e < NV; ++e) acc += v[i][e].x + v[i][e].w;
    if (acc == -1.0f) sink[0] = acc;  // never true for non-negative data
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" int bz_gather_probe(const float *src, int64_t n, int64_t n_reads, int vec16, float *sink,
                               bz_stream stream) {
    return guarded("bz_gather_probe", [&]() -> int {
        const char *fn = "bz_gather_probe";
        if (vec16 < 1 || vec16 > 4) return fail(BZ_ERR_SHAPE, "%s: vec16 %d not in 1..4", fn, vec16);
        if (n < 0 || n % 32 != 0 || n / 32 > 0xffffffffll)
            return fail(BZ_ERR_SHAPE, "%s: n %lld not a multiple of 32 floats (one line) below 2^37", fn,
                        (long long)n);
        if (n_reads < 0 || n_reads > 0x7fffffffll) return fail(BZ_ERR_SHAPE, "%s: n_reads not in 0..2^31-1", fn);
        if (n_reads == 0) return BZ_OK;
        if (n == 0) return fail(BZ_ERR_SHAPE, "%s: reads from an empty buffer", fn);
        if (!src || !sink) return fail(BZ_ERR_NULL, "%s: src and sink are required", fn);
        if (!aligned(src, 128) || !aligned(sink, 4)) return fail(BZ_ERR_ALIGN, "%s: src needs 128-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const uint32_t nl = static_cast<uint32_t>(n / 32), nr = static_cast<uint32_t>(n_reads);
        const uint32_t per_block = kBlock * 4;
        const dim3 grid((nr + per_block - 1) / per_block);
        const v4f *p = reinterpret_cast<const v4f *>(src);
        switch (vec16) {
            case 1: hipLaunchKernelGGL(k_probe_gather<1>, grid, dim3(kBlock), 0, s, p, nl, nr, sink); break;
            case 2: hipLaunchKernelGGL(k_probe_gather<2>, grid, dim3(kBlock), 0, s, p, nl, nr, sink); break;
            case 3: hipLaunchKernelGGL(k_probe_gather<3>, grid, dim3(kBlock), 0, s, p, nl, nr, sink); break;
            default: hipLaunchKernelGGL(k_probe_gather<4>, grid, dim3(kBlock), 0, s, p, nl, nr, sink); break;
        }
        BZ_CHECK_LAUNCH("k_probe_gather");
        return BZ_OK;
    });
}

extern "C" int bz_hbm_probe(int mode, const float *src, float *dst, int64_t n, int blocks_per_cu, bz_stream stream) {
    return guarded("bz_hbm_probe", [&]() -> int {
        const char *fn = "bz_hbm_probe";
        if (mode < 0 || mode > 2) return fail(BZ_ERR_SHAPE, "%s: mode %d (0 read, 1 write, 2 copy)", fn, mode);
        if (n < 0 || n % 4 != 0) return fail(BZ_ERR_SHAPE, "%s: n %lld not a multiple of 4", fn, (long long)n);
        if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(BZ_ERR_SHAPE, "%s: blocks_per_cu", fn);
        if (n == 0) return BZ_OK;
        if ((mode != 1 && !src) || !dst) return fail(BZ_ERR_NULL, "%s: buffers are required", fn);
        if (!aligned(src, 16) || !aligned(dst, 16)) return fail(BZ_ERR_ALIGN, "%s: 16-byte alignment", fn);
        const hipStream_t s = as_stream(stream);
        const int64_t n4 = n / 4;
        // blocks_per_cu 0: one 16-byte vector per thread (a grid as large as the data)
        if (blocks_per_cu == 0 && (n4 + kBlock - 1) / kBlock > 0x7fffffffll)
            return fail(BZ_ERR_SHAPE, "%s: n too large for one vector per thread", fn);
        const uint32_t blocks = blocks_per_cu == 0 ? static_cast<uint32_t>((n4 + kBlock - 1) / kBlock)
                                                   : static_cast<uint32_t>(bz_device_cu_count() * blocks_per_cu);
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
