// Zig-zag encoder of C0 piecewise chains (Sec. 2.1, Eq. 2, Fig. 2): the free
// texels of a chain of N segments are fixed by x_0 = M_0 and x_k + x_{k+1} =
// 2 M_k, an alternating prefix sum over the middle points, evaluated here as
// a three-pass FP64 block scan (per-block partials, one serial pass over the
// block partials, write): every texel is one FP32 rounding of an FP64 prefix
// sum, where an FP32 recurrence x_{k+1} = 2 M_k - x_k would let the rounding
// error grow with k.
#include <mutex>

#include "common.h"

namespace bzi {
namespace {

constexpr int kEncPerThread = 8;
constexpr int kEncPerBlock = kBlock * kEncPerThread;

// The encoder works on "channels": a quadratic chain has dim channels (one
// per coordinate); a cubic chain (Sec. 2.1, two zig-zag layers stacked front
// to back) has 2*dim, layer l of coordinate c being channel l*dim + c.  Both
// layers share the on-path texels A_k = P_3k; their middle points satisfy
// 2 E0_k = 3 P_3k+1 - P_3k and 2 E1_k = 3 P_3k+2 - P_3k+3 (exact in FP64),
// so that the depth lerp of the two layers is the cubic (P_3k .. P_3k+3).
struct EncSrc {
    const float *chain;
    int64_t n_seg;
    int dim;
    int cubic;  // 0: quadratic chain [2N+1][dim]; 1: cubic chain [3N+1][dim]
};

__device__ __forceinline__ double enc_twice_mid(const EncSrc &e, int ch, int64_t k) {
    if (!e.cubic) return 2.0 * static_cast<double>(e.chain[(2 * k + 1) * e.dim + ch]);
    const int layer = ch >= e.dim, c = ch - layer * e.dim;
    const double a = e.chain[(3 * k + (layer ? 3 : 0)) * e.dim + c];
    const double b = e.chain[(3 * k + (layer ? 2 : 1)) * e.dim + c];
    return 3.0 * b - a;
}

__device__ __forceinline__ float enc_endpoint(const EncSrc &e, int ch, int64_t k) {
    const int c = ch - (ch >= e.dim ? e.dim : 0);
    return e.chain[(e.cubic ? 3 * k : 2 * k) * e.dim + c];
}

// Element e_k = (-1)^(k+1) * 2 M_k of the alternating sum: the free texels are
// x_k = (-1)^k y_k with y_k = M_0 + sum_{j<k} e_j, which is x_{k+1} = 2M_k - x_k.
__device__ __forceinline__ double enc_elem(const EncSrc &e, int ch, int64_t k) {
    if (k >= e.n_seg) return 0.0;
    const double m2 = enc_twice_mid(e, ch, k);
    return (k & 1) ? m2 : -m2;
}

// Inclusive scan of one double per thread over the block (four waves).
__device__ double block_scan_incl(double v, double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    double pre = 0.0;
    for (int w = 0; w < wave; ++w) pre += lds[w];
    __syncthreads();
    return v + pre;
}

__global__ __launch_bounds__(kBlock) void k_enc_partials(EncSrc e, int nch, double *__restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    const int64_t k0 = static_cast<int64_t>(blockIdx.x) * kEncPerBlock + threadIdx.x * kEncPerThread;
    for (int ch = 0; ch < nch; ++ch) {
        double s = 0.0;
        for (int i = 0; i < kEncPerThread; ++i) s += enc_elem(e, ch, k0 + i);
        const double tot = block_scan_incl(s, lds);
        if (threadIdx.x == kBlock - 1) partial[static_cast<int64_t>(blockIdx.x) * nch + ch] = tot;
    }
}

// Exclusive scan of the block partials (one block, serial over chunks),
// seeded with y_0 = M_0.
__global__ __launch_bounds__(kBlock) void k_enc_offsets(EncSrc e, int nch, int64_t nb, double *__restrict__ partial) {
    __shared__ double lds[kBlock / 64];
    __shared__ double total;
    for (int ch = 0; ch < nch; ++ch) {
        double carry = 0.5 * enc_twice_mid(e, ch, 0);
        for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
            const int64_t b = b0 + threadIdx.x;
            const double v = b < nb ? partial[b * nch + ch] : 0.0;
            const double incl = block_scan_incl(v, lds);
            if (b < nb) partial[b * nch + ch] = carry + (incl - v);
            if (threadIdx.x == kBlock - 1) total = incl;
            __syncthreads();
            carry += total;
            __syncthreads();
        }
    }
}

// Writes column k of every channel: the endpoint in row k mod 2, the free
// texel in the other row.  Output [N+1][layers][2][dim] (layers = nch/dim).
__global__ __launch_bounds__(kBlock) void k_enc_write(EncSrc e, int nch, const double *__restrict__ offsets,
                                                      float *__restrict__ grid) {
    __shared__ double lds[kBlock / 64];
    const int64_t k0 = static_cast<int64_t>(blockIdx.x) * kEncPerBlock + threadIdx.x * kEncPerThread;
    const int layers = nch / e.dim;
    for (int ch = 0; ch < nch; ++ch) {
        const int layer = ch / e.dim, c = ch - layer * e.dim;
        double ev[kEncPerThread];
        double s = 0.0;
        for (int i = 0; i < kEncPerThread; ++i) {
            ev[i] = enc_elem(e, ch, k0 + i);
            s += ev[i];
        }
        const double incl = block_scan_incl(s, lds);
        double y = offsets[static_cast<int64_t>(blockIdx.x) * nch + ch] + (incl - s);
        for (int i = 0; i < kEncPerThread; ++i) {
            const int64_t k = k0 + i;
            if (k > e.n_seg) break;
            const int r = static_cast<int>(k & 1);
            const double x = r ? -y : y;
            float *col = grid + (k * layers + layer) * 2 * e.dim;
            col[r * e.dim + c] = enc_endpoint(e, ch, k);
            col[(1 - r) * e.dim + c] = static_cast<float>(x);
            y += ev[i];
        }
    }
}

}  // namespace

// Workspace of the allocation-free encoder: the block partials (one double
// per block of kEncPerBlock columns and channel) in a file-scope device array.
// Each device holds its own copy until the process ends; host code reaches it
// only through the device address looked up per device below (the array's
// name in host code is a host-side stand-in, not a device address).
constexpr int64_t kEncScratchDoubles = int64_t(1) << 18;  // 2 MiB
static __device__ __align__(256) double scratch[kEncScratchDoubles];

namespace {

// Largest chain the workspace holds: nb * dim <= kEncScratchDoubles with
// nb = ceil((n_seg + 1) / kEncPerBlock).
int64_t noalloc_max_seg(int dim) { return (kEncScratchDoubles / dim) * kEncPerBlock - 1; }

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
int scratch_address(const char *fn, double **out) {
    int dev = 0;
    BZ_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchMaxDevices) return fail(BZ_ERR_UNSUPPORTED, "%s: device %d", fn, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return BZ_OK;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

extern "C" {

// ws: caller-provided workspace of at least nb*nch doubles, or NULL for a
// stream-ordered allocation freed after the launches.
static int encode_chain(const char *fn, const float *chain, int64_t n_seg, int dim, int cubic, float *grid,
                        bz_stream stream, double *ws = nullptr) {
    if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
    if (n_seg < 0 || n_seg > (int64_t(1) << 40)) return fail(BZ_ERR_SHAPE, "%s: n_seg %lld", fn, (long long)n_seg);
    if (n_seg == 0) return BZ_OK;
    if (!chain || !grid) return fail(BZ_ERR_NULL, "%s: chain and grid are required", fn);
    if (!aligned(chain, 4) || !aligned(grid, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
    const hipStream_t s = as_stream(stream);
    const int nch = dim * (cubic ? 2 : 1);
    const int64_t nb = (n_seg + 1 + kEncPerBlock - 1) / kEncPerBlock;
    double *partial = ws;
    if (!ws) {
        hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&partial), sizeof(double) * nb * nch, s);
        if (e == hipErrorOutOfMemory) return fail(BZ_ERR_NOMEM, "%s: workspace", fn);
        BZ_CHECK_HIP(e);
    }
    // every partial is written by k_enc_partials before it is read: the
    // workspace needs no clearing
    const EncSrc src{chain, n_seg, dim, cubic};
    hipLaunchKernelGGL(k_enc_partials, dim3(static_cast<uint32_t>(nb)), dim3(kBlock), 0, s, src, nch, partial);
    hipLaunchKernelGGL(k_enc_offsets, dim3(1), dim3(kBlock), 0, s, src, nch, nb, partial);
    hipLaunchKernelGGL(k_enc_write, dim3(static_cast<uint32_t>(nb)), dim3(kBlock), 0, s, src, nch, partial, grid);
    const hipError_t le = hipGetLastError();
    if (!ws) BZ_CHECK_HIP(hipFreeAsync(partial, s));
    if (le != hipSuccess) return hip_fail(le, fn);
    return BZ_OK;
}

int bz_encode_piecewise_noalloc(const float *chain, int64_t n_seg, int dim, float *grid, bz_stream stream) {
    return guarded("bz_encode_piecewise_noalloc", [&]() -> int {
        const char *fn = "bz_encode_piecewise_noalloc";
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (n_seg < 0 || n_seg > noalloc_max_seg(dim))
            return fail(BZ_ERR_SHAPE, "%s: n_seg %lld outside 0..%lld, the workspace limit for dim %d", fn,
                        (long long)n_seg, (long long)noalloc_max_seg(dim), dim);
        if (n_seg == 0) return BZ_OK;
        double *ws = nullptr;
        const int rc = scratch_address(fn, &ws);
        if (rc) return rc;
        return encode_chain(fn, chain, n_seg, dim, 0, grid, stream, ws);
    });
}


int bz_encode_piecewise(const float *chain, int64_t n_seg, int dim, float *grid, bz_stream stream) {
    return guarded("bz_encode_piecewise",
                   [&]() -> int { return encode_chain("bz_encode_piecewise", chain, n_seg, dim, 0, grid, stream); });
}

int bz_encode_piecewise_cubic(const float *chain, int64_t n_seg, int dim, float *grid, bz_stream stream) {
    return guarded("bz_encode_piecewise_cubic", [&]() -> int {
        return encode_chain("bz_encode_piecewise_cubic", chain, n_seg, dim, 1, grid, stream);
    });
}

}  // extern "C"
