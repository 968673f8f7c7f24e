// Mixed batches (integral / rational Bezier curves of degree 1..15 and cubic
// NURBS) evaluated by one persistent launch on gfx950.
//
// Plan (host, once): objects are sorted into uniform classes (kind, degree)
// so that every 256-query tile, and hence every wavefront, runs one code path;
// NURBS are cut into rational Bezier segments by knot insertion on the GPU
// (Sec. 2.2: B-splines become piecewise Bezier curves via Boehm's algorithm)
// with the breakpoints kept for a per-query span search; tiles are ordered by
// estimated cost, heaviest first.
// Evaluation: a grid of (CUs x occupancy) workgroups pulls tiles from an atomic
// counter; the last workgroup to finish resets the counters, so consecutive
// launches (and graph replays) need no memset.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "curves_impl.h"

struct bz_plan_s;

namespace bzi {
namespace {

constexpr int kNurbsP = 3;

struct ClassInfo {
    int32_t kind;     // 0 Bezier, 1 rational, 2 NURBS
    int32_t degree;   // 1..15 (3 for NURBS)
    int32_t first;    // first slot of the class in perm
    int32_t count;    // objects in the class
};

struct Tile {
    int32_t cls;
    uint32_t q0;  // first query of the tile within its class
};

struct BatchArgs {
    const void *ctrl;
    const void *w;
    const int64_t *cp_offset;
    const int32_t *perm;
    const ClassInfo *classes;
    const Tile *tiles;
    uint32_t n_tiles;
    uint32_t qpt;          // sub-tiles of kBlock queries per tile
    const int32_t *nurbs_rank;
    const int32_t *seg_first;  // [n_nurbs+1]
    const float *brk;          // breakpoints, nseg+1 per NURBS, at seg_first[r] + r
    const float *seg;          // [n_segs][4][dim+1] homogeneous
    const float *t;
    float *out;
    int64_t plane;
    uint32_t n_t;
    FastDiv div_nt;
    int dim;
    unsigned int *counters;    // [0] next tile, [1] finished workgroups
};

// Load n contiguous storage elements as FP32.
template <typename T, int N>
__device__ __forceinline__ void load_row(const T *__restrict__ p, float (&v)[N]) {
    if constexpr (std::is_same<T, float>::value) {
        typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
        constexpr int V = N / 4;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const f4u x = *reinterpret_cast<const f4u *>(p + 4 * i);
            v[4 * i] = x[0];
            v[4 * i + 1] = x[1];
            v[4 * i + 2] = x[2];
            v[4 * i + 3] = x[3];
        }
#pragma unroll
        for (int i = 4 * V; i < N; ++i) v[i] = p[i];
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = to_f32<T>(p[i]);
    }
}

// One query of a degree-D (rational) Bezier object; P is [dim][D+1].
template <int D, bool RAT, int F, typename T>
__device__ __forceinline__ void eval_curve_query(const T *__restrict__ P, const T *__restrict__ W, int dim, float t,
                                                 float *__restrict__ out, int64_t plane, int64_t q) {
    float wv[D + 1];
    if constexpr (RAT) load_row<T, D + 1>(W, wv);
    if constexpr (F == FORM_BERN) {
        float B[D + 1];
        bernstein_basis<D>(t, B);
        float den = 1.0f;
        if constexpr (RAT) {
#pragma unroll
            for (int i = 0; i <= D; ++i) B[i] *= wv[i];
            den = B[0];
#pragma unroll
            for (int i = 1; i <= D; ++i) den += B[i];
        }
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
            if (k < dim) {
                float b[D + 1];
                load_row<T, D + 1>(P + k * (D + 1), b);
                const float v = dot_basis<D>(B, b);
                st_stream(out + k * plane + q, RAT ? v / den : v);
            }
        }
    } else {
        float den = 1.0f;
        if constexpr (RAT) den = eval_dc<D>(wv, t);
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
            if (k < dim) {
                float b[D + 1];
                load_row<T, D + 1>(P + k * (D + 1), b);
                if constexpr (RAT) {
#pragma unroll
                    for (int i = 0; i <= D; ++i) b[i] *= wv[i];
                }
                const float v = eval_dc<D>(b, t);
                st_stream(out + k * plane + q, RAT ? v / den : v);
            }
        }
    }
}

// One query of a NURBS object: clamp, binary search of the span among the
// segment breakpoints, rational cubic Bezier of that segment.
__device__ __forceinline__ void eval_nurbs_query(const float *__restrict__ brk, const float *__restrict__ seg, int nseg,
                                                 int dim, float u, float *__restrict__ out, int64_t plane, int64_t q) {
    const float lo_u = brk[0], hi_u = brk[nseg];
    u = u < lo_u ? lo_u : u;  // NaN passes
    u = u > hi_u ? hi_u : u;
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (brk[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    const float a = brk[lo], b = brk[lo + 1];
    const float tl = (u - a) / (b - a);
    float B[4];
    bernstein_basis<3>(tl, B);
    const float *__restrict__ S = seg + static_cast<size_t>(lo) * 4 * (dim + 1);
    float H[kMaxDim + 1] = {};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k <= kMaxDim; ++k)
            if (k <= dim) H[k] = __builtin_fmaf(B[i], S[i * (dim + 1) + k], H[k]);
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k)
        if (k < dim) st_stream(out + k * plane + q, H[k] / H[dim]);
}

template <int D, bool RAT, int F, typename T>
__device__ __forceinline__ void run_curve_tile(const BatchArgs &a, const ClassInfo &ci, uint32_t q0) {
    const uint32_t nq = static_cast<uint32_t>(ci.count) * a.n_t;
    for (uint32_t s = 0; s < a.qpt; ++s) {
        const uint32_t qi = q0 + s * kBlock + threadIdx.x;
        if (qi >= nq) return;
        const uint32_t slot = fdiv(qi, a.div_nt);
        const uint32_t j = qi - slot * a.n_t;
        const int64_t o = a.perm[ci.first + slot];
        const int64_t q = o * a.n_t + j;
        const float t = a.t[q];
        const int64_t cp = a.cp_offset[o];
        const T *P = static_cast<const T *>(a.ctrl) + cp * a.dim;
        const T *W = RAT ? static_cast<const T *>(a.w) + cp : nullptr;
        eval_curve_query<D, RAT, F, T>(P, W, a.dim, t, a.out, a.plane, q);
    }
}

__device__ __forceinline__ void run_nurbs_tile(const BatchArgs &a, const ClassInfo &ci, uint32_t q0) {
    const uint32_t nq = static_cast<uint32_t>(ci.count) * a.n_t;
    for (uint32_t s = 0; s < a.qpt; ++s) {
        const uint32_t qi = q0 + s * kBlock + threadIdx.x;
        if (qi >= nq) return;
        const uint32_t slot = fdiv(qi, a.div_nt);
        const uint32_t j = qi - slot * a.n_t;
        const int64_t o = a.perm[ci.first + slot];
        const int64_t q = o * a.n_t + j;
        const int r = a.nurbs_rank[o];
        const int s0 = a.seg_first[r], nseg = a.seg_first[r + 1] - s0;
        eval_nurbs_query(a.brk + s0 + r, a.seg + static_cast<size_t>(s0) * 4 * (a.dim + 1), nseg, a.dim, a.t[q], a.out,
                         a.plane, q);
    }
}

template <bool RAT, int F, typename T>
__device__ __forceinline__ void dispatch_degree(const BatchArgs &a, const ClassInfo &ci, uint32_t q0) {
    switch (ci.degree) {
        case 1: run_curve_tile<1, RAT, F, T>(a, ci, q0); break;
        case 2: run_curve_tile<2, RAT, F, T>(a, ci, q0); break;
        case 3: run_curve_tile<3, RAT, F, T>(a, ci, q0); break;
        case 4: run_curve_tile<4, RAT, F, T>(a, ci, q0); break;
        case 5: run_curve_tile<5, RAT, F, T>(a, ci, q0); break;
        case 6: run_curve_tile<6, RAT, F, T>(a, ci, q0); break;
        case 7: run_curve_tile<7, RAT, F, T>(a, ci, q0); break;
        case 8: run_curve_tile<8, RAT, F, T>(a, ci, q0); break;
        case 9: run_curve_tile<9, RAT, F, T>(a, ci, q0); break;
        case 10: run_curve_tile<10, RAT, F, T>(a, ci, q0); break;
        case 11: run_curve_tile<11, RAT, F, T>(a, ci, q0); break;
        case 12: run_curve_tile<12, RAT, F, T>(a, ci, q0); break;
        case 13: run_curve_tile<13, RAT, F, T>(a, ci, q0); break;
        case 14: run_curve_tile<14, RAT, F, T>(a, ci, q0); break;
        default: run_curve_tile<15, RAT, F, T>(a, ci, q0); break;
    }
}

template <int F, typename T>
__global__ __launch_bounds__(kBlock) void k_batch_persistent(BatchArgs a) {
    __shared__ unsigned int s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&a.counters[0], 1u);
        __syncthreads();
        const unsigned int tile = s_tile;
        __syncthreads();
        if (tile >= a.n_tiles) break;
        const Tile tl = a.tiles[tile];
        const ClassInfo ci = a.classes[tl.cls];
        if (ci.kind == 0) dispatch_degree<false, F, T>(a, ci, tl.q0);
        else if (ci.kind == 1) dispatch_degree<true, F, T>(a, ci, tl.q0);
        else run_nurbs_tile(a, ci, tl.q0);
    }
    // every workgroup has seen the end of the tile list; the last one to get
    // here resets both counters for the next launch
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.counters[1], 1u) == gridDim.x - 1) {
            atomicExch(&a.counters[0], 0u);
            atomicExch(&a.counters[1], 0u);
        }
    }
}

// Bezier extraction of one clamped cubic NURBS by knot insertion: every
// interior knot is raised to multiplicity p, leaving one rational Bezier
// segment (4 homogeneous points) per non-empty knot span.  Works left to
// right on a window of p+1 points, so only O(p) state is kept.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nurbs_extract(int n_nurbs, const int64_t *__restrict__ nurbs_obj,
                                                          const int64_t *__restrict__ cp_offset,
                                                          const int64_t *__restrict__ knot_offset,
                                                          const T *__restrict__ ctrl, const T *__restrict__ w,
                                                          const float *__restrict__ knots,
                                                          const int32_t *__restrict__ seg_first, int dim,
                                                          float *__restrict__ seg) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= n_nurbs) return;
    constexpr int p = kNurbsP;
    const int64_t o = nurbs_obj[r];
    const int64_t cp = cp_offset[o];
    const int ncp = static_cast<int>(cp_offset[o + 1] - cp);
    const float *U = knots + knot_offset[o];
    const int m = ncp + p;  // index of the last knot
    const T *P = ctrl + cp * dim;
    const T *Wt = w + cp;
    const int H = dim + 1;
    auto pw = [&](int i, int k) -> double {  // homogeneous control point i, coordinate k
        const double wi = static_cast<double>(to_f32<T>(Wt[i]));
        return k == dim ? wi : wi * static_cast<double>(to_f32<T>(P[static_cast<int64_t>(k) * ncp + i]));
    };
    double Q[p + 1][kMaxDim + 1], Nx[p + 1][kMaxDim + 1];
    for (int i = 0; i <= p; ++i)
        for (int k = 0; k < H; ++k) Q[i][k] = pw(i, k);
    float *out = seg + static_cast<size_t>(seg_first[r]) * 4 * H;
    const int nseg = seg_first[r + 1] - seg_first[r];
    int a = p, b = p + 1, ns = 0;
    while (b < m && ns < nseg) {
        const int i0 = b;
        while (b < m && U[b + 1] == U[b]) ++b;
        const int mult = b - i0 + 1;
        int rr = 0;
        if (mult < p) {
            const double numer = static_cast<double>(U[b]) - U[a];
            double alpha[p];
            for (int j = p; j > mult; --j) alpha[j - mult - 1] = numer / (static_cast<double>(U[a + j]) - U[a]);
            rr = p - mult;
            for (int j = 1; j <= rr; ++j) {
                const int save = rr - j, s = mult + j;
                for (int k = p; k >= s; --k) {
                    const double al = alpha[k - s];
                    for (int c = 0; c < H; ++c) Q[k][c] = al * Q[k][c] + (1.0 - al) * Q[k - 1][c];
                }
                if (b < m)
                    for (int c = 0; c < H; ++c) Nx[save][c] = Q[p][c];
            }
        }
        for (int i = 0; i <= p; ++i)
            for (int c = 0; c < H; ++c) out[(static_cast<size_t>(ns) * 4 + i) * H + c] = static_cast<float>(Q[i][c]);
        ++ns;
        if (b < m) {
            for (int i = (mult < p ? p - mult : 0); i <= p; ++i)
                for (int c = 0; c < H; ++c) Nx[i][c] = pw(b - p + i, c);
            for (int i = 0; i <= p; ++i)
                for (int c = 0; c < H; ++c) Q[i][c] = Nx[i][c];
            a = b;
            ++b;
        }
    }
}

int class_cost(int kind, int degree, int method, int dim) {
    const int ch = dim + (kind != 0 ? 1 : 0);
    if (kind == 2) return 60 + 4 * ch;
    if (method == BZ_DECASTELJAU) return degree * (degree + 1) / 2 * ch * 2 + 8;
    return 3 * degree + (degree + 1) * ch + 8;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

struct bz_plan_s {
    int64_t n_obj = 0, n_t = 0;
    int dim = 0, dtype = 0, method = 0;
    const void *ctrl = nullptr, *w = nullptr;  // caller-owned storage (must outlive the plan)
    // device copies owned by the plan
    int64_t *cp_offset = nullptr;
    int32_t *perm = nullptr;
    ClassInfo *classes = nullptr;
    Tile *tiles = nullptr;
    int32_t *nurbs_rank = nullptr, *seg_first = nullptr;
    float *brk = nullptr, *seg = nullptr;
    unsigned int *counters = nullptr;
    int n_classes = 0;
    uint32_t n_tiles = 0, qpt = 1;
    int64_t n_segs = 0;
    uint32_t workgroups = 0;
};

namespace {

void plan_free(bz_plan_s *p) {
    if (!p) return;
    void *bufs[] = {p->cp_offset, p->perm, p->classes, p->tiles, p->nurbs_rank, p->seg_first, p->brk, p->seg,
                    p->counters};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

template <typename X>
int dev_upload(X **dst, const std::vector<X> &src, hipStream_t s) {
    const size_t n = std::max<size_t>(src.size(), 1) * sizeof(X);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), n);
    if (e == hipErrorOutOfMemory) return fail(BZ_ERR_NOMEM, "bz_batch_plan_create: device allocation");
    BZ_CHECK_HIP(e);
    if (!src.empty()) BZ_CHECK_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice, s));
    return BZ_OK;
}

int launch_batch(const bz_plan_s *p, const float *t, float *out, hipStream_t s, uint32_t workgroups, uint32_t qpt) {
    BatchArgs a;
    a.ctrl = p->ctrl;
    a.w = p->w;
    a.cp_offset = p->cp_offset;
    a.perm = p->perm;
    a.classes = p->classes;
    a.tiles = p->tiles;
    a.n_tiles = p->n_tiles;
    a.qpt = qpt;
    a.nurbs_rank = p->nurbs_rank;
    a.seg_first = p->seg_first;
    a.brk = p->brk;
    a.seg = p->seg;
    a.t = t;
    a.out = out;
    a.plane = p->n_obj * p->n_t;
    a.n_t = static_cast<uint32_t>(p->n_t);
    a.div_nt = make_fastdiv(a.n_t);
    a.dim = p->dim;
    a.counters = p->counters;
    const dim3 g(workgroups), b(kBlock);
    const bool dc = p->method == BZ_DECASTELJAU;
    if (p->dtype == BZ_F32) {
        if (dc) hipLaunchKernelGGL((k_batch_persistent<FORM_DC, float>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_batch_persistent<FORM_BERN, float>), g, b, 0, s, a);
    } else if (p->dtype == BZ_F16) {
        if (dc) hipLaunchKernelGGL((k_batch_persistent<FORM_DC, _Float16>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_batch_persistent<FORM_BERN, _Float16>), g, b, 0, s, a);
    } else {
        if (dc) hipLaunchKernelGGL((k_batch_persistent<FORM_DC, bf16_t>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_batch_persistent<FORM_BERN, bf16_t>), g, b, 0, s, a);
    }
    BZ_CHECK_LAUNCH("k_batch_persistent");
    return BZ_OK;
}

// Rebuild the tile list for `qpt` sub-tiles per tile (heaviest class first).
int build_tiles(bz_plan_s *p, const std::vector<ClassInfo> &cls, uint32_t qpt, hipStream_t s) {
    std::vector<int> order(cls.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return class_cost(cls[x].kind, cls[x].degree, p->method, p->dim) >
               class_cost(cls[y].kind, cls[y].degree, p->method, p->dim);
    });
    std::vector<Tile> tiles;
    const uint64_t span = static_cast<uint64_t>(kBlock) * qpt;
    for (int c : order) {
        const uint64_t nq = static_cast<uint64_t>(cls[c].count) * p->n_t;
        for (uint64_t q0 = 0; q0 < nq; q0 += span) tiles.push_back(Tile{c, static_cast<uint32_t>(q0)});
    }
    if (p->tiles) BZ_CHECK_HIP(hipFree(p->tiles));
    p->tiles = nullptr;
    int rc = dev_upload(&p->tiles, tiles, s);
    if (rc) return rc;
    p->n_tiles = static_cast<uint32_t>(tiles.size());
    p->qpt = qpt;
    return BZ_OK;
}

}  // namespace

extern "C" {

int bz_batch_plan_create(int64_t n_obj, const uint16_t *kind_degree, const int64_t *cp_offset, const void *ctrl,
                         const void *w, int dtype, int dim, const int64_t *knot_offset, const float *knots,
                         int64_t n_t, int method, bz_stream stream, bz_plan *plan) {
    return guarded("bz_batch_plan_create", [&]() -> int {
        const char *fn = "bz_batch_plan_create";
        if (!plan) return fail(BZ_ERR_NULL, "%s: plan is required", fn);
        *plan = nullptr;
        if (n_obj < 0 || n_t < 0) return fail(BZ_ERR_SHAPE, "%s: negative count", fn);
        if (dim < 1 || dim > kMaxDim) return fail(BZ_ERR_SHAPE, "%s: dim %d", fn, dim);
        if (dtype_size(dtype) == 0) return fail(BZ_ERR_DTYPE, "%s: dtype %d", fn, dtype);
        if (method != BZ_DECASTELJAU && method != BZ_BERNSTEIN) return fail(BZ_ERR_UNSUPPORTED, "%s: method %d", fn, method);
        if (n_obj > (int64_t(1) << 31) - 1 || (n_obj > 0 && n_t > ((int64_t(1) << 32) - 1) / std::max<int64_t>(n_obj, 1)))
            return fail(BZ_ERR_SHAPE, "%s: n_obj*n_t must stay below 2^32", fn);
        if (n_obj > 0 && (!kind_degree || !cp_offset || !ctrl))
            return fail(BZ_ERR_NULL, "%s: kind_degree, cp_offset and ctrl are required", fn);
        const hipStream_t s = as_stream(stream);
        std::vector<uint16_t> kd(n_obj);
        std::vector<int64_t> cpo(n_obj + 1, 0), ko;
        if (n_obj > 0) {
            BZ_CHECK_HIP(hipMemcpyAsync(kd.data(), kind_degree, n_obj * sizeof(uint16_t), hipMemcpyDeviceToHost, s));
            BZ_CHECK_HIP(hipMemcpyAsync(cpo.data(), cp_offset, (n_obj + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            BZ_CHECK_HIP(hipStreamSynchronize(s));
        }
        // classes: kind 0/1 x degree 1..15, kind 2 (cubic NURBS)
        std::vector<int64_t> count(32, 0);
        bool need_w = false, any_nurbs = false;
        for (int64_t o = 0; o < n_obj; ++o) {
            const int kind = kd[o] >> 8, deg = kd[o] & 0xff;
            const int64_t ncp = cpo[o + 1] - cpo[o];
            if (kind > 2) return fail(BZ_ERR_SHAPE, "%s: object %lld has kind %d", fn, (long long)o, kind);
            if (kind == 2) {
                if (deg != kNurbsP) return fail(BZ_ERR_UNSUPPORTED, "%s: NURBS object %lld has degree %d (only cubic)", fn, (long long)o, deg);
                if (ncp < 4) return fail(BZ_ERR_SHAPE, "%s: NURBS object %lld has %lld control points", fn, (long long)o, (long long)ncp);
                any_nurbs = true;
            } else {
                if (deg < 1 || deg > kMaxDegree) return fail(BZ_ERR_SHAPE, "%s: object %lld degree %d", fn, (long long)o, deg);
                if (ncp != deg + 1) return fail(BZ_ERR_SHAPE, "%s: object %lld has %lld control points for degree %d", fn, (long long)o, (long long)ncp, deg);
            }
            if (kind != 0) need_w = true;
            count[kind == 2 ? 30 : kind * 15 + deg - 1] += 1;
        }
        if (need_w && !w) return fail(BZ_ERR_NULL, "%s: weights are required (rational or NURBS objects)", fn);
        if (!aligned(ctrl, dtype_size(dtype)) || !aligned(w, dtype_size(dtype)))
            return fail(BZ_ERR_ALIGN, "%s: misaligned ctrl or w", fn);
        // NURBS knot vectors: read, validate (clamped, non-decreasing), count segments
        std::vector<int64_t> nurbs_obj;
        std::vector<int32_t> seg_first(1, 0), rank(n_obj, -1);
        std::vector<float> brk;
        if (any_nurbs) {
            if (!knot_offset || !knots) return fail(BZ_ERR_NULL, "%s: knot_offset and knots are required for NURBS", fn);
            ko.resize(n_obj + 1);
            BZ_CHECK_HIP(hipMemcpyAsync(ko.data(), knot_offset, (n_obj + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            BZ_CHECK_HIP(hipStreamSynchronize(s));
            const int64_t nk_total = ko[n_obj];
            std::vector<float> U(nk_total);
            BZ_CHECK_HIP(hipMemcpyAsync(U.data(), knots, nk_total * sizeof(float), hipMemcpyDeviceToHost, s));
            BZ_CHECK_HIP(hipStreamSynchronize(s));
            for (int64_t o = 0; o < n_obj; ++o) {
                if ((kd[o] >> 8) != 2) continue;
                const int64_t ncp = cpo[o + 1] - cpo[o];
                const int64_t nk = ko[o + 1] - ko[o];
                if (nk != ncp + kNurbsP + 1 || ko[o] < 0 || ko[o + 1] > nk_total)
                    return fail(BZ_ERR_SHAPE, "%s: NURBS object %lld needs %lld knots", fn, (long long)o, (long long)(ncp + 4));
                const float *u = U.data() + ko[o];
                for (int64_t i = 0; i + 1 < nk; ++i)
                    if (!(u[i] <= u[i + 1])) return fail(BZ_ERR_SHAPE, "%s: NURBS object %lld knots not sorted", fn, (long long)o);
                if (u[0] != u[kNurbsP] || u[nk - 1] != u[nk - 1 - kNurbsP] || !(u[kNurbsP] < u[kNurbsP + 1]) ||
                    !(u[nk - 2 - kNurbsP] < u[nk - 1 - kNurbsP]))
                    return fail(BZ_ERR_SHAPE, "%s: NURBS object %lld knot vector is not clamped with end multiplicity 4", fn, (long long)o);
                rank[o] = static_cast<int32_t>(nurbs_obj.size());
                nurbs_obj.push_back(o);
                int32_t ns = 0;
                brk.push_back(u[kNurbsP]);
                for (int64_t i = kNurbsP; i < ncp; ++i)
                    if (u[i] < u[i + 1]) {
                        brk.push_back(u[i + 1]);
                        ++ns;
                    }
                seg_first.push_back(seg_first.back() + ns);
            }
        }
        // class list and permutation (stable counting sort)
        std::vector<ClassInfo> cls;
        std::vector<int32_t> cls_of_key(32, -1);
        int32_t first = 0;
        for (int key = 0; key < 31; ++key) {
            if (count[key] == 0) continue;
            ClassInfo ci;
            ci.kind = key == 30 ? 2 : key / 15;
            ci.degree = key == 30 ? kNurbsP : key % 15 + 1;
            ci.first = first;
            ci.count = static_cast<int32_t>(count[key]);
            cls_of_key[key] = static_cast<int32_t>(cls.size());
            cls.push_back(ci);
            first += ci.count;
        }
        std::vector<int32_t> perm(n_obj), fill(cls.size(), 0);
        for (int64_t o = 0; o < n_obj; ++o) {
            const int kind = kd[o] >> 8, deg = kd[o] & 0xff;
            const int c = cls_of_key[kind == 2 ? 30 : kind * 15 + deg - 1];
            perm[cls[c].first + fill[c]++] = static_cast<int32_t>(o);
        }
        bz_plan_s *p = new (std::nothrow) bz_plan_s();
        if (!p) return fail(BZ_ERR_NOMEM, "%s: host allocation", fn);
        p->n_obj = n_obj;
        p->n_t = n_t;
        p->dim = dim;
        p->dtype = dtype;
        p->method = method;
        p->ctrl = ctrl;
        p->w = w;
        p->n_classes = static_cast<int>(cls.size());
        p->n_segs = seg_first.back();
        int rc = dev_upload(&p->cp_offset, cpo, s);
        if (!rc) rc = dev_upload(&p->perm, perm, s);
        if (!rc) rc = dev_upload(&p->classes, cls, s);
        if (!rc) rc = dev_upload(&p->nurbs_rank, rank, s);
        if (!rc) rc = dev_upload(&p->seg_first, seg_first, s);
        if (!rc) rc = dev_upload(&p->brk, brk, s);
        if (!rc) rc = build_tiles(p, cls, 1, s);
        if (!rc) {
            hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->seg), std::max<int64_t>(p->n_segs, 1) * 4 * (dim + 1) * sizeof(float));
            if (e != hipSuccess) rc = e == hipErrorOutOfMemory ? fail(BZ_ERR_NOMEM, "%s: segments", fn) : hip_fail(e, "hipMalloc");
        }
        if (!rc) {
            hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->counters), 2 * sizeof(unsigned int));
            if (e == hipSuccess) e = hipMemsetAsync(p->counters, 0, 2 * sizeof(unsigned int), s);
            if (e != hipSuccess) rc = hip_fail(e, "counters");
        }
        if (!rc && !nurbs_obj.empty()) {
            int64_t *nobj_d = nullptr;
            rc = dev_upload(&nobj_d, nurbs_obj, s);
            if (!rc) {
                const int nn = static_cast<int>(nurbs_obj.size());
                const uint32_t blocks = (nn + kBlock - 1) / kBlock;
                if (dtype == BZ_F32)
                    hipLaunchKernelGGL((k_nurbs_extract<float>), dim3(blocks), dim3(kBlock), 0, s, nn, nobj_d, p->cp_offset,
                                       knot_offset, static_cast<const float *>(ctrl), static_cast<const float *>(w), knots,
                                       p->seg_first, dim, p->seg);
                else if (dtype == BZ_F16)
                    hipLaunchKernelGGL((k_nurbs_extract<_Float16>), dim3(blocks), dim3(kBlock), 0, s, nn, nobj_d,
                                       p->cp_offset, knot_offset, static_cast<const _Float16 *>(ctrl),
                                       static_cast<const _Float16 *>(w), knots, p->seg_first, dim, p->seg);
                else
                    hipLaunchKernelGGL((k_nurbs_extract<bf16_t>), dim3(blocks), dim3(kBlock), 0, s, nn, nobj_d,
                                       p->cp_offset, knot_offset, static_cast<const bf16_t *>(ctrl),
                                       static_cast<const bf16_t *>(w), knots, p->seg_first, dim, p->seg);
                hipError_t e = hipGetLastError();
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                (void)hipFree(nobj_d);
                if (e != hipSuccess) rc = hip_fail(e, "k_nurbs_extract");
            }
        }
        if (!rc) {
            int blocks_per_cu = 0, dev = 0, cus = 0;
            hipError_t e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e == hipSuccess)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, k_batch_persistent<FORM_BERN, float>, kBlock, 0);
            if (e != hipSuccess) rc = hip_fail(e, "occupancy query");
            p->workgroups = static_cast<uint32_t>(std::max(1, cus) * std::max(1, blocks_per_cu));
        }
        if (!rc) rc = hipStreamSynchronize(s) == hipSuccess ? BZ_OK : fail(BZ_ERR_HIP, "%s: sync", fn);
        if (rc) {
            plan_free(p);
            return rc;
        }
        *plan = p;
        return BZ_OK;
    });
}

int bz_batch_eval(bz_plan plan, const float *t, float *out, bz_stream stream) {
    return guarded("bz_batch_eval", [&]() -> int {
        if (!plan) return fail(BZ_ERR_NULL, "bz_batch_eval: plan is required");
        if (plan->n_obj == 0 || plan->n_t == 0) return BZ_OK;
        if (!t || !out) return fail(BZ_ERR_NULL, "bz_batch_eval: t and out are required");
        if (!aligned(t, 4) || !aligned(out, 4)) return fail(BZ_ERR_ALIGN, "bz_batch_eval: misaligned");
        return launch_batch(plan, t, out, as_stream(stream), plan->workgroups, plan->qpt);
    });
}

int bz_batch_plan_autotune(bz_plan plan, const float *t, float *out, bz_stream stream, int64_t *best4) {
    return guarded("bz_batch_plan_autotune", [&]() -> int {
        if (!plan) return fail(BZ_ERR_NULL, "bz_batch_plan_autotune: plan is required");
        if (plan->n_obj == 0 || plan->n_t == 0) return BZ_OK;
        if (!t || !out) return fail(BZ_ERR_NULL, "bz_batch_plan_autotune: t and out are required");
        const hipStream_t s = as_stream(stream);
        hipEvent_t e0, e1;
        BZ_CHECK_HIP(hipEventCreate(&e0));
        BZ_CHECK_HIP(hipEventCreate(&e1));
        const uint32_t base = plan->workgroups;
        std::vector<ClassInfo> cls(plan->n_classes);
        BZ_CHECK_HIP(hipMemcpy(cls.data(), plan->classes, cls.size() * sizeof(ClassInfo), hipMemcpyDeviceToHost));
        float best = 1e30f;
        uint32_t best_wg = base, best_q = plan->qpt;
        const uint32_t qpts[] = {1, 2, 4};
        const double wgf[] = {0.5, 1.0, 2.0};
        for (uint32_t q : qpts) {
            int rc = build_tiles(plan, cls, q, s);
            if (rc) return rc;
            for (double f : wgf) {
                const uint32_t wg = std::max<uint32_t>(1, static_cast<uint32_t>(base * f));
                rc = launch_batch(plan, t, out, s, wg, q);  // warm-up
                if (rc) return rc;
                BZ_CHECK_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < 5; ++r) {
                    rc = launch_batch(plan, t, out, s, wg, q);
                    if (rc) return rc;
                }
                BZ_CHECK_HIP(hipEventRecord(e1, s));
                BZ_CHECK_HIP(hipEventSynchronize(e1));
                float ms = 0;
                BZ_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_wg = wg;
                    best_q = q;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        int rc = build_tiles(plan, cls, best_q, s);
        if (rc) return rc;
        plan->workgroups = best_wg;
        BZ_CHECK_HIP(hipStreamSynchronize(s));
        if (best4) {
            best4[0] = best_wg;
            best4[1] = best_q;
            best4[2] = static_cast<int64_t>(best * 1000.0f / 5.0f);  // microseconds per launch
            best4[3] = plan->n_tiles;
        }
        return BZ_OK;
    });
}

int bz_batch_plan_info(bz_plan plan, int64_t *info4) {
    if (!plan || !info4) return fail(BZ_ERR_NULL, "bz_batch_plan_info: plan and info are required");
    info4[0] = plan->n_classes;
    info4[1] = plan->n_tiles;
    info4[2] = plan->n_segs;
    info4[3] = plan->workgroups;
    return BZ_OK;
}

int bz_plan_destroy(bz_plan plan) {
    return guarded("bz_plan_destroy", [&]() -> int {
        plan_free(plan);
        return BZ_OK;
    });
}

}  // extern "C"
