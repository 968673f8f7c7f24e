// Device code of the mixed-batch evaluator (see batched.hip for the plan):
// the persistent kernel and its per-class tile evaluators.  Included by the
// translation units that instantiate the kernel per storage type, so the six
// (form x storage) instantiations compile in parallel.
#pragma once
#include "curves_impl.h"

namespace bzi {

constexpr int kNurbsP = 3;

struct ClassInfo {
    int32_t kind;       // 0 Bezier, 1 rational (all weights > 0), 2 NURBS, 3 rational with a weight <= 0,
                        // 4 tensor-product surface patch
    int32_t degree;     // 1..15 (3 for NURBS; du << 4 | dv for patches)
    int32_t first;      // first slot of the class in perm
    int32_t count;      // objects in the class
    int64_t ctrl_base;  // first element of the class in the sorted control points
    int64_t w_base;     // first element of the class in the sorted weights (rational)
};

// A tile carries its class record, so a workgroup needs one scalar load per tile.
struct Tile {
    ClassInfo ci;
    uint32_t q0;   // first query of the tile within its class
    uint32_t q1;   // end of the tile's queries (exclusive, a multiple of n_t)
    uint32_t qpt;  // sub-tiles of kBlock lanes in this tile (1..4)
    uint32_t pad;
};

// Span lookup of a NURBS query, two ways (the persistent kernel takes the
// faster for its storage type, measured on a mixed batch in steady state):
// - bucket table (FP32 storage): the parameter range [lo, hi] of NURBS r is
//   cut into M = 2*nseg equal buckets; a parameter of bucket m lies in one of
//   the segments tab[m].s .. tab[m+1].s (indices relative to the NURBS), and
//   when those are two segments, tab[m].split (the breakpoint between them)
//   decides.  More than two candidates (two or more breakpoints in one
//   bucket) fall back to a binary search over the breakpoints of that range.
// - binary search over the NURBS's nseg+1 breakpoints (16-bit storage): a line
//   or two that the 16 queries of a NURBS share, where the table costs one
//   more random line per query.  With FP32 control rows streaming past, the
//   search's dependent probes miss the cache and the table is faster; with
//   16-bit rows they hit, and the search is.
struct NurbsHead {
    int32_t s0;    // first segment of the NURBS in the plan's segment array
    int32_t nseg;  // segments (non-empty knot spans)
    int32_t tab0;  // first of its 2*nseg+1 table entries
    int32_t brk0;  // first of its nseg+1 breakpoints (s0 + rank)
    float lo, hi;  // parameter range
    float inv_h;   // M / (hi - lo); 0 when that is not finite (one bucket)
    int32_t pad;
};

struct NurbsTab {
    int32_t s;    // first candidate segment of the bucket
    float split;  // breakpoint after segment s (start of segment s+1)
};

// Bucket of parameter u (already clamped to [lo, hi]).  Evaluated identically
// on the host (table construction) and on the device (queries): one
// subtraction, one multiplication, clamp and floor, so it is a monotone
// function of u and a breakpoint's bucket bounds the buckets of the
// parameters on either side of it.  NaN lands in bucket 0.
__host__ __device__ inline int nurbs_bucket(float u, float lo, float inv_h, int n_buckets) {
    float x = (u - lo) * inv_h;
    x = x > 0.0f ? x : 0.0f;
    x = floorf(x);
    const float top = static_cast<float>(n_buckets - 1);
    x = x < top ? x : top;
    return static_cast<int>(x);
}

// Control points per object of a class: degree+1, or (du+1)(dv+1) for a patch.
__host__ __device__ inline int class_ncp(int kind, int degree) {
    return kind == 4 ? ((degree >> 4) + 1) * ((degree & 15) + 1) : degree + 1;
}

struct BatchArgs {
    const void *ctrl_s;        // control points in class-sorted order (plan copy)
    const void *w_s;           // weights of rational objects, class-sorted (plan copy)
    const int32_t *perm;       // sorted slot -> object
    const Tile *tiles;
    uint32_t n_tiles;          // tiles of the persistent launch
    uint32_t n_signed;         // tiles of signed-weight rationals, after those (a launch of their own)
    const NurbsHead *nhead;    // [n_nurbs], NURBS ranked in sorted order
    const NurbsTab *ntab;      // span lookup tables, 2*nseg+1 entries per NURBS (FP32 storage only)
    const float *brk;          // breakpoints, nseg+1 per NURBS, from NurbsHead::brk0
    const float *seg;          // [n_segs][4][dim+1] homogeneous
    const float *t;
    const float *v;            // second parameters (patches' v), [n_obj][n_t]; read for patches only
    float *out;
    int64_t plane;
    uint32_t n_t;
    FastDiv div_nt;
    int dim;
    unsigned int *counters;    // [0] next tile, [1] finished workgroups
    int dynamic;               // 1: atomic tile counter, 0: static round robin
    int vq;                    // queries per lane: 1, or 4 consecutive parameters of one object
};

namespace batch_dev {

// FP32 value of 16-bit storage bits.
template <typename T>
__device__ __forceinline__ float bits_to_f32(uint16_t b) {
    if constexpr (std::is_same<T, _Float16>::value) return static_cast<float>(__builtin_bit_cast(_Float16, b));
    else return __uint_as_float(static_cast<uint32_t>(b) << 16);  // bf16
}

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
        // 16-bit storage: the row in 16-, 8-, 4- and 2-byte pieces (rows are only
        // 2-byte aligned), each element widened from its bits
        typedef uint16_t u16x8 __attribute__((ext_vector_type(8), aligned(2)));
        typedef uint16_t u16x4 __attribute__((ext_vector_type(4), aligned(2)));
        typedef uint16_t u16x2 __attribute__((ext_vector_type(2), aligned(2)));
        const uint16_t *__restrict__ q = reinterpret_cast<const uint16_t *>(p);
        constexpr int N8 = N / 8 * 8, R = N - N8;
#pragma unroll
        for (int i = 0; i < N8; i += 8) {
            const u16x8 x = *reinterpret_cast<const u16x8 *>(q + i);
#pragma unroll
            for (int e = 0; e < 8; ++e) v[i + e] = bits_to_f32<T>(x[e]);
        }
        constexpr int O4 = N8, O2 = N8 + (R & 4), O1 = O2 + (R & 2);
        if constexpr ((R & 4) != 0) {
            const u16x4 x = *reinterpret_cast<const u16x4 *>(q + O4);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[O4 + e] = bits_to_f32<T>(x[e]);
        }
        if constexpr ((R & 2) != 0) {
            const u16x2 x = *reinterpret_cast<const u16x2 *>(q + O2);
            v[O2] = bits_to_f32<T>(x[0]);
            v[O2 + 1] = bits_to_f32<T>(x[1]);
        }
        if constexpr ((R & 1) != 0) v[O1] = bits_to_f32<T>(q[O1]);
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
        const float rden = RAT ? 1.0f / den : 1.0f;  // one division per query, not per coordinate
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
            if (k < dim) {
                float b[D + 1];
                load_row<T, D + 1>(P + k * (D + 1), b);
                const float v = dot_basis<D>(B, b);
                st_stream(out + k * plane + q, RAT ? v * rden : v);
            }
        }
    } else {
        float rden = 1.0f;
        if constexpr (RAT) rden = 1.0f / eval_dc<D>(wv, t);
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
                st_stream(out + k * plane + q, RAT ? v * rden : v);
            }
        }
    }
}

// Four consecutive queries (one object, parameters t[0..3]) per lane: the
// object's coefficients are loaded once for four evaluations, the parameters
// come in one 16-byte load and each coordinate leaves in one 16-byte store.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

template <int D, bool RAT, int F, typename T>
__device__ __forceinline__ void eval_curve_query4(const T *__restrict__ P, const T *__restrict__ W, int dim,
                                                  const float (&t)[4], float *__restrict__ out, int64_t plane,
                                                  int64_t q) {
    float wv[D + 1];
    if constexpr (RAT) load_row<T, D + 1>(W, wv);
    if constexpr (F == FORM_BERN) {
        float B[4][D + 1], den[4];  // den: reciprocal of the weight sum (rational)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bernstein_basis<D>(t[i], B[i]);
            den[i] = 1.0f;
            if constexpr (RAT) {
#pragma unroll
                for (int e = 0; e <= D; ++e) B[i][e] *= wv[e];
                den[i] = B[i][0];
#pragma unroll
                for (int e = 1; e <= D; ++e) den[i] += B[i][e];
                den[i] = 1.0f / den[i];  // reciprocal: one division per query
            }
        }
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
            if (k < dim) {
                float b[D + 1];
                load_row<T, D + 1>(P + k * (D + 1), b);
                f4u v;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float x = dot_basis<D>(B[i], b);
                    v[i] = RAT ? x * den[i] : x;
                }
                __builtin_nontemporal_store(v, reinterpret_cast<f4u *>(out + k * plane + q));
            }
        }
    } else {
        float den[4] = {1.0f, 1.0f, 1.0f, 1.0f};  // reciprocals of the weight sums
        if constexpr (RAT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) den[i] = 1.0f / eval_dc<D>(wv, t[i]);  // reciprocals
        }
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
            if (k < dim) {
                float b[D + 1];
                load_row<T, D + 1>(P + k * (D + 1), b);
                if constexpr (RAT) {
#pragma unroll
                    for (int e = 0; e <= D; ++e) b[e] *= wv[e];
                }
                f4u v;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float x = eval_dc<D>(b, t[i]);
                    v[i] = RAT ? x * den[i] : x;
                }
                __builtin_nontemporal_store(v, reinterpret_cast<f4u *>(out + k * plane + q));
            }
        }
    }
}

// Rational objects with a weight that is not positive: the denominator
// sum w_i B_i can cancel, so each query gets the conditioning test of
// bz_eval_rational, kappa = sum |w_i| B_i / |sum w_i B_i| computed from the
// FP32 Bernstein basis, and a query with kappa above the threshold (or a zero
// or non-finite weight sum) is evaluated again by FP64 de Casteljau on the
// homogeneous points.  (With all weights positive kappa is 1, so those objects
// form classes of their own that skip the test.)
constexpr float kBatchKappa = 64.0f;

template <int D, typename T>
__device__ __attribute__((noinline)) void batch_rational_fp64(const T *__restrict__ P, const T *__restrict__ W, int dim,
                                                              float t, float *__restrict__ out, int64_t plane,
                                                              int64_t q) {
    const double td = static_cast<double>(t);
    double ww[D + 1], den[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) den[i] = ww[i] = static_cast<double>(to_f32<T>(W[i]));
#pragma unroll
    for (int lvl = 1; lvl <= D; ++lvl)
#pragma unroll
        for (int i = 0; i <= D - lvl; ++i) den[i] = lerp(den[i], den[i + 1], td);
    for (int k = 0; k < dim; ++k) {
        double H[D + 1];
#pragma unroll
        for (int i = 0; i <= D; ++i) H[i] = ww[i] * static_cast<double>(to_f32<T>(P[k * (D + 1) + i]));
#pragma unroll
        for (int lvl = 1; lvl <= D; ++lvl)
#pragma unroll
            for (int i = 0; i <= D - lvl; ++i) H[i] = lerp(H[i], H[i + 1], td);
        st_stream(out + k * plane + q, static_cast<float>(H[0] / den[0]));
    }
}

constexpr int kMaxQpt = 4;

// Index, permutation and parameter loads of every sub-tile are issued before
// any evaluation, so their latencies overlap instead of adding up.  Tail lanes
// re-read the last query of the tile and store nothing.
struct SubTileQueries {
    uint32_t slot[kMaxQpt], j[kMaxQpt];
    int64_t q[kMaxQpt];
    float t[kMaxQpt];
    bool ok[kMaxQpt];
};

__device__ __forceinline__ void prefetch_queries(const BatchArgs &a, const Tile &tl, SubTileQueries &sq) {
    const uint32_t nq = static_cast<uint32_t>(tl.ci.count) * a.n_t;
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        const uint32_t qi = tl.q0 + s * kBlock + threadIdx.x;
        sq.ok[s] = s < static_cast<int>(tl.qpt) && qi < tl.q1;
        const uint32_t qc = min(qi, nq - 1);
        sq.slot[s] = fdiv(qc, a.div_nt);
        sq.j[s] = qc - sq.slot[s] * a.n_t;
    }
    int64_t o[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) o[s] = a.perm[tl.ci.first + sq.slot[s]];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        sq.q[s] = o[s] * a.n_t + sq.j[s];
        sq.t[s] = a.t[sq.q[s]];
    }
}

template <int D, bool RAT, int F, typename T>
__device__ __forceinline__ void run_curve_tile(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    SubTileQueries sq;
    prefetch_queries(a, tl, sq);
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        if (!sq.ok[s]) continue;
        // the control points' address needs no index load: classes are contiguous
        const T *P = static_cast<const T *>(a.ctrl_s) + tl.ci.ctrl_base + static_cast<size_t>(sq.slot[s]) * (D + 1) * a.dim;
        const T *W = RAT ? static_cast<const T *>(a.w_s) + tl.ci.w_base + static_cast<size_t>(sq.slot[s]) * (D + 1)
                         : nullptr;
        eval_curve_query<D, RAT, F, T>(P, W, a.dim, sq.t[s], out, a.plane, sq.q[s]);
    }
}

// One query per lane; the conditioning test decides between the FP32 form
// and the FP64 recomputation per query.
template <int D, int F, typename T>
__device__ __forceinline__ void run_signed_tile(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    SubTileQueries sq;
    prefetch_queries(a, tl, sq);
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        if (!sq.ok[s]) continue;
        const T *P = static_cast<const T *>(a.ctrl_s) + tl.ci.ctrl_base + static_cast<size_t>(sq.slot[s]) * (D + 1) * a.dim;
        const T *W = static_cast<const T *>(a.w_s) + tl.ci.w_base + static_cast<size_t>(sq.slot[s]) * (D + 1);
        const float t = sq.t[s];
        float wv[D + 1], B[D + 1];
        load_row<T, D + 1>(W, wv);
        bernstein_basis<D>(t, B);
        float den = 0.0f, mag = 0.0f;
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            den = __builtin_fmaf(wv[i], B[i], den);
            mag = __builtin_fmaf(__builtin_fabsf(wv[i]), B[i], mag);
        }
        // NaN t: no recomputation, the FP32 form passes the NaN on
        const bool fix = (t == t) && !(den != 0.0f && mag <= kBatchKappa * __builtin_fabsf(den));
        if (fix) batch_rational_fp64<D, T>(P, W, a.dim, t, out, a.plane, sq.q[s]);
        else eval_curve_query<D, true, F, T>(P, W, a.dim, t, out, a.plane, sq.q[s]);
    }
}

// Lane l of sub-tile s takes the four queries starting at q0 + 4(s*256 + l);
// n_t is a multiple of 4, so they belong to one object.
template <int D, bool RAT, int F, typename T>
__device__ __forceinline__ void run_curve_tile4(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    const uint32_t nq = static_cast<uint32_t>(tl.ci.count) * a.n_t;
    uint32_t slot[kMaxQpt];
    int64_t q[kMaxQpt];
    bool ok[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        const uint32_t qi = tl.q0 + 4 * (s * kBlock + threadIdx.x);
        ok[s] = s < static_cast<int>(tl.qpt) && qi < tl.q1;
        const uint32_t qc = min(qi, nq - 4);
        slot[s] = fdiv(qc, a.div_nt);
        q[s] = qc - slot[s] * a.n_t;  // j for now
    }
    int64_t o[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) o[s] = a.perm[tl.ci.first + slot[s]];
    float tv[kMaxQpt][4];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        q[s] += o[s] * a.n_t;
        const f4u x = *reinterpret_cast<const f4u *>(a.t + q[s]);
        tv[s][0] = x[0], tv[s][1] = x[1], tv[s][2] = x[2], tv[s][3] = x[3];
    }
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        if (!ok[s]) continue;
        const T *P = static_cast<const T *>(a.ctrl_s) + tl.ci.ctrl_base + static_cast<size_t>(slot[s]) * (D + 1) * a.dim;
        const T *W = RAT ? static_cast<const T *>(a.w_s) + tl.ci.w_base + static_cast<size_t>(slot[s]) * (D + 1)
                         : nullptr;
        eval_curve_query4<D, RAT, F, T>(P, W, a.dim, tv[s], out, a.plane, q[s]);
    }
}

// NURBS queries, staged across the sub-tiles so that the dependent loads of
// one stage (header and object index; parameter; table entries; breakpoints
// and segment) overlap over all of a lane's queries: clamp u to the NURBS's
// range, find its bucket and segment, and evaluate that segment's rational
// cubic.  Every stage moves its bytes in as few vector loads as it can: the
// address unit serves about one distinct cache line per cycle, and a wave's
// 64 queries spread over many segments.
typedef int32_t i4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

template <int DIM, bool SEARCH>
__device__ __forceinline__ void run_nurbs_tile(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    constexpr int H = DIM + 1;  // homogeneous coordinates; a segment is 4*H floats = H vectors
    const uint32_t nq = static_cast<uint32_t>(tl.ci.count) * a.n_t;
    uint32_t slot[kMaxQpt];
    bool ok[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        const uint32_t qi = tl.q0 + s * kBlock + threadIdx.x;
        ok[s] = s < static_cast<int>(tl.qpt) && qi < tl.q1;
        slot[s] = min(qi, nq - 1);
    }
    NurbsHead h[kMaxQpt];
    int64_t q[kMaxQpt];
    uint32_t j[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        const uint32_t r = fdiv(slot[s], a.div_nt);  // NURBS rank = slot in the class
        j[s] = slot[s] - r * a.n_t;
        slot[s] = r;
        h[s] = a.nhead[r];
    }
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) q[s] = static_cast<int64_t>(a.perm[tl.ci.first + slot[s]]) * a.n_t + j[s];
    // the search's first probe depends only on the header: loaded beside t, it
    // brings the breakpoints' line in while the parameter is on its way
    float u[kMaxQpt];
    [[maybe_unused]] float first[kMaxQpt];
    if constexpr (SEARCH) {
#pragma unroll
        for (int s = 0; s < kMaxQpt; ++s) first[s] = a.brk[h[s].brk0 + (h[s].nseg >> 1)];
    }
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        const float v = a.t[q[s]];
        float c = v < h[s].lo ? h[s].lo : v;  // NaN passes
        u[s] = c > h[s].hi ? h[s].hi : c;
    }
    int32_t sg[kMaxQpt];
    if constexpr (SEARCH) {
        // the last breakpoint <= u among the first nseg, by a binary search on
        // [sg, sg + cnt) stepped for all of a lane's queries together (u is
        // clamped to [lo, hi]; a NaN u stays in segment 0 and gives NaN)
        int32_t cnt[kMaxQpt];
#pragma unroll
        for (int s = 0; s < kMaxQpt; ++s) {
            const int n = h[s].nseg, half = n >> 1;
            const bool up = n > 1 && first[s] <= u[s];
            sg[s] = up ? half : 0;
            cnt[s] = n > 1 ? (up ? n - half : half) : n;
        }
        bool more = true;
        while (more) {
            more = false;
#pragma unroll
            for (int s = 0; s < kMaxQpt; ++s) {
                if (cnt[s] > 1) {
                    const int half = cnt[s] >> 1;
                    if (a.brk[h[s].brk0 + sg[s] + half] <= u[s]) {
                        sg[s] += half;
                        cnt[s] -= half;
                    } else {
                        cnt[s] = half;
                    }
                    more = more || cnt[s] > 1;
                }
            }
        }
    } else {
        i4u e[kMaxQpt];  // table entries m and m+1: {s, split bits, s, split bits}
#pragma unroll
        for (int s = 0; s < kMaxQpt; ++s) {
            const int m = nurbs_bucket(u[s], h[s].lo, h[s].inv_h, 2 * h[s].nseg);
            e[s] = *reinterpret_cast<const i4u *>(a.ntab + h[s].tab0 + m);
        }
#pragma unroll
        for (int s = 0; s < kMaxQpt; ++s) {
            int lo = e[s][0], hi = e[s][2];
            if (hi - lo <= 1) {
                sg[s] = (hi > lo && __int_as_float(e[s][1]) <= u[s]) ? hi : lo;
            } else {  // two or more breakpoints inside the bucket
                const float *b = a.brk + h[s].brk0;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (b[mid] <= u[s]) lo = mid;
                    else hi = mid - 1;
                }
                sg[s] = lo;
            }
        }
    }
    f2u br[kMaxQpt];
    float S[kMaxQpt][4 * H];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        br[s] = *reinterpret_cast<const f2u *>(a.brk + h[s].brk0 + sg[s]);
        const float *__restrict__ p = a.seg + static_cast<size_t>(h[s].s0 + sg[s]) * 4 * H;
#pragma unroll
        for (int v = 0; v < H; ++v) {
            const f4u x = *reinterpret_cast<const f4u *>(p + 4 * v);
            S[s][4 * v] = x[0], S[s][4 * v + 1] = x[1], S[s][4 * v + 2] = x[2], S[s][4 * v + 3] = x[3];
        }
    }
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        if (!ok[s]) continue;
        const float tseg = (u[s] - br[s][0]) / (br[s][1] - br[s][0]);
        float B[4];
        bernstein_basis<3>(tseg, B);
        float acc[H] = {};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < H; ++k) acc[k] = __builtin_fmaf(B[i], S[s][i * H + k], acc[k]);
        const float rw = 1.0f / acc[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) st_stream(out + k * a.plane + q[s], acc[k] * rw);
    }
}

template <bool SEARCH>
__device__ __forceinline__ void run_nurbs_tile_dim(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    switch (a.dim) {
        case 1: run_nurbs_tile<1, SEARCH>(a, tl, out); break;
        case 2: run_nurbs_tile<2, SEARCH>(a, tl, out); break;
        case 3: run_nurbs_tile<3, SEARCH>(a, tl, out); break;
        default: run_nurbs_tile<4, SEARCH>(a, tl, out); break;
    }
}

// Tensor-product surface patches (Sec. 2.2: the surface is the tensor product
// of two curve bases): control points [dim][(DU+1)(DV+1)], index i*(DV+1)+j
// (u major).  Bernstein form: both bases, then the double sum; de Casteljau
// form: each u-row reduced in v, then the column in u.
template <int DU, int DV, int F>
__device__ __forceinline__ float patch_value(const float (&P)[(DU + 1) * (DV + 1)], const float (&Bu)[DU + 1],
                                             const float (&Bv)[DV + 1], float u, float v) {
    float col[DU + 1];
#pragma unroll
    for (int i = 0; i <= DU; ++i) {
        float row[DV + 1];
#pragma unroll
        for (int j = 0; j <= DV; ++j) row[j] = P[i * (DV + 1) + j];
        col[i] = F == FORM_BERN ? dot_basis<DV>(Bv, row) : eval_dc<DV>(row, v);
    }
    return F == FORM_BERN ? dot_basis<DU>(Bu, col) : eval_dc<DU>(col, u);
}

// VQ consecutive queries of one patch per lane (VQ = 4 needs n_t % 4 == 0):
// the patch's net is loaded once for them, u and v come in VQ-wide loads and
// each coordinate leaves in one VQ-wide store.
template <int DU, int DV, int F, typename T, int VQ>
__device__ __forceinline__ void run_patch_tile(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    constexpr int NCP = (DU + 1) * (DV + 1);
    const uint32_t nq = static_cast<uint32_t>(tl.ci.count) * a.n_t;
    uint32_t slot[kMaxQpt];
    int64_t q[kMaxQpt];
    bool ok[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        const uint32_t qi = tl.q0 + VQ * (s * kBlock + threadIdx.x);
        ok[s] = s < static_cast<int>(tl.qpt) && qi < tl.q1;
        const uint32_t qc = min(qi, nq - VQ);
        slot[s] = fdiv(qc, a.div_nt);
        q[s] = qc - slot[s] * a.n_t;  // j for now
    }
    int64_t o[kMaxQpt];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) o[s] = a.perm[tl.ci.first + slot[s]];
    float uu[kMaxQpt][VQ], vv[kMaxQpt][VQ];
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        q[s] += o[s] * a.n_t;
        if constexpr (VQ == 4) {
            const f4u x = *reinterpret_cast<const f4u *>(a.t + q[s]);
            const f4u y = *reinterpret_cast<const f4u *>(a.v + q[s]);
#pragma unroll
            for (int e = 0; e < 4; ++e) uu[s][e] = x[e], vv[s][e] = y[e];
        } else {
            uu[s][0] = a.t[q[s]];
            vv[s][0] = a.v[q[s]];
        }
    }
#pragma unroll
    for (int s = 0; s < kMaxQpt; ++s) {
        if (!ok[s]) continue;
        const T *P = static_cast<const T *>(a.ctrl_s) + tl.ci.ctrl_base + static_cast<size_t>(slot[s]) * NCP * a.dim;
        float Bu[VQ][DU + 1], Bv[VQ][DV + 1];
        if constexpr (F == FORM_BERN) {
#pragma unroll
            for (int e = 0; e < VQ; ++e) {
                bernstein_basis<DU>(uu[s][e], Bu[e]);
                bernstein_basis<DV>(vv[s][e], Bv[e]);
            }
        }
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
            if (k < a.dim) {
                float p[NCP];
                load_row<T, NCP>(P + k * NCP, p);
                if constexpr (VQ == 4) {
                    f4u r;
#pragma unroll
                    for (int e = 0; e < 4; ++e) r[e] = patch_value<DU, DV, F>(p, Bu[e], Bv[e], uu[s][e], vv[s][e]);
                    __builtin_nontemporal_store(r, reinterpret_cast<f4u *>(out + k * a.plane + q[s]));
                } else {
                    st_stream(out + k * a.plane + q[s], patch_value<DU, DV, F>(p, Bu[0], Bv[0], uu[s][0], vv[s][0]));
                }
            }
        }
    }
}

template <int F, typename T, int VQ>
__device__ __forceinline__ void dispatch_patch(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    switch (tl.ci.degree) {
        case 0x11: run_patch_tile<1, 1, F, T, VQ>(a, tl, out); break;
        case 0x12: run_patch_tile<1, 2, F, T, VQ>(a, tl, out); break;
        case 0x13: run_patch_tile<1, 3, F, T, VQ>(a, tl, out); break;
        case 0x21: run_patch_tile<2, 1, F, T, VQ>(a, tl, out); break;
        case 0x22: run_patch_tile<2, 2, F, T, VQ>(a, tl, out); break;
        case 0x23: run_patch_tile<2, 3, F, T, VQ>(a, tl, out); break;
        case 0x31: run_patch_tile<3, 1, F, T, VQ>(a, tl, out); break;
        case 0x32: run_patch_tile<3, 2, F, T, VQ>(a, tl, out); break;
        default: run_patch_tile<3, 3, F, T, VQ>(a, tl, out); break;
    }
}

template <int D, bool RAT, int F, typename T, int VQ>
__device__ __forceinline__ void run_curve_tile_vq(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    if constexpr (VQ == 4) run_curve_tile4<D, RAT, F, T>(a, tl, out);
    else run_curve_tile<D, RAT, F, T>(a, tl, out);
}

template <bool RAT, int F, typename T, int VQ>
__device__ __forceinline__ void dispatch_degree(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    switch (tl.ci.degree) {
        case 1: run_curve_tile_vq<1, RAT, F, T, VQ>(a, tl, out); break;
        case 2: run_curve_tile_vq<2, RAT, F, T, VQ>(a, tl, out); break;
        case 3: run_curve_tile_vq<3, RAT, F, T, VQ>(a, tl, out); break;
        case 4: run_curve_tile_vq<4, RAT, F, T, VQ>(a, tl, out); break;
        case 5: run_curve_tile_vq<5, RAT, F, T, VQ>(a, tl, out); break;
        case 6: run_curve_tile_vq<6, RAT, F, T, VQ>(a, tl, out); break;
        case 7: run_curve_tile_vq<7, RAT, F, T, VQ>(a, tl, out); break;
        case 8: run_curve_tile_vq<8, RAT, F, T, VQ>(a, tl, out); break;
        case 9: run_curve_tile_vq<9, RAT, F, T, VQ>(a, tl, out); break;
        case 10: run_curve_tile_vq<10, RAT, F, T, VQ>(a, tl, out); break;
        case 11: run_curve_tile_vq<11, RAT, F, T, VQ>(a, tl, out); break;
        case 12: run_curve_tile_vq<12, RAT, F, T, VQ>(a, tl, out); break;
        case 13: run_curve_tile_vq<13, RAT, F, T, VQ>(a, tl, out); break;
        case 14: run_curve_tile_vq<14, RAT, F, T, VQ>(a, tl, out); break;
        default: run_curve_tile_vq<15, RAT, F, T, VQ>(a, tl, out); break;
    }
}

template <int F, typename T>
__device__ __forceinline__ void dispatch_degree_signed(const BatchArgs &a, const Tile &tl, float *__restrict__ out) {
    switch (tl.ci.degree) {
        case 1: run_signed_tile<1, F, T>(a, tl, out); break;
        case 2: run_signed_tile<2, F, T>(a, tl, out); break;
        case 3: run_signed_tile<3, F, T>(a, tl, out); break;
        case 4: run_signed_tile<4, F, T>(a, tl, out); break;
        case 5: run_signed_tile<5, F, T>(a, tl, out); break;
        case 6: run_signed_tile<6, F, T>(a, tl, out); break;
        case 7: run_signed_tile<7, F, T>(a, tl, out); break;
        case 8: run_signed_tile<8, F, T>(a, tl, out); break;
        case 9: run_signed_tile<9, F, T>(a, tl, out); break;
        case 10: run_signed_tile<10, F, T>(a, tl, out); break;
        case 11: run_signed_tile<11, F, T>(a, tl, out); break;
        case 12: run_signed_tile<12, F, T>(a, tl, out); break;
        case 13: run_signed_tile<13, F, T>(a, tl, out); break;
        case 14: run_signed_tile<14, F, T>(a, tl, out); break;
        default: run_signed_tile<15, F, T>(a, tl, out); break;
    }
}

template <int F, typename T, int VQ>
__device__ __forceinline__ void run_tile(const BatchArgs &a, unsigned int tile, float *__restrict__ out) {
    const Tile tl = a.tiles[tile];
    if (tl.ci.kind == 0) dispatch_degree<false, F, T, VQ>(a, tl, out);
    else if (tl.ci.kind == 1) dispatch_degree<true, F, T, VQ>(a, tl, out);
    else if (tl.ci.kind == 4) dispatch_patch<F, T, VQ>(a, tl, out);
    else run_nurbs_tile_dim<!std::is_same<T, float>::value>(a, tl, out);
}

// Dynamic schedule: workgroups pull tiles from an atomic counter (the next
// index is fetched while the current tile is evaluated).  Static schedule:
// workgroup g takes tiles g, g+G, g+2G, ... -- balanced because tiles are
// ordered by cost and every tile of a class costs the same.
// FP32 storage with four queries per lane runs at four waves per SIMD (the
// register budget then spills a few dwords on the degree-15 path; measured
// faster than three waves without spills); FP16/BF16 storage is faster at the
// compiler's own choice.
template <int F, typename T, int VQ>
// out is also a parameter of its own, declared not to alias anything else the
// kernel reads, so a lane's loads for its next coordinate or sub-tile need not
// wait behind its stores.
__global__ __launch_bounds__(kBlock, (VQ == 4 && std::is_same<T, float>::value) ? 4 : 1) void k_batch_persistent(
    BatchArgs a, float *__restrict__ out) {
    if (!a.dynamic) {
        for (unsigned int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) run_tile<F, T, VQ>(a, tile, out);
        return;
    }
    __shared__ unsigned int s_tile;
    if (threadIdx.x == 0) s_tile = atomicAdd(&a.counters[0], 1u);
    __syncthreads();
    unsigned int tile = s_tile;
    __syncthreads();
    while (tile < a.n_tiles) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&a.counters[0], 1u);
        run_tile<F, T, VQ>(a, tile, out);
        __syncthreads();
        tile = s_tile;
        __syncthreads();
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

// The signed-weight rational tiles run in a launch of their own, one
// workgroup per tile: their FP64 recomputation needs far more registers than
// any path of the persistent kernel, whose occupancy would otherwise drop for
// every batch.
template <int F, typename T>
__global__ __launch_bounds__(kBlock) void k_batch_signed(BatchArgs a, float *__restrict__ out) {
    const Tile tl = a.tiles[a.n_tiles + blockIdx.x];
    dispatch_degree_signed<F, T>(a, tl, out);
}

}  // namespace batch_dev

// Launch of the persistent kernel (instantiated in batched_{dc,bern}_{f32,f16,bf16}.hip),
// then the signed-weight rationals' own launch.
template <int F, typename T>
int launch_batch_kernel(uint32_t workgroups, const BatchArgs &a, hipStream_t s) {
    if (a.vq == 4)
        hipLaunchKernelGGL((batch_dev::k_batch_persistent<F, T, 4>), dim3(workgroups), dim3(kBlock), 0, s, a, a.out);
    else
        hipLaunchKernelGGL((batch_dev::k_batch_persistent<F, T, 1>), dim3(workgroups), dim3(kBlock), 0, s, a, a.out);
    BZ_CHECK_LAUNCH("k_batch_persistent");
    if (a.n_signed > 0) {
        hipLaunchKernelGGL((batch_dev::k_batch_signed<F, T>), dim3(a.n_signed), dim3(kBlock), 0, s, a, a.out);
        BZ_CHECK_LAUNCH("k_batch_signed");
    }
    return BZ_OK;
}


#define BZI_BATCH_EXTERN(F, T) extern template int launch_batch_kernel<F, T>(uint32_t, const BatchArgs &, hipStream_t);
BZI_BATCH_EXTERN(FORM_DC, float)
BZI_BATCH_EXTERN(FORM_BERN, float)
BZI_BATCH_EXTERN(FORM_DC, _Float16)
BZI_BATCH_EXTERN(FORM_BERN, _Float16)
BZI_BATCH_EXTERN(FORM_DC, bf16_t)
BZI_BATCH_EXTERN(FORM_BERN, bf16_t)
#undef BZI_BATCH_EXTERN

}  // namespace bzi
