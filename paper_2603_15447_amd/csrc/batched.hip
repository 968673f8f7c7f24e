// Mixed batches (integral / rational Bezier curves of degree 1..15 and cubic
// NURBS) evaluated by one persistent launch on gfx950.
//
// Plan (host, once): objects are sorted into uniform classes (kind, degree)
// so that every 256-query tile, and hence every wavefront, runs one code path;
// NURBS are cut into rational Bezier segments by knot insertion on the GPU
// (Sec. 2.2: B-splines become piecewise Bezier curves via Boehm's algorithm)
// with the breakpoints kept for a per-query span search; tiles are ordered by
// estimated cost, heaviest first.
// Evaluation (batched_impl.h): a grid of (CUs x occupancy) workgroups takes
// tiles round-robin or from an atomic counter; the last workgroup to finish
// resets the counters, so consecutive launches (and graph replays) need no
// memset.  (The 16 lanes that evaluate one object load the same addresses,
// which the memory pipeline merges into one access; sharing the coefficients
// by DPP row broadcasts instead was measured slower.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "batched_impl.h"

struct bz_plan_s;

namespace bzi {
namespace {

// Plan-time gather of control points (and weights of rational objects) into
// class-sorted, contiguous order: sorted object i of class c lands at
// ctrl_base(c) + slot*(d+1)*dim.  One thread per sorted object.
template <typename U>
__global__ __launch_bounds__(kBlock) void k_gather_sorted(int64_t n_sorted, const int32_t *__restrict__ perm,
                                                          const int64_t *__restrict__ cp_offset,
                                                          const ClassInfo *__restrict__ classes, int n_classes, int dim,
                                                          const U *__restrict__ ctrl, const U *__restrict__ w,
                                                          U *__restrict__ ctrl_s, U *__restrict__ w_s) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_sorted) return;
    int c = 0;
    while (c + 1 < n_classes && classes[c + 1].first <= i) ++c;
    const ClassInfo ci = classes[c];
    if (ci.kind == 2) return;
    const int64_t slot = i - ci.first, o = perm[i];
    const int n = class_ncp(ci.kind, ci.degree) * dim;
    const U *src = ctrl + cp_offset[o] * dim;
    U *dst = ctrl_s + ci.ctrl_base + slot * n;
    for (int e = 0; e < n; ++e) dst[e] = src[e];
    if (ci.kind == 1 || ci.kind == 3)
        for (int e = 0; e <= ci.degree; ++e) w_s[ci.w_base + slot * (ci.degree + 1) + e] = w[cp_offset[o] + e];
}

// Plan-time weight check: flags[o] = 1 when a rational or NURBS object has a
// weight that is not positive (zero, negative or NaN).  One thread per object.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_weight_flags(int64_t n_obj, const uint16_t *__restrict__ kind_degree,
                                                         const int64_t *__restrict__ cp_offset, const T *__restrict__ w,
                                                         uint8_t *__restrict__ flags) {
    const int64_t o = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (o >= n_obj) return;
    uint8_t f = 0;
    const int kind = kind_degree[o] >> 8;
    if (kind == 1 || kind == 2)
        for (int64_t i = cp_offset[o]; i < cp_offset[o + 1]; ++i) f |= !(to_f32<T>(w[i]) > 0.0f);
    flags[o] = f;
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

// Span lookup tables of the NURBS (see NurbsHead): for bucket m, the first
// segment whose end breakpoint lies in bucket m or later; a parameter of
// bucket m then lies in segments tab[m].s .. tab[m+1].s, because the bucket
// function is monotone.  Returns false if an entry is out of range (which the
// construction excludes; checked before anything reaches the device).
// with_table false: the headers alone (16-bit plans search the breakpoints).
bool build_nurbs_tables(const std::vector<int32_t> &seg_first, const std::vector<float> &brk,
                        std::vector<NurbsHead> &head, std::vector<NurbsTab> &tab, bool with_table) {
    const size_t n = seg_first.size() - 1;
    head.resize(n);
    tab.clear();
    tab.reserve(2 * static_cast<size_t>(seg_first.back()) + n);
    std::vector<int> bk;
    for (size_t r = 0; r < n; ++r) {
        NurbsHead h{};
        h.s0 = seg_first[r];
        h.nseg = seg_first[r + 1] - seg_first[r];
        h.brk0 = h.s0 + static_cast<int32_t>(r);
        h.tab0 = static_cast<int32_t>(tab.size());
        const float *b = brk.data() + h.brk0;
        h.lo = b[0];
        h.hi = b[h.nseg];
        const int M = 2 * h.nseg;
        h.inv_h = static_cast<float>(M) / (h.hi - h.lo);
        if (!std::isfinite(h.inv_h)) h.inv_h = 0.0f;  // one bucket holds every segment
        if (!with_table) {
            head[r] = h;
            continue;
        }
        bk.resize(h.nseg + 1);
        for (int i = 0; i <= h.nseg; ++i) bk[i] = nurbs_bucket(b[i], h.lo, h.inv_h, M);
        int i = 0;
        for (int m = 0; m <= M; ++m) {
            while (i < h.nseg - 1 && bk[i + 1] < m) ++i;
            tab.push_back(NurbsTab{i, b[i + 1]});
        }
        for (int m = 0; m <= M; ++m) {
            const int32_t v = tab[h.tab0 + m].s;
            if (v < 0 || v >= h.nseg || (m > 0 && v < tab[h.tab0 + m - 1].s)) return false;
        }
        head[r] = h;
    }
    return true;
}

// Objects per window of the default tile order (see build_tiles).
constexpr uint32_t kDefaultWindow = 131072;

int class_cost(int kind, int degree, int method, int dim) {
    const int ch = dim + (kind != 0 ? 1 : 0);
    if (kind == 2) return 60 + 4 * ch;
    if (kind == 4) {
        const int du = degree >> 4, dv = degree & 15, ncp = (du + 1) * (dv + 1);
        if (method == BZ_DECASTELJAU) return ((du + 1) * dv * (dv + 1) / 2 + du * (du + 1) / 2) * 2 * dim + 8;
        return 3 * (du + dv) + ncp * dim + 8;
    }
    if (kind == 3) return 4 * degree + (degree + 1) * (ch + 2) + 8 + (method == BZ_DECASTELJAU ? degree * (degree + 1) / 2 * ch * 2 : 0);
    if (method == BZ_DECASTELJAU) return degree * (degree + 1) / 2 * ch * 2 + 8;
    return 3 * degree + (degree + 1) * ch + 8;
}

}  // namespace
}  // namespace bzi

using namespace bzi;

struct bz_plan_s {
    int64_t n_obj = 0, n_t = 0;
    int dim = 0, dtype = 0, method = 0;
    // device buffers owned by the plan
    void *ctrl_s = nullptr, *w_s = nullptr;
    int32_t *perm = nullptr;
    Tile *tiles = nullptr;
    int32_t *seg_first = nullptr;
    NurbsHead *nhead = nullptr;
    NurbsTab *ntab = nullptr;
    float *brk = nullptr, *seg = nullptr;
    unsigned int *counters = nullptr;
    std::vector<ClassInfo> classes;
    std::vector<int32_t> perm_h;  // host copy of perm (window boundaries of the tile order)
    uint32_t n_tiles = 0, n_signed = 0, qpt = 1, vq = 1, window = 0;
    bool has_patches = false;
    int64_t n_segs = 0;
    uint32_t workgroups = 0, cus = 1;
    int dynamic = 1;
};

namespace {

void plan_free(bz_plan_s *p) {
    if (!p) return;
    void *bufs[] = {p->ctrl_s, p->w_s, p->perm, p->tiles, p->seg_first, p->nhead, p->ntab, p->brk, p->seg,
                    p->counters};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

// Device copy of a host vector; waits for the copy, so the vector may be
// freed when this returns (plan-time only).
template <typename X>
int dev_upload(X **dst, const std::vector<X> &src, hipStream_t s) {
    const size_t n = std::max<size_t>(src.size(), 1) * sizeof(X);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), n);
    if (e == hipErrorOutOfMemory) return fail(BZ_ERR_NOMEM, "bz_batch_plan_create: device allocation");
    BZ_CHECK_HIP(e);
    if (!src.empty()) {
        BZ_CHECK_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(X), hipMemcpyHostToDevice, s));
        BZ_CHECK_HIP(hipStreamSynchronize(s));
    }
    return BZ_OK;
}

int launch_batch(const bz_plan_s *p, const float *t, const float *v, float *out, hipStream_t s, uint32_t workgroups,
                 int dynamic, uint32_t vq) {
    BatchArgs a;
    a.vq = static_cast<int>(vq);
    a.dynamic = dynamic;
    a.ctrl_s = p->ctrl_s;
    a.w_s = p->w_s;
    a.perm = p->perm;
    a.tiles = p->tiles;
    a.n_tiles = p->n_tiles;
    a.n_signed = p->n_signed;
    a.nhead = p->nhead;
    a.ntab = p->ntab;
    a.brk = p->brk;
    a.seg = p->seg;
    a.t = t;
    a.v = v;
    a.out = out;
    a.plane = p->n_obj * p->n_t;
    a.n_t = static_cast<uint32_t>(p->n_t);
    a.div_nt = make_fastdiv(a.n_t);
    a.dim = p->dim;
    a.counters = p->counters;
    const bool dc = p->method == BZ_DECASTELJAU;
    if (p->dtype == BZ_F32)
        return dc ? launch_batch_kernel<FORM_DC, float>(workgroups, a, s)
                  : launch_batch_kernel<FORM_BERN, float>(workgroups, a, s);
    if (p->dtype == BZ_F16)
        return dc ? launch_batch_kernel<FORM_DC, _Float16>(workgroups, a, s)
                  : launch_batch_kernel<FORM_BERN, _Float16>(workgroups, a, s);
    return dc ? launch_batch_kernel<FORM_DC, bf16_t>(workgroups, a, s)
              : launch_batch_kernel<FORM_BERN, bf16_t>(workgroups, a, s);
}

// Rebuild the tile list for `qpt` sub-tiles of 256 lanes x `vq` queries per
// tile (NURBS tiles one query per lane).  window = 0: class-major order,
// heaviest class first.  window = W: window-major order over consecutive
// blocks of W objects (in the caller's order), and within a window every
// class, heaviest first, for that window's objects -- so the points and
// parameter rows of neighbouring objects, which share cache lines, are
// written and read close together in time.
int build_tiles(bz_plan_s *p, uint32_t qpt, uint32_t vq, uint32_t window, hipStream_t s) {
    const std::vector<ClassInfo> &cls = p->classes;
    std::vector<int> order(cls.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return class_cost(cls[x].kind, cls[x].degree, p->method, p->dim) >
               class_cost(cls[y].kind, cls[y].degree, p->method, p->dim);
    });
    std::vector<Tile> tiles;
    auto emit = [&](int c, uint64_t a, uint64_t b) {  // queries [a, b) of class c
        const uint64_t span =
            static_cast<uint64_t>(kBlock) * qpt * (cls[c].kind == 0 || cls[c].kind == 1 || cls[c].kind == 4 ? vq : 1);
        for (uint64_t q0 = a; q0 < b; q0 += span)
            tiles.push_back(Tile{cls[c], static_cast<uint32_t>(q0), static_cast<uint32_t>(b), qpt, 0});
    };
    const uint64_t nt = static_cast<uint64_t>(p->n_t);
    // signed-weight rational classes (kind 3) go to a launch of their own:
    // their tiles are appended after all others, in class order
    std::vector<int> signed_cls;
    for (int c : order)
        if (cls[c].kind == 3) signed_cls.push_back(c);
    order.erase(std::remove_if(order.begin(), order.end(), [&](int c) { return cls[c].kind == 3; }), order.end());
    if (window == 0) {
        for (int c : order) emit(c, 0, static_cast<uint64_t>(cls[c].count) * nt);
    } else {
        // a class's slots hold its objects in increasing caller order, so the
        // objects of window w are one run of slots per class
        std::vector<int64_t> cur(cls.size(), 0);
        for (int64_t w0 = 0; w0 < p->n_obj; w0 += window) {
            const int32_t w1 = static_cast<int32_t>(std::min<int64_t>(p->n_obj, w0 + window));
            for (int c : order) {
                const int32_t *first = p->perm_h.data() + cls[c].first;
                const int64_t a = cur[c];
                const int64_t b = std::lower_bound(first + a, first + cls[c].count, w1) - first;
                if (b > a) emit(c, static_cast<uint64_t>(a) * nt, static_cast<uint64_t>(b) * nt);
                cur[c] = b;
            }
        }
    }
    // FP32 plans: NURBS tiles (a chain of dependent random loads per query,
    // cold in steady state) spread evenly through the others instead of one
    // run per window or class, so every stretch of the launch overlaps a few
    // of them with the streaming Bezier tiles (measured faster for FP32
    // storage, whose NURBS queries go through the bucket table, and no
    // faster for 16-bit storage)
    if (p->dtype == BZ_F32) {
        std::vector<Tile> nb, rest;
        for (const Tile &t : tiles) (t.ci.kind == 2 ? nb : rest).push_back(t);
        if (!nb.empty() && !rest.empty()) {
            tiles.clear();
            const uint64_t R = rest.size(), N = nb.size();
            size_t k = 0;
            for (uint64_t i = 0; i < R; ++i) {  // NURBS tile k goes before other tile floor(k*R/N)
                for (; k < N && k * R / N <= i; ++k) tiles.push_back(nb[k]);
                tiles.push_back(rest[i]);
            }
            for (; k < N; ++k) tiles.push_back(nb[k]);
        }
    }
    const size_t n_main = tiles.size();
    for (int c : signed_cls) emit(c, 0, static_cast<uint64_t>(cls[c].count) * nt);
    if (p->tiles) BZ_CHECK_HIP(hipStreamSynchronize(s));
    if (p->tiles) BZ_CHECK_HIP(hipFree(p->tiles));
    p->tiles = nullptr;
    int rc = dev_upload(&p->tiles, tiles, s);
    if (rc) return rc;
    p->n_tiles = static_cast<uint32_t>(n_main);
    p->n_signed = static_cast<uint32_t>(tiles.size() - n_main);
    p->qpt = qpt;
    p->vq = vq;
    p->window = window;
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
        if (method == BZ_AUTO) method = BZ_BERNSTEIN;
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
        // validate the objects
        bool need_w = false, any_nurbs = false;
        for (int64_t o = 0; o < n_obj; ++o) {
            const int kind = kd[o] >> 8, deg = kd[o] & 0xff;
            const int64_t ncp = cpo[o + 1] - cpo[o];
            if (kind > 3) return fail(BZ_ERR_SHAPE, "%s: object %lld has kind %d", fn, (long long)o, kind);
            if (kind == 3) {
                const int du = deg >> 4, dv = deg & 15;
                if (du < 1 || du > 3 || dv < 1 || dv > 3)
                    return fail(BZ_ERR_UNSUPPORTED, "%s: patch object %lld has degree (%d, %d) (1..3 each)", fn, (long long)o, du, dv);
                if (ncp != (du + 1) * (dv + 1))
                    return fail(BZ_ERR_SHAPE, "%s: patch object %lld has %lld control points for degree (%d, %d)", fn, (long long)o, (long long)ncp, du, dv);
            } else if (kind == 2) {
                if (deg != kNurbsP) return fail(BZ_ERR_UNSUPPORTED, "%s: NURBS object %lld has degree %d (only cubic)", fn, (long long)o, deg);
                if (ncp < 4) return fail(BZ_ERR_SHAPE, "%s: NURBS object %lld has %lld control points", fn, (long long)o, (long long)ncp);
                any_nurbs = true;
            } else {
                if (deg < 1 || deg > kMaxDegree) return fail(BZ_ERR_SHAPE, "%s: object %lld degree %d", fn, (long long)o, deg);
                if (ncp != deg + 1) return fail(BZ_ERR_SHAPE, "%s: object %lld has %lld control points for degree %d", fn, (long long)o, (long long)ncp, deg);
            }
            if (kind == 1 || kind == 2) need_w = true;
        }
        if (need_w && !w) return fail(BZ_ERR_NULL, "%s: weights are required (rational or NURBS objects)", fn);
        if (!aligned(ctrl, dtype_size(dtype)) || !aligned(w, dtype_size(dtype)))
            return fail(BZ_ERR_ALIGN, "%s: misaligned ctrl or w", fn);
        // which weighted objects have a weight that is not positive
        std::vector<uint8_t> wflag(n_obj, 0);
        if (need_w) {
            uint8_t *flags_d = nullptr;
            hipError_t e = hipMalloc(reinterpret_cast<void **>(&flags_d), std::max<int64_t>(n_obj, 1));
            if (e == hipErrorOutOfMemory) return fail(BZ_ERR_NOMEM, "%s: device allocation", fn);
            BZ_CHECK_HIP(e);
            const uint32_t blocks = static_cast<uint32_t>((n_obj + kBlock - 1) / kBlock);
            if (dtype == BZ_F32)
                hipLaunchKernelGGL((k_weight_flags<float>), dim3(blocks), dim3(kBlock), 0, s, n_obj, kind_degree,
                                   cp_offset, static_cast<const float *>(w), flags_d);
            else if (dtype == BZ_F16)
                hipLaunchKernelGGL((k_weight_flags<_Float16>), dim3(blocks), dim3(kBlock), 0, s, n_obj, kind_degree,
                                   cp_offset, static_cast<const _Float16 *>(w), flags_d);
            else
                hipLaunchKernelGGL((k_weight_flags<bf16_t>), dim3(blocks), dim3(kBlock), 0, s, n_obj, kind_degree,
                                   cp_offset, static_cast<const bf16_t *>(w), flags_d);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(wflag.data(), flags_d, n_obj, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            (void)hipFree(flags_d);
            if (e != hipSuccess) return hip_fail(e, "k_weight_flags");
        }
        // classes, keyed: 0..14 integral Bezier of degree 1..15, 15..29
        // rational with positive weights, 30..44 rational with a weight <= 0
        // (conditioning test), 45..53 patches of degree (du, dv) in 1..3, 54
        // cubic NURBS (last, so the NURBS rank is its slot in the last class)
        constexpr int kKeys = 55, kPatchKey = 45, kNurbsKey = 54;
        auto key_of = [&](int64_t o) {
            const int kind = kd[o] >> 8, deg = kd[o] & 0xff;
            if (kind == 2) return kNurbsKey;
            if (kind == 3) return kPatchKey + ((deg >> 4) - 1) * 3 + (deg & 15) - 1;
            if (kind == 1 && wflag[o]) return 30 + deg - 1;
            return kind * 15 + deg - 1;
        };
        std::vector<int64_t> count(kKeys, 0);
        for (int64_t o = 0; o < n_obj; ++o) {
            if ((kd[o] >> 8) == 2 && wflag[o])
                return fail(BZ_ERR_UNSUPPORTED, "%s: NURBS object %lld has a weight that is not positive", fn, (long long)o);
            count[key_of(o)] += 1;
        }
        // class list and permutation (stable counting sort by key)
        std::vector<ClassInfo> cls;
        std::vector<int32_t> cls_of_key(kKeys, -1);
        int32_t first = 0;
        int64_t ctrl_elems = 0, w_elems = 0;
        for (int key = 0; key < kKeys; ++key) {
            if (count[key] == 0) continue;
            ClassInfo ci;
            if (key == kNurbsKey) {
                ci.kind = 2;
                ci.degree = kNurbsP;
            } else if (key >= kPatchKey) {
                ci.kind = 4;
                ci.degree = ((key - kPatchKey) / 3 + 1) << 4 | ((key - kPatchKey) % 3 + 1);
            } else {
                ci.kind = key / 15 == 2 ? 3 : key / 15;
                ci.degree = key % 15 + 1;
            }
            ci.first = first;
            ci.count = static_cast<int32_t>(count[key]);
            ci.ctrl_base = ctrl_elems;
            ci.w_base = w_elems;
            if (ci.kind != 2) ctrl_elems += count[key] * class_ncp(ci.kind, ci.degree) * dim;
            if (ci.kind == 1 || ci.kind == 3) w_elems += count[key] * (ci.degree + 1);
            cls_of_key[key] = static_cast<int32_t>(cls.size());
            cls.push_back(ci);
            first += ci.count;
        }
        std::vector<int32_t> perm(n_obj), fill(cls.size(), 0);
        for (int64_t o = 0; o < n_obj; ++o) {
            const int c = cls_of_key[key_of(o)];
            perm[cls[c].first + fill[c]++] = static_cast<int32_t>(o);
        }
        // NURBS (in sorted order, so a NURBS's rank is its slot in the class):
        // read and validate the knot vectors, count segments, keep breakpoints
        std::vector<int64_t> nurbs_obj;
        std::vector<int32_t> seg_first(1, 0);
        std::vector<float> brk;
        if (any_nurbs) {
            if (!knot_offset || !knots) return fail(BZ_ERR_NULL, "%s: knot_offset and knots are required for NURBS", fn);
            ko.resize(n_obj + 1);
            BZ_CHECK_HIP(hipMemcpyAsync(ko.data(), knot_offset, (n_obj + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            BZ_CHECK_HIP(hipStreamSynchronize(s));
            const int64_t nk_total = ko[n_obj];
            if (nk_total < 0 || nk_total > (int64_t(1) << 34)) return fail(BZ_ERR_SHAPE, "%s: knot_offset", fn);
            std::vector<float> U(nk_total);
            BZ_CHECK_HIP(hipMemcpyAsync(U.data(), knots, nk_total * sizeof(float), hipMemcpyDeviceToHost, s));
            BZ_CHECK_HIP(hipStreamSynchronize(s));
            const ClassInfo &nc = cls.back();
            for (int32_t r = 0; r < nc.count; ++r) {
                const int64_t o = perm[nc.first + r];
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
        bz_plan_s *p = new (std::nothrow) bz_plan_s();
        if (!p) return fail(BZ_ERR_NOMEM, "%s: host allocation", fn);
        p->n_obj = n_obj;
        p->n_t = n_t;
        p->dim = dim;
        p->dtype = dtype;
        p->method = method;
        p->classes = cls;
        for (const ClassInfo &ci : cls) p->has_patches = p->has_patches || ci.kind == 4;
        p->n_segs = seg_first.back();
        const int es = dtype_size(dtype);
        auto dmalloc = [&](void **ptr, size_t bytes) -> int {
            hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
            if (e == hipErrorOutOfMemory) return fail(BZ_ERR_NOMEM, "%s: device allocation of %zu bytes", fn, bytes);
            return e == hipSuccess ? BZ_OK : hip_fail(e, "hipMalloc");
        };
        p->perm_h = perm;
        int rc = dev_upload(&p->perm, perm, s);
        if (!rc) rc = dev_upload(&p->seg_first, seg_first, s);
        if (!rc) rc = dev_upload(&p->brk, brk, s);
        if (!rc) {
            std::vector<NurbsHead> nh;
            std::vector<NurbsTab> nt;
            // the span table serves FP32 plans only (see NurbsHead)
            if (!build_nurbs_tables(seg_first, brk, nh, nt, dtype == BZ_F32))
                rc = fail(BZ_ERR_INTERNAL, "%s: NURBS span table", fn);
            if (!rc) rc = dev_upload(&p->nhead, nh, s);
            if (!rc && !nt.empty()) rc = dev_upload(&p->ntab, nt, s);
        }
        if (!rc) rc = build_tiles(p, 4, n_t % 4 == 0 ? 4 : 1, kDefaultWindow, s);
        if (!rc) rc = dmalloc(&p->ctrl_s, ctrl_elems * es);
        if (!rc) rc = dmalloc(&p->w_s, w_elems * es);
        if (!rc) rc = dmalloc(reinterpret_cast<void **>(&p->seg), std::max<int64_t>(p->n_segs, 1) * 4 * (dim + 1) * sizeof(float));
        if (!rc) {
            rc = dmalloc(reinterpret_cast<void **>(&p->counters), 2 * sizeof(unsigned int));
            if (!rc && hipMemsetAsync(p->counters, 0, 2 * sizeof(unsigned int), s) != hipSuccess) rc = fail(BZ_ERR_HIP, "%s: memset", fn);
        }
        if (!rc && n_obj > 0) {  // class-sorted copies of control points and weights
            ClassInfo *cls_d = nullptr;
            rc = dev_upload(&cls_d, cls, s);
            if (!rc) {
                const int64_t n_sorted = cls.back().kind == 2 ? cls.back().first : n_obj;
                const uint32_t blocks = static_cast<uint32_t>((n_sorted + kBlock - 1) / kBlock);
                if (n_sorted > 0) {
                    if (es == 4)
                        hipLaunchKernelGGL((k_gather_sorted<uint32_t>), dim3(blocks), dim3(kBlock), 0, s, n_sorted, p->perm,
                                           cp_offset, cls_d, static_cast<int>(cls.size()), dim,
                                           static_cast<const uint32_t *>(ctrl), static_cast<const uint32_t *>(w),
                                           static_cast<uint32_t *>(p->ctrl_s), static_cast<uint32_t *>(p->w_s));
                    else
                        hipLaunchKernelGGL((k_gather_sorted<uint16_t>), dim3(blocks), dim3(kBlock), 0, s, n_sorted, p->perm,
                                           cp_offset, cls_d, static_cast<int>(cls.size()), dim,
                                           static_cast<const uint16_t *>(ctrl), static_cast<const uint16_t *>(w),
                                           static_cast<uint16_t *>(p->ctrl_s), static_cast<uint16_t *>(p->w_s));
                }
                hipError_t e = hipGetLastError();
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                (void)hipFree(cls_d);
                if (e != hipSuccess) rc = hip_fail(e, "k_gather_sorted");
            }
        }
        if (!rc && !nurbs_obj.empty()) {
            int64_t *nobj_d = nullptr;
            rc = dev_upload(&nobj_d, nurbs_obj, s);
            if (!rc) {
                const int nn = static_cast<int>(nurbs_obj.size());
                const uint32_t blocks = (nn + kBlock - 1) / kBlock;
                if (dtype == BZ_F32)
                    hipLaunchKernelGGL((k_nurbs_extract<float>), dim3(blocks), dim3(kBlock), 0, s, nn, nobj_d, cp_offset,
                                       knot_offset, static_cast<const float *>(ctrl), static_cast<const float *>(w), knots,
                                       p->seg_first, dim, p->seg);
                else if (dtype == BZ_F16)
                    hipLaunchKernelGGL((k_nurbs_extract<_Float16>), dim3(blocks), dim3(kBlock), 0, s, nn, nobj_d,
                                       cp_offset, knot_offset, static_cast<const _Float16 *>(ctrl),
                                       static_cast<const _Float16 *>(w), knots, p->seg_first, dim, p->seg);
                else
                    hipLaunchKernelGGL((k_nurbs_extract<bf16_t>), dim3(blocks), dim3(kBlock), 0, s, nn, nobj_d,
                                       cp_offset, knot_offset, static_cast<const bf16_t *>(ctrl),
                                       static_cast<const bf16_t *>(w), knots, p->seg_first, dim, p->seg);
                hipError_t e = hipGetLastError();
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                (void)hipFree(nobj_d);
                if (e != hipSuccess) rc = hip_fail(e, "k_nurbs_extract");
            }
        }
        if (!rc) {
            // default launch: the configuration the autotuner picks on MI355X for
            // mixed batches (static schedule, four sub-tiles per tile, four
            // parameters per lane where n_t allows, windows of 2^17 objects,
            // eight workgroups per CU)
            int dev = 0, cus = 0;
            hipError_t e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) rc = hip_fail(e, "device query");
            p->cus = static_cast<uint32_t>(std::max(1, cus));
            p->workgroups = 8 * p->cus;
            p->dynamic = 0;
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

static int batch_eval(const char *fn, bz_plan plan, const float *t, const float *v, float *out, bz_stream stream) {
    if (!plan) return fail(BZ_ERR_NULL, "%s: plan is required", fn);
    if (plan->n_obj == 0 || plan->n_t == 0) return BZ_OK;
    if (!t || !out) return fail(BZ_ERR_NULL, "%s: t and out are required", fn);
    if (plan->has_patches && !v)
        return fail(BZ_ERR_NULL, "%s: the plan has surface patches, which need v (bz_batch_eval_uv)", fn);
    if (!aligned(t, 4) || !aligned(v, 4) || !aligned(out, 4)) return fail(BZ_ERR_ALIGN, "%s: misaligned", fn);
    return launch_batch(plan, t, v, out, as_stream(stream), plan->workgroups, plan->dynamic, plan->vq);
}

int bz_batch_eval(bz_plan plan, const float *t, float *out, bz_stream stream) {
    return guarded("bz_batch_eval", [&]() -> int { return batch_eval("bz_batch_eval", plan, t, nullptr, out, stream); });
}

int bz_batch_eval_uv(bz_plan plan, const float *t, const float *v, float *out, bz_stream stream) {
    return guarded("bz_batch_eval_uv",
                   [&]() -> int { return batch_eval("bz_batch_eval_uv", plan, t, v, out, stream); });
}

int bz_batch_plan_autotune(bz_plan plan, const float *t, float *out, bz_stream stream, int64_t *best6) {
    return guarded("bz_batch_plan_autotune", [&]() -> int {
        if (!plan) return fail(BZ_ERR_NULL, "bz_batch_plan_autotune: plan is required");
        if (plan->n_obj == 0 || plan->n_t == 0) return BZ_OK;
        if (!t || !out) return fail(BZ_ERR_NULL, "bz_batch_plan_autotune: t and out are required");
        if (!aligned(t, 4) || !aligned(out, 4)) return fail(BZ_ERR_ALIGN, "bz_batch_plan_autotune: misaligned");
        const hipStream_t s = as_stream(stream);
        hipEvent_t e0, e1;
        BZ_CHECK_HIP(hipEventCreate(&e0));
        BZ_CHECK_HIP(hipEventCreate(&e1));
        const uint32_t cus = plan->cus;
        float best = 1e30f;
        uint32_t best_wg = plan->workgroups, best_q = plan->qpt, best_vq = plan->vq, best_win = plan->window;
        int best_dyn = plan->dynamic;
        const uint32_t qpts[] = {1, 2, 4};
        const uint32_t vqs[] = {1, 4};
        const uint32_t wg_per_cu[] = {4, 8, 12, 16};
        const uint32_t windows[] = {0, 32768, 131072, 262144};
        struct Layout {
            uint32_t win, vq, q;
        };
        std::vector<Layout> layouts;
        for (uint32_t win : windows) {
            if (win != 0 && win >= plan->n_obj) continue;  // one window is the class-major order
            for (uint32_t vq : vqs) {
                if (vq == 4 && plan->n_t % 4 != 0) continue;  // four queries of one object per lane
                for (uint32_t q : qpts) layouts.push_back(Layout{win, vq, q});
            }
        }
        // best of three rounds of 5 launches: one round is noisy enough to rank
        // close configurations wrongly.  Patches read their v from t while
        // timing (same size and layout).
        auto time_cfg = [&](uint32_t wg, int dyn, uint32_t vq, float *ms_out) -> int {
            int r0 = launch_batch(plan, t, t, out, s, wg, dyn, vq);  // warm-up
            float ms = 1e30f;
            for (int round = 0; round < 3 && !r0; ++round) {
                BZ_CHECK_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < 5 && !r0; ++r) r0 = launch_batch(plan, t, t, out, s, wg, dyn, vq);
                if (r0) break;
                BZ_CHECK_HIP(hipEventRecord(e1, s));
                BZ_CHECK_HIP(hipEventSynchronize(e1));
                float r_ms = 0;
                BZ_CHECK_HIP(hipEventElapsedTime(&r_ms, e0, e1));
                ms = std::min(ms, r_ms);
            }
            *ms_out = ms;
            return r0;
        };
        int rc = BZ_OK;
        for (const Layout &L : layouts) {
            rc = build_tiles(plan, L.q, L.vq, L.win, s);
            if (rc) break;
            for (int dyn = 1; dyn >= 0 && !rc; --dyn)
                for (uint32_t f : wg_per_cu) {
                    float ms = 0;
                    rc = time_cfg(f * cus, dyn, L.vq, &ms);
                    if (rc) break;
                    if (ms < best) {
                        best = ms;
                        best_wg = f * cus;
                        best_q = L.q;
                        best_dyn = dyn;
                        best_vq = L.vq;
                        best_win = L.win;
                    }
                }
            if (rc) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        rc = build_tiles(plan, best_q, best_vq, best_win, s);
        if (rc) return rc;
        plan->workgroups = best_wg;
        plan->dynamic = best_dyn;
        BZ_CHECK_HIP(hipStreamSynchronize(s));
        if (best6) {
            best6[0] = best_wg;
            best6[1] = best_q;
            best6[2] = static_cast<int64_t>(best * 1000.0f / 5.0f);  // microseconds per launch
            best6[3] = best_dyn;
            best6[4] = best_vq;
            best6[5] = best_win;
        }
        return BZ_OK;
    });
}

int bz_batch_plan_configure(bz_plan plan, int64_t workgroups, int sub_tiles, int schedule, int queries_per_lane,
                            int64_t window, bz_stream stream) {
    return guarded("bz_batch_plan_configure", [&]() -> int {
        const char *fn = "bz_batch_plan_configure";
        if (!plan) return fail(BZ_ERR_NULL, "%s: plan is required", fn);
        if (workgroups < 1 || workgroups > (int64_t(1) << 20)) return fail(BZ_ERR_SHAPE, "%s: workgroups", fn);
        if (sub_tiles != 1 && sub_tiles != 2 && sub_tiles != 4) return fail(BZ_ERR_SHAPE, "%s: sub_tiles", fn);
        if (schedule != 0 && schedule != 1) return fail(BZ_ERR_SHAPE, "%s: schedule", fn);
        if (queries_per_lane != 1 && queries_per_lane != 4) return fail(BZ_ERR_SHAPE, "%s: queries_per_lane", fn);
        if (queries_per_lane == 4 && plan->n_t % 4 != 0)
            return fail(BZ_ERR_UNSUPPORTED, "%s: 4 queries per lane need n_t a multiple of 4", fn);
        if (window < 0 || window > (int64_t(1) << 31) - 1) return fail(BZ_ERR_SHAPE, "%s: window", fn);
        const hipStream_t s = as_stream(stream);
        const int rc = build_tiles(plan, static_cast<uint32_t>(sub_tiles), static_cast<uint32_t>(queries_per_lane),
                                   static_cast<uint32_t>(window), s);
        if (rc) return rc;
        plan->workgroups = static_cast<uint32_t>(workgroups);
        plan->dynamic = schedule;
        BZ_CHECK_HIP(hipStreamSynchronize(s));
        return BZ_OK;
    });
}

int bz_batch_plan_info(bz_plan plan, int64_t *info4) {
    if (!plan || !info4) return fail(BZ_ERR_NULL, "bz_batch_plan_info: plan and info are required");
    info4[0] = static_cast<int64_t>(plan->classes.size());
    info4[1] = plan->n_tiles + plan->n_signed;
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
