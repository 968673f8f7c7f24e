/*
 * bzo.c -- FP64 CPU oracle for Bezier-family evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or helper with the GPU library; it is a plain, slow,
 * obviously-correct restatement of the mathematics of Anas & Wolfe,
 * "A Texture Lookup Approach to Bezier Curve Evaluation on the GPU"
 * (arXiv 2603.15447), evaluated in double precision.
 *
 * Conventions shared with the GPU library's interface (not its code):
 *   curve control points   ctrl[n][dim][deg+1]
 *   parameters             t[n_t] (shared) or t[n][n_t] (per object)
 *   results                out[dim][n*n_t], query q = c*n_t + j
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no -ffast-math,
 * so every product and sum is rounded exactly as written).
 *
 * Parity status: every function below is pinned by a CPU test against an
 * independent fact (exact rational arithmetic, a closed form, the paper's
 * printed formulas, or a second algorithm).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BZO_MAXDEG 63

int bzo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count for the parallel loops that follow (timing only: every result
   is computed per object, so the outputs do not depend on it).  Returns the
   previous count. */
int bzo_set_threads(int n)
{
#ifdef _OPENMP
    const int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}

/* Exact binomial coefficient (exact in double for n <= 63). */
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    uint64_t r = 1;
    for (int i = 0; i < k; ++i) r = r * (uint64_t)(n - i) / (uint64_t)(i + 1);
    return (double)r;
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* Linear interpolation L(a,b,t) = (1-t)a + tb, exact at t = 0 and t = 1. */
static double lerp(double a, double b, double t) { return (1.0 - t) * a + t * b; }

/* Bernstein basis polynomial B_{i,d}(t) = C(d,i) (1-t)^(d-i) t^i. */
static double bernstein(int d, int i, double t)
{
    if (i < 0 || i > d) return 0.0;
    return binom(d, i) * ipow(1.0 - t, d - i) * ipow(t, i);
}

/* ------------------------------------------------------------------ */
/* Bezier curves: de Casteljau recursive lerps (Sec. 2, first paragraph:
 * interpolate neighbouring points with the same t until one remains).   */
static double decasteljau(const double *b, int stride, int deg, double t)
{
    double tmp[BZO_MAXDEG + 1];
    for (int i = 0; i <= deg; ++i) tmp[i] = b[(int64_t)i * stride];
    for (int r = 1; r <= deg; ++r)
        for (int i = 0; i <= deg - r; ++i) tmp[i] = lerp(tmp[i], tmp[i + 1], t);
    return tmp[0];
}

/* Bernstein polynomial form (the "Polynomial" baseline of Sec. 5):
 * C(t) = sum_i B_{i,d}(t) b_i. */
static double bernstein_sum(const double *b, int deg, double t)
{
    double acc = 0.0;
    for (int i = 0; i <= deg; ++i) acc += bernstein(deg, i, t) * b[i];
    return acc;
}

static double param(const double *t, int64_t c, int64_t j, int64_t nt, int per_object)
{
    return per_object ? t[c * nt + j] : t[j];
}

void bzo_bezier_decasteljau(const double *ctrl, int64_t n, int deg, int dim, const double *t,
                            int64_t nt, int per_object, double *out)
{
    const int64_t nq = n * nt;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        for (int64_t j = 0; j < nt; ++j) {
            const double tt = param(t, c, j, nt, per_object);
            for (int k = 0; k < dim; ++k)
                out[k * nq + c * nt + j] = decasteljau(ctrl + (c * dim + k) * (deg + 1), 1, deg, tt);
        }
}

void bzo_bezier_bernstein(const double *ctrl, int64_t n, int deg, int dim, const double *t,
                          int64_t nt, int per_object, double *out)
{
    const int64_t nq = n * nt;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        for (int64_t j = 0; j < nt; ++j) {
            const double tt = param(t, c, j, nt, per_object);
            for (int k = 0; k < dim; ++k)
                out[k * nq + c * nt + j] = bernstein_sum(ctrl + (c * dim + k) * (deg + 1), deg, tt);
        }
}

/* ------------------------------------------------------------------ */
/* Seiler interpolation (Sec. 3.1).  C(t) = L(b_0, b_d, t) + (1-t)t D_1(t)
 * with D_i = 0 when 2i = d+1, d_i when 2i = d, and otherwise
 * L(d_i, d_{d-i}, t) + (1-t)t D_{i+1}(t).
 *
 * Difference terms by peeling: a degree-n polynomial Q with Bernstein
 * coefficients Q_0..Q_n satisfies Q - L(Q_0,Q_n,t) = (1-t)t Q'(t), where Q'
 * has degree n-2 and Bernstein coefficients
 *     Q'_{i-1} = (Q_i - ((n-i)/n) Q_0 - (i/n) Q_n) * C(n,i)/C(n-2,i-1).
 * Starting from Q = C gives D_1 = Q', whose end coefficients are d_1 and
 * d_{d-1}; peeling Q' gives D_2, and so on.  For the outer level this
 * reproduces the paper's d_1 and d_{d-1}; the paper gives closed forms up
 * to degree 5, peeling covers every degree.
 *
 * Storage order per curve and coordinate: [b0, bd, d1, d_{d-1}, d2,
 * d_{d-2}, ...], d+1 values, the middle term d_{d/2} once for even d.   */
static void seiler_coeffs(const double *b, int deg, double *out)
{
    double Q[BZO_MAXDEG + 1], R[BZO_MAXDEG + 1];
    for (int i = 0; i <= deg; ++i) Q[i] = b[i];
    out[0] = b[0];
    if (deg == 0) return;
    out[1] = b[deg];
    int pos = 2, n = deg;
    while (n >= 2) {
        for (int i = 1; i <= n - 1; ++i) {
            const double r = Q[i] - ((double)(n - i) / n * Q[0] + (double)i / n * Q[n]);
            R[i - 1] = r * (binom(n, i) / binom(n - 2, i - 1));
        }
        n -= 2;
        for (int i = 0; i <= n; ++i) Q[i] = R[i];
        out[pos++] = Q[0];
        if (n > 0) out[pos++] = Q[n];
    }
}

static double seiler_point(const double *sc, int deg, double t)
{
    const double st = (1.0 - t) * t;
    if (deg == 0) return sc[0];
    const int npairs = (deg - 1) / 2;
    double D = (deg % 2 == 0) ? sc[2 + 2 * npairs] : 0.0;
    for (int i = npairs; i >= 1; --i) D = lerp(sc[2 * i], sc[2 * i + 1], t) + st * D;
    return lerp(sc[0], sc[1], t) + st * D;
}

void bzo_seiler_from_bezier(const double *ctrl, int64_t n, int deg, int dim, double *seiler)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        for (int k = 0; k < dim; ++k)
            seiler_coeffs(ctrl + (c * dim + k) * (deg + 1), deg, seiler + (c * dim + k) * (deg + 1));
}

void bzo_seiler_eval(const double *seiler, int64_t n, int deg, int dim, const double *t, int64_t nt,
                     int per_object, double *out)
{
    const int64_t nq = n * nt;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        for (int64_t j = 0; j < nt; ++j) {
            const double tt = param(t, c, j, nt, per_object);
            for (int k = 0; k < dim; ++k)
                out[k * nq + c * nt + j] = seiler_point(seiler + (c * dim + k) * (deg + 1), deg, tt);
        }
}

/* ------------------------------------------------------------------ */
/* C0 piecewise quadratic chain with the shared-diagonal ("zig-zag")
 * encoding (Sec. 2.1, Eq. 1-2, Fig. 2).
 *
 * chain[2N+1][dim]: A_k = chain[2k] (segment endpoints, shared),
 *                   M_k = chain[2k+1] (middle control point of segment k).
 * grid[N+1][2][dim]: column k holds A_k in row r_k = k mod 2 (the sampling
 * path zig-zags between the rows) and a free texel x_k in the other row.
 * Segment k is the bilinear patch [A_k x_{k+1}; x_k A_{k+1}] read along its
 * diagonal, i.e. A s^2 + (x_k + x_{k+1}) s t + A' t^2 (Eq. 1), which is the
 * quadratic with middle point M_k iff (x_k + x_{k+1})/2 = M_k (Eq. 2).
 * N constraints, N+1 free texels: fix x_0 = M_0 and x_{k+1} = 2 M_k - x_k.  */
void bzo_piecewise_encode(const double *chain, int64_t nseg, int dim, double *grid)
{
    for (int k = 0; k < dim; ++k) {
        double x = chain[1 * dim + k]; /* x_0 = M_0 */
        for (int64_t s = 0; s <= nseg; ++s) {
            const int r = (int)(s & 1);
            grid[(s * 2 + r) * dim + k] = chain[(2 * s) * dim + k];
            grid[(s * 2 + (1 - r)) * dim + k] = x;
            if (s < nseg) x = 2.0 * chain[(2 * s + 1) * dim + k] - x;
        }
    }
}

/* Decode a global parameter T in [0,N] into (segment k, local t).
 * T is clamped to [0,N]; T = N maps to (N-1, 1); NaN stays NaN in t.      */
static int64_t chain_decode(double T, int64_t nseg, double *t)
{
    if (isnan(T)) { *t = NAN; return 0; }
    double Tc = T < 0.0 ? 0.0 : (T > (double)nseg ? (double)nseg : T);
    int64_t k = (int64_t)floor(Tc);
    if (k > nseg - 1) k = nseg - 1;
    *t = Tc - (double)k;
    return k;
}

void bzo_piecewise_eval(const double *grid, int64_t nseg, int dim, const double *T, int64_t nq,
                        double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        double t;
        const int64_t k = chain_decode(T[q], nseg, &t);
        const int r = (int)(k & 1);
        const double s = 1.0 - t;
        for (int c = 0; c < dim; ++c) {
            const double A = grid[(k * 2 + r) * dim + c];
            const double xk = grid[(k * 2 + 1 - r) * dim + c];
            const double xk1 = grid[((k + 1) * 2 + r) * dim + c];
            const double D = grid[((k + 1) * 2 + 1 - r) * dim + c];
            out[c * nq + q] = A * s * s + (xk + xk1) * s * t + D * t * t;
        }
    }
}

/* The chain's plain definition: segment k is the quadratic Bezier curve
 * (A_k, M_k, A_{k+1}) at local parameter t.                               */
void bzo_chain_eval(const double *chain, int64_t nseg, int dim, const double *T, int64_t nq,
                    double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        double t;
        const int64_t k = chain_decode(T[q], nseg, &t);
        for (int c = 0; c < dim; ++c) {
            double b[3] = {chain[(2 * k) * dim + c], chain[(2 * k + 1) * dim + c],
                           chain[(2 * k + 2) * dim + c]};
            out[c * nq + q] = decasteljau(b, 1, 2, t);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Rational Bezier curves (Sec. 2.2: one integral spline divided by
 * another): de Casteljau on homogeneous points (w_i b_i, w_i), then divide. */
static void rational_point(const double *b, const double *w, int dim, int deg, double t, double *res)
{
    double hw[BZO_MAXDEG + 1], h[BZO_MAXDEG + 1];
    for (int i = 0; i <= deg; ++i) hw[i] = w[i];
    const double W = decasteljau(hw, 1, deg, t);
    for (int k = 0; k < dim; ++k) {
        for (int i = 0; i <= deg; ++i) h[i] = w[i] * b[k * (deg + 1) + i];
        res[k] = decasteljau(h, 1, deg, t) / W;
    }
}

void bzo_rational_eval(const double *ctrl, const double *w, int64_t n, int deg, int dim,
                       const double *t, int64_t nt, int per_object, double *out)
{
    const int64_t nq = n * nt;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        for (int64_t j = 0; j < nt; ++j) {
            double res[8];
            rational_point(ctrl + c * dim * (deg + 1), w + c * (deg + 1), dim, deg,
                           param(t, c, j, nt, per_object), res);
            for (int k = 0; k < dim; ++k) out[k * nq + c * nt + j] = res[k];
        }
}

/* ------------------------------------------------------------------ */
/* NURBS (Sec. 2.2) by the rational de Boor algorithm on homogeneous
 * points; a different algorithm from Bezier-segment extraction, so the two
 * check each other.  U[0..ncp+p], clamped; u is clamped to [U_p, U_ncp].  */
static int nurbs_span(const double *U, int ncp, int p, double u)
{
    const int n = ncp - 1;
    if (u >= U[n + 1]) {
        int j = n;
        while (j > p && !(U[j] < U[j + 1])) --j;
        return j;
    }
    int j = p;
    while (j < n && !(u < U[j + 1])) ++j;
    return j;
}

static void nurbs_point(const double *P, int stride_dim, const double *w, const double *U, int ncp,
                        int p, int dim, double u, double *res)
{
    double d[BZO_MAXDEG + 1][9];
    if (isnan(u)) {
        for (int k = 0; k < dim; ++k) res[k] = NAN;
        return;
    }
    if (u < U[p]) u = U[p];
    if (u > U[ncp]) u = U[ncp];
    const int j = nurbs_span(U, ncp, p, u);
    for (int i = 0; i <= p; ++i) {
        const int idx = j - p + i;
        for (int k = 0; k < dim; ++k) d[i][k] = w[idx] * P[(int64_t)k * stride_dim + idx];
        d[i][dim] = w[idx];
    }
    for (int r = 1; r <= p; ++r)
        for (int i = p; i >= r; --i) {
            const int idx = j - p + i;
            const double a = (u - U[idx]) / (U[idx + p + 1 - r] - U[idx]);
            for (int k = 0; k <= dim; ++k) d[i][k] = (1.0 - a) * d[i - 1][k] + a * d[i][k];
        }
    for (int k = 0; k < dim; ++k) res[k] = d[p][k] / d[p][dim];
}

/* One NURBS curve: ctrl[dim][ncp], w[ncp], knots[ncp+p+1], u[nu] -> out[dim][nu]. */
void bzo_nurbs_eval(const double *ctrl, const double *w, const double *knots, int ncp, int p, int dim,
                    const double *u, int64_t nu, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nu; ++q) {
        double res[8];
        nurbs_point(ctrl, ncp, w, knots, ncp, p, dim, u[q], res);
        for (int k = 0; k < dim; ++k) out[k * nu + q] = res[k];
    }
}

static double tensor_point(const double *P, int du, int dv, int dw, double u, double v, double w);

/* Mixed batch: kind_degree[o] = kind<<8 | degree (0 Bezier, 1 rational,
 * 2 NURBS, 3 tensor-product surface patch with degree byte du<<4 | dv, Sec.
 * 2.2).  Object o's control points are ctrl[cp_offset[o]*dim ...] laid out
 * [dim][ncp] (a patch's ncp = (du+1)(dv+1) points indexed i*(dv+1)+j); w is
 * aligned with control points; NURBS knots at knots[knot_offset[o] ...].
 * t[n_obj][nt] (a patch's u), v[n_obj][nt] (a patch's v; read for patches
 * only, may be NULL without them), out[dim][n_obj*nt].                     */
void bzo_batch_eval(int64_t n_obj, const uint16_t *kind_degree, const int64_t *cp_offset,
                    const double *ctrl, const double *w, const int64_t *knot_offset,
                    const double *knots, int dim, const double *t, const double *v, int64_t nt, double *out)
{
    const int64_t nq = n_obj * nt;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t o = 0; o < n_obj; ++o) {
        const int kind = kind_degree[o] >> 8, deg = kind_degree[o] & 0xff;
        const int ncp = (int)(cp_offset[o + 1] - cp_offset[o]);
        const double *P = ctrl + cp_offset[o] * dim;
        const double *W = w + cp_offset[o];
        for (int64_t j = 0; j < nt; ++j) {
            const double tt = t[o * nt + j];
            double res[8];
            if (kind == 0) {
                for (int k = 0; k < dim; ++k) res[k] = decasteljau(P + k * ncp, 1, deg, tt);
            } else if (kind == 1) {
                rational_point(P, W, dim, deg, tt, res);
            } else if (kind == 2) {
                nurbs_point(P, ncp, W, knots + knot_offset[o], ncp, deg, dim, tt, res);
            } else {
                const int du = deg >> 4, dv = deg & 15;
                for (int k = 0; k < dim; ++k) res[k] = tensor_point(P + k * ncp, du, dv, 0, tt, v[o * nt + j], 0.0);
            }
            for (int k = 0; k < dim; ++k) out[k * nq + o * nt + j] = res[k];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Tensor-product surfaces and volumes (Sec. 2.2): S = sum_ijk B_i(u)
 * B_j(v) B_k(w) P_ijk, evaluated separably by de Casteljau along w, then v,
 * then u.  ctrl[n_obj][dim][(du+1)(dv+1)(dw+1)], index (i*(dv+1)+j)*(dw+1)+k.  */
static double tensor_point(const double *P, int du, int dv, int dw, double u, double v, double w)
{
    double row[BZO_MAXDEG + 1], col[BZO_MAXDEG + 1];
    for (int i = 0; i <= du; ++i) {
        for (int j = 0; j <= dv; ++j) row[j] = decasteljau(P + (i * (dv + 1) + j) * (dw + 1), 1, dw, w);
        col[i] = decasteljau(row, 1, dv, v);
    }
    return decasteljau(col, 1, du, u);
}

/* Points mode: uvw[n_obj][n_per][npar] with npar = 2 (surfaces, dw = 0) or
 * 3 (volumes); out[dim][n_obj*n_per].                                      */
void bzo_tensor_points(const double *ctrl, int64_t n_obj, int du, int dv, int dw, int dim,
                       const double *uvw, int64_t n_per, double *out)
{
    const int npar = dw > 0 ? 3 : 2;
    const int ncp = (du + 1) * (dv + 1) * (dw + 1);
    const int64_t nq = n_obj * n_per;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < n_obj; ++o)
        for (int64_t j = 0; j < n_per; ++j) {
            const double *p = uvw + (o * n_per + j) * npar;
            const double w = npar == 3 ? p[2] : 0.0;
            for (int k = 0; k < dim; ++k)
                out[k * nq + o * n_per + j] = tensor_point(ctrl + (o * dim + k) * ncp, du, dv, dw, p[0], p[1], w);
        }
}

/* Grid mode for surfaces: u_a = a/(nu-1), v_b = b/(nv-1) inclusive;
 * out[dim][n_obj*nu*nv], point index o*nu*nv + a*nv + b.                   */
void bzo_tensor_grid(const double *ctrl, int64_t n_obj, int du, int dv, int dim, int nu, int nv,
                     double *out)
{
    const int ncp = (du + 1) * (dv + 1);
    const int64_t per = (int64_t)nu * nv, nq = n_obj * per;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < n_obj; ++o)
        for (int a = 0; a < nu; ++a)
            for (int b = 0; b < nv; ++b) {
                const double u = nu > 1 ? (double)a / (nu - 1) : 0.0;
                const double v = nv > 1 ? (double)b / (nv - 1) : 0.0;
                for (int k = 0; k < dim; ++k)
                    out[k * nq + o * per + a * nv + b] = tensor_point(ctrl + (o * dim + k) * ncp, du, dv, 0, u, v, 0.0);
            }
}

/* ------------------------------------------------------------------ */
/* Adjoint of curve evaluation.  For C(t) = H(t)/W(t) with H = sum w_i b_i
 * B_i, W = sum w_i B_i (W = 1, w_i = 1 for integral curves):
 *   dC/db_i = w_i B_i / W,   dC/dw_i = B_i (b_i - C) / W,
 *   dC/dt   = (H' - C W') / W, with the hodograph
 *   H' = d sum_{i<d} (w_{i+1} b_{i+1} - w_i b_i) B_{i,d-1}(t).
 * Given grad_out[dim][n*nt] (dL/dC) this accumulates
 *   grad_ctrl[n][dim][deg+1], grad_w[n][deg+1] (rational only) and
 *   grad_t[n][nt] (per-object t only).  Outputs are overwritten.           */
void bzo_bezier_adjoint(const double *ctrl, const double *w, int64_t n, int deg, int dim,
                        const double *t, int64_t nt, int per_object, const double *gout,
                        double *gctrl, double *gw, double *gt)
{
    const int64_t nq = n * nt;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        const double *b = ctrl + c * dim * (deg + 1);
        const double *wc = w ? w + c * (deg + 1) : 0;
        double *gb = gctrl ? gctrl + c * dim * (deg + 1) : 0;
        double *gwc = gw ? gw + c * (deg + 1) : 0;
        if (gb) memset(gb, 0, sizeof(double) * dim * (deg + 1));
        if (gwc) memset(gwc, 0, sizeof(double) * (deg + 1));
        for (int64_t j = 0; j < nt; ++j) {
            const double tt = param(t, c, j, nt, per_object);
            double B[BZO_MAXDEG + 1], Bm[BZO_MAXDEG + 1];
            for (int i = 0; i <= deg; ++i) B[i] = bernstein(deg, i, tt);
            for (int i = 0; i < deg; ++i) Bm[i] = bernstein(deg - 1, i, tt);
            double W = 1.0, Wp = 0.0;
            if (wc) {
                W = 0.0;
                for (int i = 0; i <= deg; ++i) W += wc[i] * B[i];
                for (int i = 0; i < deg; ++i) Wp += deg * (wc[i + 1] - wc[i]) * Bm[i];
            }
            double dt_acc = 0.0;
            for (int k = 0; k < dim; ++k) {
                const double *bk = b + k * (deg + 1);
                const double g = gout[k * nq + c * nt + j];
                double H = 0.0, Hp = 0.0;
                for (int i = 0; i <= deg; ++i) H += (wc ? wc[i] : 1.0) * bk[i] * B[i];
                for (int i = 0; i < deg; ++i) {
                    const double wi1 = wc ? wc[i + 1] : 1.0, wi = wc ? wc[i] : 1.0;
                    Hp += deg * (wi1 * bk[i + 1] - wi * bk[i]) * Bm[i];
                }
                const double C = H / W;
                dt_acc += g * (Hp - C * Wp) / W;
                if (gb)
                    for (int i = 0; i <= deg; ++i) gb[k * (deg + 1) + i] += g * (wc ? wc[i] : 1.0) * B[i] / W;
                if (gwc)
                    for (int i = 0; i <= deg; ++i) gwc[i] += g * B[i] * (bk[i] - C) / W;
            }
            if (gt && per_object) gt[c * nt + j] = dt_acc;
        }
    }
}

/* Least-squares fit of integral curves to targets y[dim][n*nt]:
 *   L = (1/M) sum_q |C(t_q) - y_q|^2, M = m_total (n*nt when m_total <= 0;
 *   a larger M lets a subset of curves reproduce a bigger problem's scale).
 * Returns L and writes dL/dctrl[n][dim][deg+1] and dL/dt[n][nt].           */
double bzo_fit_loss_grad(const double *ctrl, int64_t n, int deg, int dim, const double *t, int64_t nt,
                         const double *y, double m_total, double *gctrl, double *gt)
{
    const int64_t nq = n * nt;
    const double M = m_total > 0.0 ? m_total : (double)nq;
    double *C = (double *)malloc(sizeof(double) * (size_t)(nq * dim));
    double *g = (double *)malloc(sizeof(double) * (size_t)(nq * dim));
    bzo_bezier_decasteljau(ctrl, n, deg, dim, t, nt, 1, C);
    double L = 0.0;
    for (int64_t i = 0; i < nq * dim; ++i) {
        const double r = C[i] - y[i];
        L += r * r;
        g[i] = 2.0 * r / M;
    }
    bzo_bezier_adjoint(ctrl, 0, n, deg, dim, t, nt, 1, g, gctrl, 0, gt);
    free(C);
    free(g);
    return L / M;
}

/* Adam (Kingma & Ba 2015) with bias correction, step counted from 1;
 * after the update each parameter is clamped to [lo,hi] when lo <= hi.     */
void bzo_adam(double *p, double *m, double *v, const double *g, int64_t n, int step, double lr,
              double b1, double b2, double eps, double lo, double hi)
{
    const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        const double mh = m[i] / c1, vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
        if (lo <= hi) p[i] = p[i] < lo ? lo : (p[i] > hi ? hi : p[i]);
    }
}

/* ------------------------------------------------------------------ */
/* C0 piecewise cubic chain from two stacked zig-zag layers (Sec. 2.1, last
 * paragraph: two C0 quadratic textures front to back, the depth read
 * interpolating between them).  chain[3N+1][dim]: segment k is the cubic
 * Bezier (P_3k, P_3k+1, P_3k+2, P_3k+3).  Reading: both layers share the
 * on-path texels A_k = P_3k; their middle points are
 *   E0_k = (3 P_3k+1 - P_3k) / 2   and   E1_k = (3 P_3k+2 - P_3k+3) / 2,
 * because (1-t) Q0(t) + t Q1(t) with Q_l = A s^2 + 2 E_l s t + A' t^2 has
 * Bernstein coefficients (A, (A + 2 E0)/3, (A' + 2 E1)/3, A').
 * grid[N+1][2 layers][2 rows][dim]; each layer is zig-zag encoded as above.  */
void bzo_cubic_chain_encode(const double *chain, int64_t nseg, int dim, double *grid)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)((2 * nseg + 1) * dim));
    double *g = (double *)malloc(sizeof(double) * (size_t)((nseg + 1) * 2 * dim));
    for (int layer = 0; layer < 2; ++layer) {
        for (int64_t k = 0; k <= nseg; ++k)
            for (int c = 0; c < dim; ++c) q[(2 * k) * dim + c] = chain[(3 * k) * dim + c];
        for (int64_t k = 0; k < nseg; ++k)
            for (int c = 0; c < dim; ++c) {
                const double A = chain[(3 * k) * dim + c], A1 = chain[(3 * k + 3) * dim + c];
                const double B = chain[(3 * k + 1) * dim + c], C = chain[(3 * k + 2) * dim + c];
                q[(2 * k + 1) * dim + c] = layer == 0 ? (3.0 * B - A) / 2.0 : (3.0 * C - A1) / 2.0;
            }
        bzo_piecewise_encode(q, nseg, dim, g);
        for (int64_t k = 0; k <= nseg; ++k)
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < dim; ++c) grid[((k * 2 + layer) * 2 + r) * dim + c] = g[(k * 2 + r) * dim + c];
    }
    free(q);
    free(g);
}

/* Trilinear read of the two layers along the zig-zag path: the bilinear
 * value of each layer (Eq. 1), then a lerp between layers with the same t. */
void bzo_cubic_chain_grid_eval(const double *grid, int64_t nseg, int dim, const double *T, int64_t nq, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        double t;
        const int64_t k = chain_decode(T[q], nseg, &t);
        const int r = (int)(k & 1);
        const double s = 1.0 - t;
        for (int c = 0; c < dim; ++c) {
            double v[2];
            for (int layer = 0; layer < 2; ++layer) {
                const double A = grid[((k * 2 + layer) * 2 + r) * dim + c];
                const double xk = grid[((k * 2 + layer) * 2 + 1 - r) * dim + c];
                const double xk1 = grid[(((k + 1) * 2 + layer) * 2 + r) * dim + c];
                const double D = grid[(((k + 1) * 2 + layer) * 2 + 1 - r) * dim + c];
                v[layer] = A * s * s + (xk + xk1) * s * t + D * t * t;
            }
            out[c * nq + q] = lerp(v[0], v[1], t);
        }
    }
}

/* The chain's plain definition: segment k is the cubic Bezier
 * (P_3k .. P_3k+3) at local parameter t (de Casteljau).                    */
void bzo_cubic_chain_eval(const double *chain, int64_t nseg, int dim, const double *T, int64_t nq, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        double t;
        const int64_t k = chain_decode(T[q], nseg, &t);
        for (int c = 0; c < dim; ++c) {
            double b[4];
            for (int i = 0; i < 4; ++i) b[i] = chain[(3 * k + i) * dim + c];
            out[c * nq + q] = decasteljau(b, 1, 3, t);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Texture-filter emulation (Sec. 2: texel values sit at texel centres and
 * 2x2 / 2x2x2 textures hold de Casteljau levels; Sec. 2.1: the zig-zag
 * chain texture; Sec. 2.3: fixed-point filter weights with 8 fractional
 * bits; Sec. 4 with Table 1: Seiler textures read at (t, st[, st]), degrees 6 and 7 at (t, st, (st)^2);
 * Fig. 3: the trilinear, hybrid and Seiler modes of a cubic).
 *
 * Per axis a linear filter blends the two texels around the sample with
 * the sample's fractional position between their centres.  Readings (the
 * paper names the 8 fractional bits but no rounding rule):
 *   - that fraction is rounded to F fractional bits, to nearest with halves
 *     up (rounding = 0) or by truncation (rounding = 1); F = 0 leaves it
 *     unrounded;
 *   - coordinates and the weight decision are FP32 (shader arithmetic), each
 *     operation rounded as written; the blends here are FP64;
 *   - every axis of a curve texture has two texels and a parameter p in
 *     [0,1] is placed by the texel-centre remap x = 1/4 + p/2 (normalised),
 *     which the filter turns back into the texel-space position 2x - 1/2;
 *   - clamp-to-edge addressing: the curve parameter is clamped to [0,1] (the
 *     shader lerps use the clamped value too), the chain's T to [0,N].     */
#define BZO_TEX_DC 0
#define BZO_TEX_HYBRID 1
#define BZO_TEX_SEILER 2

/* Fraction f in [0,1] held with F fractional bits. */
static double tex_round_fraction(float f, int frac_bits, int rounding)
{
    if (frac_bits == 0) return (double)f;
    const float scaled = ldexpf(f, frac_bits); /* exact: power-of-two scale */
    const float q = rounding == 0 ? floorf(scaled + 0.5f) : floorf(scaled);
    return ldexp((double)q, -frac_bits);
}

/* Filter weight of a 2-texel axis sampled at parameter p in [0,1]. */
double bzo_tex_axis_weight(float p, int frac_bits, int rounding)
{
    const float x = 0.25f + 0.5f * p; /* normalised coordinate */
    const float xb = 2.0f * x - 0.5f; /* texel-space position, centres at 0 and 1 */
    if (isnan(xb)) return NAN;
    if (xb <= 0.0f) return 0.0;
    if (xb >= 1.0f) return 1.0;
    return tex_round_fraction(xb, frac_bits, rounding);
}

void bzo_tex_axis_weights(const float *p, int64_t n, int frac_bits, int rounding, double *w)
{
    for (int64_t i = 0; i < n; ++i) w[i] = bzo_tex_axis_weight(p[i], frac_bits, rounding);
}

/* Bilinear filter of a 2x2 layer L[row*2 + col]: x blends along a row
 * (column 0 -> 1), y across rows (row 0 -> 1).                             */
static double tex_bilinear(const double *L, double wx, double wy)
{
    return (1.0 - wy) * ((1.0 - wx) * L[0] + wx * L[1]) + wy * ((1.0 - wx) * L[2] + wx * L[3]);
}

static double tex_trilinear(const double *L0, const double *L1, double wx, double wy, double wz)
{
    return (1.0 - wz) * tex_bilinear(L0, wx, wy) + wz * tex_bilinear(L1, wx, wy);
}

/* Texels per curve and coordinate. */
int bzo_tex_texels(int deg, int mode)
{
    if (mode == BZO_TEX_SEILER) return deg <= 3 ? 4 : 8;
    return 4 * (deg - 1);
}

/* Curve textures, tex[n][dim][texels].
 * De Casteljau / hybrid (degree >= 2): deg-1 layers, layer i the quadratic
 * (b_i, b_i+1, b_i+2) as [[b_i, b_i+1], [b_i+1, b_i+2]]: its bilinear read
 * at (t,t) is that quadratic's point, and the trilinear read of layers i
 * and i+1 at (t,t,t) is the point of the cubic (b_i .. b_i+3).
 * Seiler (degree 2..5 as Table 1, 6..7 below), with d_j the difference terms:
 *   2: [[b0, b2], [b0+d1, b2+d1]]      3: [[b0, b3], [b0+d1, b3+d2]]
 *   4: [[b0, b4], [b0, b4]] then [[b0+d1, b4+d3], [b0+d1+d2, b4+d3+d2]]
 *   5: [[b0, b5], [b0, b5]] then [[b0+d1, b5+d4], [b0+d1+d2, b5+d4+d3]]
 * read at (t, st) or (t, st, st).  Degrees 6 and 7 (the 2x2x2 case the
 * paper's conclusion expects to exist): a trilinear read at (x, y, z) spans
 * {1, x, y, z, xy, xz, yz, xyz}; at (t, st, (st)^2) these have the distinct
 * degrees 0..7 in t, so every degree-7 curve fits.  Matching
 *   L(b0,bd,t) + st L(d1,d_{d-1},t) + (st)^2 L(d2,d_{d-2},t) + (st)^3 L(d3,d_{d-3},t)
 * (d_{d-3} = d3 for d = 6) term by term gives
 *   6/7: [[b0, bd], [b0+d1, bd+d_{d-1}]] then
 *        [[b0+d2, bd+d_{d-2}], [b0+d1+d2+d3, bd+d_{d-1}+d_{d-2}+d_{d-3}]]      */
void bzo_tex_build(const double *ctrl, int64_t n, int deg, int dim, int mode, double *tex)
{
    const int nt = bzo_tex_texels(deg, mode);
    for (int64_t c = 0; c < n; ++c)
        for (int k = 0; k < dim; ++k) {
            const double *b = ctrl + (c * dim + k) * (deg + 1);
            double *T = tex + (c * dim + k) * nt;
            if (mode != BZO_TEX_SEILER) {
                for (int i = 0; i < deg - 1; ++i) {
                    T[4 * i + 0] = b[i];
                    T[4 * i + 1] = b[i + 1];
                    T[4 * i + 2] = b[i + 1];
                    T[4 * i + 3] = b[i + 2];
                }
                continue;
            }
            double sc[BZO_MAXDEG + 1];
            seiler_coeffs(b, deg, sc);
            /* sc = [b0, bd, d1, d_{d-1}, d2, d_{d-2}, ...] */
            const double b0 = sc[0], bd = sc[1];
            if (deg == 2) {
                const double d1 = sc[2];
                T[0] = b0, T[1] = bd, T[2] = b0 + d1, T[3] = bd + d1;
            } else if (deg == 3) {
                const double d1 = sc[2], d2 = sc[3];
                T[0] = b0, T[1] = bd, T[2] = b0 + d1, T[3] = bd + d2;
            } else if (deg >= 6) {
                /* deg 6: d1, d5, d2, d4, d3 = sc[2..6];
                 * deg 7: d1, d6, d2, d5, d3, d4 = sc[2..7]                   */
                const double d1 = sc[2], dl1 = sc[3], d2 = sc[4], dl2 = sc[5], d3 = sc[6];
                const double dl3 = deg == 6 ? sc[6] : sc[7];
                T[0] = b0, T[1] = bd, T[2] = b0 + d1, T[3] = bd + dl1;
                T[4] = b0 + d2, T[5] = bd + dl2;
                T[6] = b0 + d1 + d2 + d3, T[7] = bd + dl1 + dl2 + dl3;
            } else {
                /* deg 4: d1, d3, d2 = sc[2], sc[3], sc[4];
                 * deg 5: d1, d4, d2, d3 = sc[2], sc[3], sc[4], sc[5]         */
                const double d1 = sc[2], dl = sc[3], d2 = sc[4];
                const double dm = deg == 4 ? d2 : sc[5];
                T[0] = b0, T[1] = bd, T[2] = b0, T[3] = bd;
                T[4] = b0 + d1, T[5] = bd + dl;
                T[6] = b0 + d1 + d2, T[7] = bd + dl + dm;
            }
        }
}

/* Sampling of the curve textures (float texels, as stored for the GPU). */
void bzo_tex_eval(const float *tex, int64_t n, int deg, int dim, int mode, const float *t, int64_t nt,
                  int per_object, int frac_bits, int rounding, double *out)
{
    const int ntx = bzo_tex_texels(deg, mode);
    const int64_t nq = n * nt;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c)
        for (int64_t j = 0; j < nt; ++j) {
            float p = per_object ? t[c * nt + j] : t[j];
            if (p < 0.0f) p = 0.0f;
            if (p > 1.0f) p = 1.0f;
            const double w = bzo_tex_axis_weight(p, frac_bits, rounding);
            const float st = (1.0f - p) * p;
            const double wst = bzo_tex_axis_weight(st, frac_bits, rounding);
            const double wst2 = bzo_tex_axis_weight(st * st, frac_bits, rounding);
            for (int k = 0; k < dim; ++k) {
                const float *T = tex + (c * dim + k) * ntx;
                double L[8 * BZO_MAXDEG];
                for (int i = 0; i < ntx; ++i) L[i] = (double)T[i];
                double v;
                if (isnan(p)) {
                    v = NAN;
                } else if (mode == BZO_TEX_SEILER) {
                    v = deg <= 3 ? tex_bilinear(L, w, wst)
                                 : tex_trilinear(L, L + 4, w, wst, deg <= 5 ? wst : wst2);
                } else {
                    /* texture reads: level-3 points (trilinear, de Casteljau
                     * mode from degree 3) or level-2 points (bilinear) */
                    double lv[BZO_MAXDEG + 1];
                    int m;
                    if (mode == BZO_TEX_DC && deg >= 3) {
                        m = deg - 2;
                        for (int i = 0; i < m; ++i) lv[i] = tex_trilinear(L + 4 * i, L + 4 * i + 4, w, w, w);
                    } else {
                        m = deg - 1;
                        for (int i = 0; i < m; ++i) lv[i] = tex_bilinear(L + 4 * i, w, w);
                    }
                    /* remaining de Casteljau levels in the shader, exact t */
                    v = decasteljau(lv, 1, m - 1, (double)p);
                }
                out[k * nq + c * nt + j] = v;
            }
        }
}

/* Zig-zag chain (grid[N+1][2][dim], as bzo_piecewise_encode writes it) read
 * by the emulated bilinear filter: texel (column, row) has its centre at
 * (column + 1/2, row + 1/2) in texel space; segment k's sample runs from the
 * centre of (k, k mod 2) to that of (k+1, 1 - k mod 2).                    */
void bzo_chain_texemu_eval(const float *grid, int64_t nseg, int dim, const float *T, int64_t nq, int frac_bits,
                           int rounding, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        float Tc = T[q];
        if (isnan(Tc)) {
            for (int c = 0; c < dim; ++c) out[c * nq + q] = NAN;
            continue;
        }
        if (Tc < 0.0f) Tc = 0.0f;
        if (Tc > (float)nseg) Tc = (float)nseg;
        const float x = Tc + 0.5f;
        const float xb = x - 0.5f;
        int64_t k = (int64_t)floorf(xb);
        if (k > nseg - 1) k = nseg - 1;
        const float fx = xb - (float)k;
        const double wx = tex_round_fraction(fx, frac_bits, rounding);
        const int r = (int)(k & 1);
        const float y = r == 0 ? fx + 0.5f : 1.5f - fx;
        float yb = y - 0.5f;
        if (yb < 0.0f) yb = 0.0f;
        if (yb > 1.0f) yb = 1.0f;
        const double wy = tex_round_fraction(yb, frac_bits, rounding);
        for (int c = 0; c < dim; ++c) {
            const double L[4] = {grid[(k * 2 + 0) * dim + c], grid[((k + 1) * 2 + 0) * dim + c],
                                 grid[(k * 2 + 1) * dim + c], grid[((k + 1) * 2 + 1) * dim + c]};
            out[c * nq + q] = tex_bilinear(L, wx, wy);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Seiler surfaces and volumes (Sec. 2.2 splits a tensor product over its
 * axes; Sec. 3 gives the Seiler form of one axis; Sec. 6 leaves surfaces
 * and volumes in Seiler form open).  Reading: per-axis Seiler terms -- the
 * Seiler conversion of a curve applied to every fibre of the control net
 * along w, then v, then u (it is linear, so the order is immaterial);
 * storage sc[n][dim][(du+1)(dv+1)(dw+1)] indexed like the control points,
 * each axis in the curve order [b0, bd, d1, d_{d-1}, ...].  Evaluation nests
 * the Seiler recursion of each axis: w innermost, then v, then u.          */
static void fibre_to_seiler(double *a, int64_t stride, int deg)
{
    double b[BZO_MAXDEG + 1] = {0}, sc[BZO_MAXDEG + 1];
    if (deg < 1) return;
    for (int i = 0; i <= deg; ++i) b[i] = a[i * stride];
    seiler_coeffs(b, deg, sc);
    for (int i = 0; i <= deg; ++i) a[i * stride] = sc[i];
}

void bzo_tensor_to_seiler(const double *ctrl, int64_t n, int du, int dv, int dw, int dim, double *sc)
{
    const int nv = dv + 1, nw = dw + 1, ncp = (du + 1) * nv * nw;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n * dim; ++r) {
        double *a = sc + r * ncp;
        for (int e = 0; e < ncp; ++e) a[e] = ctrl[r * ncp + e];
        for (int i = 0; i <= du; ++i)
            for (int j = 0; j <= dv; ++j) fibre_to_seiler(a + (i * nv + j) * nw, 1, dw);
        for (int i = 0; i <= du; ++i)
            for (int k = 0; k <= dw; ++k) fibre_to_seiler(a + i * nv * nw + k, nw, dv);
        for (int j = 0; j <= dv; ++j)
            for (int k = 0; k <= dw; ++k) fibre_to_seiler(a + j * nw + k, nv * nw, du);
    }
}

static double seiler_fibre_point(const double *a, int64_t stride, int deg, double t)
{
    double sc[BZO_MAXDEG + 1];
    for (int i = 0; i <= deg; ++i) sc[i] = a[i * stride];
    return seiler_point(sc, deg, t);
}

void bzo_tensor_seiler_points(const double *sc, int64_t n, int du, int dv, int dw, int dim, const double *uvw,
                              int64_t n_per, double *out)
{
    const int nv = dv + 1, nw = dw + 1, ncp = (du + 1) * nv * nw;
    const int npar = dw > 0 ? 3 : 2;
    const int64_t nq = n * n_per;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < n; ++o)
        for (int64_t j = 0; j < n_per; ++j) {
            const double *p = uvw + (o * n_per + j) * npar;
            for (int c = 0; c < dim; ++c) {
                const double *a = sc + (o * dim + c) * ncp;
                double Ru[BZO_MAXDEG + 1];
                for (int i = 0; i <= du; ++i) {
                    double Rv[BZO_MAXDEG + 1];
                    for (int jj = 0; jj <= dv; ++jj)
                        Rv[jj] = dw > 0 ? seiler_fibre_point(a + (i * nv + jj) * nw, 1, dw, p[2]) : a[i * nv + jj];
                    Ru[i] = seiler_point(Rv, dv, p[1]);
                }
                out[c * nq + o * n_per + j] = seiler_point(Ru, du, p[0]);
            }
        }
}

/* ------------------------------------------------------------------ */
/* Surfaces through the emulated filter (Sec. 2.2: a surface splits its
 * order between the texture and the shader; Sec. 6: Seiler surfaces in the
 * interpolator).  Patch ctrl[n][dim][(du+1)(dv+1)] (u major), du in {2, 3},
 * dv in 1..4.  For every v-index j the u-fibre gets its own curve texture:
 *   de Casteljau (BZO_TEX_DC): the layers of bzo_tex_build for (P_0j..P_duj),
 *     read at (u,u[,u]) -> the isoline control point R_j(u); the shader then
 *     runs de Casteljau over R_0..R_dv at the exact v.
 *   Seiler (BZO_TEX_SEILER): the net converted to per-axis Seiler terms s_kj
 *     (bzo_tensor_to_seiler), fibre j as the 2x2 Seiler texture of degree du
 *     (Table 1); textures j and j+1 stacked front to back form a 2x2x2
 *     texture whose trilinear read at (u, su, v) is L(c_j, c_j+1, v), c_j the
 *     v-direction Seiler terms of the isoline at u.  The shader finishes the
 *     v recursion: pairs (0,1), (2,3) by trilinear reads, an unpaired middle
 *     term (even dv) by a bilinear read, then c = r0 + sv (r1 + sv c_mid).
 * Texels per coordinate: (dv+1) x 4(du-1) (de Casteljau) or (dv+1) x 4 (Seiler).
 * Weights as bzo_tex_axis_weight; v is clamped to [0,1] like u.            */
int bzo_tex_patch_texels(int du, int dv, int mode)
{
    return (dv + 1) * (mode == BZO_TEX_SEILER ? 4 : 4 * (du - 1));
}

void bzo_tex_patch_build(const double *ctrl, int64_t n, int du, int dv, int dim, int mode, double *tex)
{
    const int ncp = (du + 1) * (dv + 1), per = mode == BZO_TEX_SEILER ? 4 : 4 * (du - 1);
    double *sc = (double *)malloc(sizeof(double) * (size_t)(n * dim * ncp));
    if (mode == BZO_TEX_SEILER) bzo_tensor_to_seiler(ctrl, n, du, dv, 0, dim, sc);
    else memcpy(sc, ctrl, sizeof(double) * (size_t)(n * dim * ncp));
    for (int64_t r = 0; r < n * dim; ++r)
        for (int j = 0; j <= dv; ++j) {
            double fib[4];
            for (int i = 0; i <= du; ++i) fib[i] = sc[r * ncp + i * (dv + 1) + j];
            double *T = tex + (r * (dv + 1) + j) * per;
            if (mode != BZO_TEX_SEILER) {
                for (int i = 0; i < du - 1; ++i) {
                    T[4 * i + 0] = fib[i];
                    T[4 * i + 1] = fib[i + 1];
                    T[4 * i + 2] = fib[i + 1];
                    T[4 * i + 3] = fib[i + 2];
                }
            } else if (du == 2) { /* [b0, b2, d1] */
                T[0] = fib[0], T[1] = fib[1], T[2] = fib[0] + fib[2], T[3] = fib[1] + fib[2];
            } else { /* [b0, b3, d1, d2] */
                T[0] = fib[0], T[1] = fib[1], T[2] = fib[0] + fib[2], T[3] = fib[1] + fib[3];
            }
        }
    free(sc);
}

void bzo_tex_patch_eval(const float *tex, int64_t n, int du, int dv, int dim, int mode, const float *uv,
                        int64_t n_per, int frac_bits, int rounding, double *out)
{
    const int per = mode == BZO_TEX_SEILER ? 4 : 4 * (du - 1);
    const int64_t nq = n * n_per;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < n; ++o)
        for (int64_t q = 0; q < n_per; ++q) {
            float u = uv[(o * n_per + q) * 2], v = uv[(o * n_per + q) * 2 + 1];
            u = u < 0.0f ? 0.0f : (u > 1.0f ? 1.0f : u);
            v = v < 0.0f ? 0.0f : (v > 1.0f ? 1.0f : v);
            const double wu = bzo_tex_axis_weight(u, frac_bits, rounding);
            const double wsu = bzo_tex_axis_weight((1.0f - u) * u, frac_bits, rounding);
            const double wv = bzo_tex_axis_weight(v, frac_bits, rounding);
            for (int c = 0; c < dim; ++c) {
                double L[5 * 8];
                const float *T = tex + (o * dim + c) * (int64_t)(dv + 1) * per;
                for (int e = 0; e < (dv + 1) * per; ++e) L[e] = (double)T[e];
                double val;
                if (isnan(u) || isnan(v)) {
                    val = NAN;
                } else if (mode != BZO_TEX_SEILER) {
                    double R[5];
                    for (int j = 0; j <= dv; ++j)
                        R[j] = du == 3 ? tex_trilinear(L + j * 8, L + j * 8 + 4, wu, wu, wu)
                                       : tex_bilinear(L + j * 4, wu, wu);
                    val = decasteljau(R, 1, dv, (double)v);
                } else {
                    const double sv = (1.0 - (double)v) * (double)v;
                    /* v-Seiler terms in storage order [b0, bd, d1, d_{d-1}, d2 ...]:
                     * pairs (0,1) and (2,3) by trilinear reads, the middle term
                     * of even dv (index dv) by a bilinear read                 */
                    const double r0 = tex_trilinear(L, L + 4, wu, wsu, wv);
                    double acc = 0.0;
                    if (dv == 2) acc = tex_bilinear(L + 8, wu, wsu);
                    if (dv >= 3) {
                        const double r1 = tex_trilinear(L + 8, L + 12, wu, wsu, wv);
                        acc = r1 + (dv == 4 ? sv * tex_bilinear(L + 16, wu, wsu) : 0.0);
                    }
                    val = r0 + sv * acc;
                }
                out[c * nq + o * n_per + q] = val;
            }
        }
}

/* ------------------------------------------------------------------ */
/* Particle ring (Sec. 5: particles moving along cubic Bezier curves chained
 * into a ring, the curve evaluated per particle per frame, beside other
 * work).  seg[N][3][4] per-segment cubic control points (closed ring).  One
 * frame per particle p:
 *   T <- T + speed * dt, wrapped into [0, N) -- FP32, operations as written;
 *   k = min(floor T, N-1), t = T - k (FP32);
 *   position by the method:
 *     0 polynomial (Bernstein), 1 Seiler terms: the cubic at (k, t) (FP64);
 *     2 emulated 8-bit Seiler texture: the segment's Table 1 texture read at
 *       (t, st) through the emulated filter (frac_bits 8, nearest);
 *     3 sampled table of S points per segment: x = T * S (FP32),
 *       i = min(floor x, N*S - 1), f = x - i, lerp of the exact samples
 *       C(i) and C(i+1) (C(j) the ring at segment j / S, local (j mod S) / S,
 *       C(N*S) = C(0));
 *   consumer (K steps of arithmetic on the position):
 *     v_0 = 0, v_{i+1} = a v_i + (b x + c y + d z)
 *     with a = 23/32, b = 1/4, c = -1/8, d = 1/16 (FP64 here).
 * Reading: the paper's consumer is a shader's other work; a fixed K-step
 * linear recurrence stands in for it (its cost scales with K).              */
static double ring_point(const double *seg, int64_t k, int c, double t)
{
    return decasteljau(seg + (k * 3 + c) * 4, 1, 3, t);
}

void bzo_particles_step(const double *seg, int64_t nseg, int method, int samples, float *T, const float *speed,
                        float dt, int64_t np, int iters, double *pos, double *shade)
{
    const double a = 23.0 / 32.0, b = 0.25, cc = -0.125, d = 0.0625;
    const int64_t ntab = nseg * samples;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np; ++p) {
        float Tn = T[p] + speed[p] * dt;
        const float nf = (float)nseg;
        if (Tn >= nf) Tn -= nf;
        if (Tn < 0.0f) Tn += nf;
        if (Tn >= nf) Tn = 0.0f; /* only if the subtraction rounded up to N */
        T[p] = Tn;
        int64_t k = (int64_t)floorf(Tn);
        if (k > nseg - 1) k = nseg - 1;
        if (k < 0) k = 0; /* only for |speed dt| >= N, outside the documented domain */
        const float t = Tn - (float)k;
        double xyz[3];
        for (int c = 0; c < 3; ++c) {
            if (method == 0 || method == 1) {
                xyz[c] = ring_point(seg, k, c, (double)t);
            } else if (method == 2) {
                double sc[4];
                seiler_coeffs(seg + (k * 3 + c) * 4, 3, sc);
                const double L[4] = {sc[0], sc[1], sc[0] + sc[2], sc[1] + sc[3]};
                const float st = (1.0f - t) * t;
                xyz[c] = tex_bilinear(L, bzo_tex_axis_weight(t, 8, 0), bzo_tex_axis_weight(st, 8, 0));
            } else {
                const float x = Tn * (float)samples;
                int64_t i = (int64_t)floorf(x);
                if (i > ntab - 1) i = ntab - 1;
                if (i < 0) i = 0;
                const float f = x - (float)i;
                const int64_t i1 = (i + 1) % ntab;
                const double c0 = ring_point(seg, i / samples, c, (double)(i % samples) / samples);
                const double c1 = ring_point(seg, i1 / samples, c, (double)(i1 % samples) / samples);
                xyz[c] = lerp(c0, c1, (double)f);
            }
            pos[c * np + p] = xyz[c];
        }
        double v = 0.0;
        const double drive = b * xyz[0] + cc * xyz[1] + d * xyz[2];
        for (int i = 0; i < iters; ++i) v = a * v + drive;
        shade[p] = v;
    }
}
