"""Pins for the oracle's rational curves, NURBS (Sec. 2.2: rational = ratio
of integral splines; B-splines via conversion to Bezier segments), mixed
batches and tensor-product surfaces/volumes."""
from fractions import Fraction

import numpy as np
import pytest

import bz_synth
from tests import _exact as ex


def test_rational_equal_weights_is_integral(orc):
    rng = np.random.default_rng(1)
    for d in (1, 3, 7, 15):
        ctrl = rng.uniform(-1, 1, size=(8, 3, d + 1))
        w = np.full((8, d + 1), 2.5)
        t = rng.random((8, 11))
        np.testing.assert_allclose(orc.rational_eval(ctrl, w, t, True), orc.bezier_decasteljau(ctrl, t, True),
                                   rtol=0, atol=1e-14)


def test_rational_quarter_circle(orc):
    """(1,0),(1,1),(0,1) with weights (1, sqrt(2)/2, 1) is the unit quarter
    circle: |C(t)| = 1 for every t (closed form)."""
    ctrl = np.array([[[1.0, 1.0, 0.0], [0.0, 1.0, 1.0]]])
    w = np.array([[1.0, np.sqrt(0.5), 1.0]])
    t = np.linspace(0, 1, 257)
    out = orc.rational_eval(ctrl, w, t)
    np.testing.assert_allclose(np.hypot(out[0], out[1]), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out[:, 128], [np.sqrt(0.5), np.sqrt(0.5)], atol=1e-15)


def test_rational_exact_brute_force(orc):
    rng = np.random.default_rng(2)
    ctrl, w, t = bz_synth.rational_curves(3, 4, 2, 5, seed=3)
    out = orc.rational_eval(ctrl, w, t, True)
    for c in range(3):
        for k in range(2):
            for j in range(5):
                val = ex.rational([ex.F(x) for x in ctrl[c, k]], [ex.F(x) for x in w[c]], ex.F(t[c, j]))
                assert abs(Fraction(out[k, c * 5 + j]) - val) < Fraction(1, 2 ** 46)


def test_nurbs_single_span_is_rational_bezier(orc):
    """Knots [0,0,0,0,1,1,1,1] reduce a cubic NURBS to a rational Bezier."""
    rng = np.random.default_rng(4)
    P = rng.uniform(-1, 1, size=(3, 4))
    w = rng.uniform(0.25, 4, size=4)
    u = np.concatenate([[0.0, 1.0], rng.random(30)])
    a = orc.nurbs_eval(P, w, [0, 0, 0, 0, 1, 1, 1, 1], u)
    b = orc.rational_eval(P[None], w[None], u)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_uniform_bspline_basis_matrix(orc):
    """On uniform knots a cubic B-spline span equals the textbook uniform
    basis matrix (1/6)[[1,4,1,0],[-3,0,3,0],[3,-6,3,0],[-1,3,-3,1]]."""
    rng = np.random.default_rng(5)
    ncp = 9
    P = rng.uniform(-1, 1, size=(2, ncp))
    U = np.arange(ncp + 4, dtype=np.float64)  # unclamped uniform knots 0..12
    Mb = np.array([[1, 4, 1, 0], [-3, 0, 3, 0], [3, -6, 3, 0], [-1, 3, -3, 1]]) / 6.0
    for span in range(3, ncp):
        for x in (0.0, 0.3, 0.75):
            u = np.array([span + x])
            got = orc.nurbs_eval(P, np.ones(ncp), U, u)[:, 0]
            mono = np.array([1, x, x * x, x ** 3])
            expect = mono @ Mb @ P[:, span - 3:span + 1].T
            np.testing.assert_allclose(got, expect, rtol=0, atol=1e-14)


def test_nurbs_matches_cox_de_boor_exact(orc):
    """Rational de Boor agrees with the exact Cox-de Boor basis sum."""
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=3, dim=2, n_t=4, knots_lo=10, knots_hi=12, seed=6)
    for o in range(3):
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        ncp = a1 - a0
        P = b.ctrl[a0 * 2:a1 * 2].reshape(2, ncp)
        w = b.w[a0:a1]
        U = b.knots[b.knot_offset[o]:b.knot_offset[o + 1]]
        u = b.t[o]
        got = orc.nurbs_eval(P, w, U, u)
        Uf = [ex.F(x) for x in U]
        for j in range(4):
            val = ex.nurbs([[ex.F(x) for x in P[k]] for k in range(2)], [ex.F(x) for x in w], Uf, 3, ex.F(u[j]))
            for k in range(2):
                assert abs(Fraction(got[k, j]) - val[k]) < Fraction(1, 2 ** 40)


def test_nurbs_partition_of_unity_and_ends(orc):
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=1, dim=3, n_t=4, seed=7)
    ncp = b.cp_offset[1]
    U = b.knots
    w = b.w
    P = np.ones((3, ncp)) * np.array([[0.5], [-2.0], [3.0]])
    u = np.linspace(0, 1, 101)
    np.testing.assert_allclose(orc.nurbs_eval(P, w, U, u), np.repeat(P[:, :1], 101, axis=1), rtol=0, atol=1e-14)
    P = b.ctrl.reshape(3, ncp).astype(np.float64)
    ends = orc.nurbs_eval(P, w, U, np.array([0.0, 1.0]))
    np.testing.assert_allclose(ends[:, 0], P[:, 0], atol=1e-15)
    np.testing.assert_allclose(ends[:, 1], P[:, -1], atol=1e-15)


def _boehm_segments(P, w, U, p=3):
    """Independent pure-Python Boehm knot insertion to full multiplicity,
    returning rational Bezier segments (homogeneous) and their intervals."""
    H = [list(np.append(w[i] * P[:, i], w[i])) for i in range(len(w))]
    U = list(U)
    for x in sorted(set(U[p + 1:len(U) - p - 1])):
        while U.count(x) < p:
            k = max(i for i in range(len(U) - 1) if U[i] <= x < U[i + 1])
            s = U.count(x)
            newH = []
            for i in range(len(H) + 1):
                if i <= k - p:
                    newH.append(H[i])
                elif i >= k - s + 1:
                    newH.append(H[i - 1])
                else:
                    a = (x - U[i]) / (U[i + p] - U[i])
                    newH.append([(1 - a) * H[i - 1][c] + a * H[i][c] for c in range(len(H[0]))])
            H = newH
            U.insert(k + 1, x)
    brk = sorted(set(U))
    segs = [(brk[i], brk[i + 1], H[3 * i:3 * i + 4]) for i in range(len(brk) - 1)]
    return segs


def test_de_boor_equals_boehm_bezier(orc):
    """De Boor (oracle) = Boehm knot insertion + rational Bezier per span."""
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=4, dim=3, n_t=16, knots_lo=8, knots_hi=20, seed=8)
    for o in range(4):
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        ncp = a1 - a0
        P = b.ctrl[a0 * 3:a1 * 3].reshape(3, ncp).astype(np.float64)
        w = b.w[a0:a1].astype(np.float64)
        U = b.knots[b.knot_offset[o]:b.knot_offset[o + 1]].astype(np.float64)
        segs = _boehm_segments(P, w, U)
        u = b.t[o].astype(np.float64)
        got = orc.nurbs_eval(P, w, U, u)
        for j, uj in enumerate(u):
            lo, hi, H = next(s for s in segs if s[0] <= uj < s[1])
            tl = (uj - lo) / (hi - lo)
            Hn = np.array(H)
            ctrl = (Hn[:, :3] / Hn[:, 3:]).T[None]
            val = orc.rational_eval(ctrl, Hn[:, 3][None], np.array([tl]))[:, 0]
            np.testing.assert_allclose(got[:, j], val, rtol=0, atol=1e-12)


def test_batch_dispatches_each_kind(orc):
    b = bz_synth.mixed_batch(n_bezier=40, n_nurbs=10, dim=3, n_t=5, seed=9)
    out = orc.batch_eval(b)
    nq = b.n_obj * 5
    for o in range(b.n_obj):
        kind, d = b.kind_degree[o] >> 8, b.kind_degree[o] & 0xff
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        ncp = a1 - a0
        P = b.ctrl[a0 * 3:a1 * 3].reshape(3, ncp)
        w = b.w[a0:a1]
        if kind == 0:
            ref = orc.bezier_bernstein(P[None], b.t[o])
            assert np.all(w == 1.0)
        elif kind == 1:
            ref = orc.rational_eval(P[None], w[None], b.t[o])
        else:
            ref = orc.nurbs_eval(P, w, b.knots[b.knot_offset[o]:b.knot_offset[o + 1]], b.t[o])
        np.testing.assert_allclose(out[:, o * 5:(o + 1) * 5], ref, rtol=0, atol=1e-13)
    assert out.shape == (3, nq)


# ------------------------------------------------------------- tensor
def test_bilinear_trilinear_reduction(orc):
    """Degree (1,1) and (1,1,1) reduce to bi- and trilinear interpolation."""
    rng = np.random.default_rng(10)
    P = rng.uniform(-1, 1, size=(4, 2, 4))
    uv = rng.random((4, 7, 2))
    got = orc.tensor_points(P, 1, 1, 0, uv)
    u, v = uv[..., 0], uv[..., 1]
    for k in range(2):
        p = P[:, k]
        ref = ((1 - u) * (1 - v) * p[:, :1] + (1 - u) * v * p[:, 1:2] + u * (1 - v) * p[:, 2:3] + u * v * p[:, 3:4])
        np.testing.assert_allclose(got[k], ref.reshape(-1), atol=1e-15)
    P = rng.uniform(-1, 1, size=(3, 1, 8))
    uvw = rng.random((3, 5, 3))
    got = orc.tensor_points(P, 1, 1, 1, uvw)[0].reshape(3, 5)
    u, v, w = uvw[..., 0], uvw[..., 1], uvw[..., 2]
    ref = np.zeros((3, 5))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                ref += (u if i else 1 - u) * (v if j else 1 - v) * (w if k else 1 - w) * P[:, 0, (i * 2 + j) * 2 + k, None]
    np.testing.assert_allclose(got, ref, atol=1e-15)


@pytest.mark.parametrize("degs", [(3, 3, 0), (2, 4, 0), (3, 3, 3), (1, 2, 3)])
def test_tensor_matches_exact_triple_sum(orc, degs):
    du, dv, dw = degs
    ncp = (du + 1) * (dv + 1) * (dw + 1)
    rng = np.random.default_rng(11)
    P = rng.uniform(-1, 1, size=(2, 2, ncp)).astype(np.float32)
    npar = 3 if dw else 2
    uvw = rng.random((2, 3, npar)).astype(np.float32)
    got = orc.tensor_points(P, du, dv, dw, uvw)
    for o in range(2):
        for j in range(3):
            w = ex.F(uvw[o, j, 2]) if dw else Fraction(0)
            for k in range(2):
                val = ex.tensor([ex.F(x) for x in P[o, k]], du, dv, dw, ex.F(uvw[o, j, 0]), ex.F(uvw[o, j, 1]), w)
                assert abs(Fraction(got[k, o * 3 + j]) - val) < Fraction(1, 2 ** 46)


def test_grid_mode_equals_points_mode(orc):
    P = bz_synth.patches(n_obj=5, seed=12).astype(np.float64)
    nu, nv = 6, 5
    g = orc.tensor_grid(P, 3, 3, nu, nv)
    a, b = np.meshgrid(np.arange(nu) / (nu - 1), np.arange(nv) / (nv - 1), indexing="ij")
    uv = np.repeat(np.stack([a.ravel(), b.ravel()], axis=1)[None], 5, axis=0)
    np.testing.assert_allclose(g, orc.tensor_points(P, 3, 3, 0, uv), rtol=0, atol=1e-15)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 3), (2, 4)])
def test_patch_diagonal_is_degree_sum_curve(orc, m, n):
    """S(t,t) of a degree-(m,n) patch is the degree-(m+n) curve with
    c_k = sum_{i+j=k} C(m,i)C(n,j)/C(m+n,k) P_ij (generalises Sec. 2.2's
    order split M + N = O)."""
    from math import comb
    rng = np.random.default_rng(13)
    P = rng.uniform(-1, 1, size=(3, 2, (m + 1) * (n + 1)))
    c = np.zeros((3, 2, m + n + 1))
    for i in range(m + 1):
        for j in range(n + 1):
            c[:, :, i + j] += comb(m, i) * comb(n, j) / comb(m + n, i + j) * P[:, :, i * (n + 1) + j]
    t = rng.random(20)
    uv = np.repeat(np.stack([t, t], axis=1)[None], 3, axis=0)
    np.testing.assert_allclose(orc.tensor_points(P, m, n, 0, uv), orc.bezier_decasteljau(c, t), atol=1e-14)


def test_volume_corners_exact(orc):
    ctrl, _ = bz_synth.volumes(n_obj=3, n_q=3 * 8, seed=14)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], np.float64)
    uvw = np.repeat(corners[None], 3, axis=0)
    got = orc.tensor_points(ctrl, 3, 3, 3, uvw).reshape(3, 3, 8)
    for o in range(3):
        for idx, (i, j, k) in enumerate(corners.astype(int)):
            np.testing.assert_array_equal(got[:, o, idx], ctrl[o, :, (i * 3 * 4 + j * 3) * 4 + k * 3])


def test_batch_patches_exact_brute_force(orc):
    """Surface patches inside a mixed batch (kind 3, degree byte du<<4 | dv,
    Sec. 2.2): every point equals the exact tensor-product Bernstein double
    sum of its net at its (u, v), for bilinear to bicubic patches and mixed
    degrees, with curves and NURBS around them."""
    from tests._exact import F, tensor
    b = bz_synth.mixed_batch(n_bezier=30, n_nurbs=6, n_patches=40, n_t=3, patch_deg_lo=1, patch_deg_hi=3, seed=21)
    out = orc.batch_eval(b)
    kinds = b.kind_degree >> 8
    assert (kinds == 3).sum() == 40 and len(set((b.kind_degree[kinds == 3] & 0xff).tolist())) > 4
    for o in np.nonzero(kinds == 3)[0]:
        du, dv = int(b.kind_degree[o] & 0xff) >> 4, int(b.kind_degree[o] & 15)
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        assert a1 - a0 == (du + 1) * (dv + 1)
        P = b.ctrl[a0 * 3:a1 * 3].reshape(3, -1)
        for j in range(3):
            u, v = F(b.t[o, j]), F(b.v[o, j])
            for k in range(3):
                want = tensor([F(x) for x in P[k]], du, dv, 0, u, v, 0)
                assert abs(out[k, o * 3 + j] - float(want)) <= 1e-15 * max(1.0, abs(float(want)))


def test_batch_bilinear_patch_closed_form(orc):
    """A (1,1) patch in a batch is the bilinear interpolation of its corners,
    (1-u)(1-v)P00 + (1-u)v P01 + u(1-v)P10 + uv P11."""
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=0, n_patches=25, n_t=7, patch_deg_lo=1, patch_deg_hi=1, seed=22)
    out = orc.batch_eval(b).reshape(3, 25, 7)
    for o in range(25):
        P = b.ctrl[b.cp_offset[o] * 3:b.cp_offset[o + 1] * 3].reshape(3, 2, 2).astype(np.float64)
        u, v = b.t[o].astype(np.float64), b.v[o].astype(np.float64)
        want = ((1 - u) * (1 - v))[None] * P[:, 0, 0, None] + ((1 - u) * v)[None] * P[:, 0, 1, None] + \
            (u * (1 - v))[None] * P[:, 1, 0, None] + (u * v)[None] * P[:, 1, 1, None]
        np.testing.assert_allclose(out[:, o], want, rtol=0, atol=1e-15)


def test_batch_without_patches_is_unchanged_by_the_second_parameters(orc):
    """Curves and NURBS do not read v."""
    b = bz_synth.mixed_batch(n_bezier=50, n_nurbs=8, n_t=4, seed=23)
    ref = orc.batch_eval(b)
    b.v = np.full_like(b.t, np.nan)
    np.testing.assert_array_equal(orc.batch_eval(b), ref)
