"""Pins for the oracle's texture-filter emulation: filter weights on a
two-texel axis after the texel-centre remap, rounded to F fractional bits
(Sec. 2, Sec. 2.3), the de Casteljau / hybrid / Seiler curve textures
(Sec. 2, Sec. 4 with Table 1, Fig. 3) and the zig-zag chain read by the
emulated bilinear filter (Sec. 2.1)."""
import numpy as np
import pytest

import bz_synth
from tests.test_oracle_curves import _parse_table1, _seiler_index

def _curves(n, d, dim, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, dim, d + 1)).astype(np.float32)


def _ext(ctrl):
    c = np.asarray(ctrl, np.float64)
    return max(float((c.max(axis=2) - c.min(axis=2)).max()), float(np.abs(c).max()))


# ------------------------------------------------------------ axis weights
@pytest.mark.parametrize("F", [4, 8, 12])
@pytest.mark.parametrize("rounding", ["nearest", "truncate"])
def test_weights_on_the_fixed_point_grid_are_exact(orc, F, rounding):
    """A parameter that is a multiple of 2^-F passes the remap and the
    rounding unchanged; 0 and 1 are the edge texels."""
    p = np.arange(2 ** F + 1, dtype=np.float64) / 2 ** F
    w = orc.tex_axis_weights(p.astype(np.float32), F, rounding)
    np.testing.assert_array_equal(w, p)


def test_weight_rounding_rules(orc):
    """Halfway between grid points: nearest goes up, truncation down; a
    quarter past a grid point goes down for both."""
    j = np.arange(255, dtype=np.float64)
    half = ((j + 0.5) / 256).astype(np.float32)
    quarter = ((j + 0.25) / 256).astype(np.float32)
    np.testing.assert_array_equal(orc.tex_axis_weights(half, 8, "nearest"), (j + 1) / 256)
    np.testing.assert_array_equal(orc.tex_axis_weights(half, 8, "truncate"), j / 256)
    np.testing.assert_array_equal(orc.tex_axis_weights(quarter, 8, "nearest"), j / 256)
    np.testing.assert_array_equal(orc.tex_axis_weights(quarter, 8, "truncate"), j / 256)


def test_weight_bounds_clamp_and_monotone(orc):
    """|w - p| <= 2^-9 (nearest) and 0 <= p - w < 2^-8 (truncation), up to
    the 2^-24 the FP32 remap may move p; F = 0 leaves only that; weights are
    non-decreasing in p; outside [0,1] the edge texel is taken; NaN stays."""
    rng = np.random.default_rng(300)
    p = np.sort(rng.random(20000)).astype(np.float32)
    pd = p.astype(np.float64)
    wn = orc.tex_axis_weights(p, 8, "nearest")
    wt = orc.tex_axis_weights(p, 8, "truncate")
    w0 = orc.tex_axis_weights(p, 0, "nearest")
    assert np.abs(wn - pd).max() <= 2 ** -9 + 2 ** -24
    assert (pd - wt).min() >= -2 ** -24 and (pd - wt).max() < 2 ** -8 + 2 ** -24
    assert np.abs(w0 - pd).max() <= 2 ** -24
    for w in (wn, wt, w0):
        assert (np.diff(w) >= 0).all()
    edge = orc.tex_axis_weights(np.array([-3.0, -0.0, 1.0, 7.0, np.inf, -np.inf, np.nan], np.float32), 8)
    np.testing.assert_array_equal(edge[:6], [0.0, 0.0, 1.0, 1.0, 1.0, 0.0])
    assert np.isnan(edge[6])
    # the quantised weights take only the 257 values k/256
    assert set(np.unique(wn * 256)) <= set(range(257))


# ------------------------------------------------------------ curve textures
def test_texel_counts(orc):
    assert [orc.tex_texels(d, "decasteljau") for d in (2, 3, 4, 7)] == [4, 8, 12, 24]
    assert [orc.tex_texels(d, "seiler") for d in (2, 3, 4, 5, 6, 7)] == [4, 4, 8, 8, 8, 8]


def test_decasteljau_layers_are_the_quadratic_textures(orc):
    """Layer i holds [[b_i, b_i+1], [b_i+1, b_i+2]] (Sec. 2): the 2x2 texture
    whose bilinear read at (t,t) is the quadratic's de Casteljau point."""
    ctrl = _curves(3, 6, 2, 301)
    tex = orc.tex_build(ctrl, "decasteljau")
    for i in range(5):
        np.testing.assert_array_equal(tex[:, :, 4 * i + 0], ctrl[:, :, i])
        np.testing.assert_array_equal(tex[:, :, 4 * i + 1], ctrl[:, :, i + 1])
        np.testing.assert_array_equal(tex[:, :, 4 * i + 2], ctrl[:, :, i + 1])
        np.testing.assert_array_equal(tex[:, :, 4 * i + 3], ctrl[:, :, i + 2])
    np.testing.assert_array_equal(orc.tex_build(ctrl, "hybrid"), tex)


def test_seiler_textures_match_table1(orc):
    """The Seiler textures are the Table 1 layouts (tests/golden), cell by
    cell, filled with the oracle's difference terms."""
    table = _parse_table1()
    for d, layers in table.items():
        ctrl = _curves(4, d, 3, 310 + d)
        tex = orc.tex_build(ctrl, "seiler")
        sc = orc.seiler_from_bezier(ctrl)
        idx = _seiler_index(d)
        for z, cells in layers.items():
            for pos, name in enumerate(("TL", "TR", "BL", "BR")):
                want = sum(sc[:, :, idx[tok]] for tok in cells[name].split("+"))
                np.testing.assert_allclose(tex[:, :, 4 * z + pos], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("mode,degs", [("decasteljau", range(2, 9)), ("hybrid", range(2, 9)),
                                       ("seiler", range(2, 8))])
def test_unrounded_weights_give_the_curve(orc, mode, degs):
    """F = 0: every mode reads the curve itself (texels rounded once to
    FP32; the remap moves p by at most 2^-24)."""
    rng = np.random.default_rng(320)
    t = np.concatenate([[0.0, 1.0, 0.5], rng.random(200)]).astype(np.float32)
    for d in degs:
        ctrl = _curves(20, d, 3, 330 + d)
        tex = orc.tex_build(ctrl, mode).astype(np.float32)
        got = orc.tex_eval(tex, d, mode, t, frac_bits=0)
        ref = orc.bezier_decasteljau(ctrl, t)
        assert np.abs(got - ref).max() <= 2e-6 * _ext(ctrl) * d, (mode, d)


@pytest.mark.parametrize("mode", ["decasteljau", "hybrid", "seiler"])
@pytest.mark.parametrize("rounding", ["nearest", "truncate"])
def test_parameters_on_the_grid_are_exact(orc, mode, rounding):
    """Where t and st are both multiples of 2^-8 no weight is rounded, so
    every mode (cubic, the Fig. 3 case) returns the curve, endpoints
    bit-exactly."""
    t = np.array([0.0, 1.0, 0.5, 0.25, 0.75, 0.125, 0.875, 1 / 16, 15 / 16], np.float32)
    st = (1 - t.astype(np.float64)) * t
    assert ((st * 256) % 1 == 0).all()
    ctrl = _curves(30, 3, 3, 340)
    tex = orc.tex_build(ctrl, mode).astype(np.float32)
    got = orc.tex_eval(tex, 3, mode, t, frac_bits=8, rounding=rounding)
    ref = orc.bezier_decasteljau(ctrl, t)
    assert np.abs(got - ref).max() <= 2e-6 * _ext(ctrl)
    if mode != "seiler":  # de Casteljau texels are the control points themselves
        g = got.reshape(3, 30, -1)
        np.testing.assert_array_equal(g[:, :, 0], ctrl[:, :, 0].T)
        np.testing.assert_array_equal(g[:, :, 1], ctrl[:, :, 3].T)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("rounding", ["nearest", "truncate"])
def test_trilinear_mode_is_the_curve_at_the_rounded_parameter(orc, d, rounding):
    """With one weight w on every axis, the bilinear (d = 2) / trilinear
    (d = 3) read of the de Casteljau texture is the curve at w (Fig. 3's
    single-read mode): its error is the curve's motion over w - t."""
    rng = np.random.default_rng(350 + d)
    ctrl = _curves(40, d, 3, 360 + d)
    t = rng.random(300).astype(np.float32)
    tex = orc.tex_build(ctrl, "decasteljau").astype(np.float32)
    got = orc.tex_eval(tex, d, "decasteljau", t, frac_bits=8, rounding=rounding)
    w = orc.tex_axis_weights(t, 8, rounding)
    ref = orc.bezier_decasteljau(ctrl, w)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_hybrid_mode_is_the_lerp_of_two_rounded_quadratics(orc):
    """Hybrid cubic (Fig. 3): two bilinear reads give the quadratics (b0, b1,
    b2) and (b1, b2, b3) at the rounded weight w, the shader lerps them with
    the exact t."""
    rng = np.random.default_rng(370)
    ctrl = _curves(40, 3, 2, 371)
    t = rng.random(300).astype(np.float32)
    tex = orc.tex_build(ctrl, "hybrid").astype(np.float32)
    got = orc.tex_eval(tex, 3, "hybrid", t, frac_bits=8)
    w = orc.tex_axis_weights(t, 8)
    q0 = orc.bezier_decasteljau(np.ascontiguousarray(ctrl[:, :, 0:3]), w).reshape(2, 40, -1)
    q1 = orc.bezier_decasteljau(np.ascontiguousarray(ctrl[:, :, 1:4]), w).reshape(2, 40, -1)
    td = t.astype(np.float64)
    ref = ((1 - td) * q0 + td * q1).reshape(2, -1)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


def test_seiler_mode_error_bound(orc):
    """Seiler cubic read at rounded (t, st): the value L(b0,b3,a) + b L(d1,d2,a)
    moves by at most (|b3-b0| + |d2-d1|/4)|a-t| + max(|d1|,|d2|)|b-st|, with
    |a-t|, |b-st| <= 2^-9 + 2^-24 (nearest)."""
    rng = np.random.default_rng(380)
    ctrl = _curves(200, 3, 1, 381)
    t = rng.random(64).astype(np.float32)
    tex = orc.tex_build(ctrl, "seiler").astype(np.float32)
    got = orc.tex_eval(tex, 3, "seiler", t, frac_bits=8).reshape(200, 64)
    ref = orc.bezier_decasteljau(ctrl, t).reshape(200, 64)
    sc = orc.seiler_from_bezier(ctrl)[:, 0]
    e = 2 ** -9 + 2 ** -24
    bound = (np.abs(sc[:, 1] - sc[:, 0]) + np.abs(sc[:, 3] - sc[:, 2]) / 4) * e + \
        np.maximum(np.abs(sc[:, 2]), np.abs(sc[:, 3])) * e
    assert (np.abs(got - ref).max(axis=1) <= bound * (1 + 1e-6) + 1e-6).all()
    # and the rounding is visible: not the exact curve
    assert np.abs(got - ref).max() > 1e-4


def test_texture_clamps_the_parameter(orc):
    ctrl = _curves(5, 3, 2, 390)
    t = np.array([-2.0, 0.0, 1.0, 3.0, np.nan], np.float32)
    for mode in ("decasteljau", "hybrid", "seiler"):
        got = orc.tex_eval(orc.tex_build(ctrl, mode).astype(np.float32), 3, mode, t).reshape(2, 5, 5)
        np.testing.assert_allclose(got[:, :, 0], got[:, :, 1], rtol=0, atol=1e-7)
        np.testing.assert_allclose(got[:, :, 3], got[:, :, 2], rtol=0, atol=1e-7)
        assert np.isnan(got[:, :, 4]).all()


# ------------------------------------------------------------ chain
def _chain_grid(orc, n_seg, dim=3, seed=400):
    chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=seed)
    return chain, orc.piecewise_encode(chain).astype(np.float32)


def test_chain_unrounded_weights_give_the_chain(orc):
    chain, grid = _chain_grid(orc, 300)
    rng = np.random.default_rng(401)
    T = np.concatenate([rng.uniform(0, 300, 5000), np.arange(301.0), [-4.0, 310.0]]).astype(np.float32)
    got = orc.chain_texemu_eval(grid, T, frac_bits=0)
    ref = orc.chain_eval(chain, T)
    ext = float((chain.max(axis=0) - chain.min(axis=0)).max())
    assert np.abs(got - ref).max() <= 1e-6 * ext


@pytest.mark.parametrize("rounding", ["nearest", "truncate"])
def test_chain_dyadic_parameters_are_exact(orc, rounding):
    """T = k + j/256: no weight is rounded; integer T hits the shared
    endpoints exactly (C0 through the filter too)."""
    chain, grid = _chain_grid(orc, 64)
    k = np.repeat(np.arange(64), 9)
    j = np.tile([0, 1, 37, 128, 200, 255, 64, 3, 250], 64)
    T = (k + j / 256).astype(np.float32)
    got = orc.chain_texemu_eval(grid, T, 8, rounding)
    np.testing.assert_allclose(got, orc.chain_eval(chain, T), rtol=0, atol=1e-6)
    ends = orc.chain_texemu_eval(grid, np.arange(65, dtype=np.float32), 8, rounding)
    np.testing.assert_array_equal(ends.T, chain[0::2])


def test_chain_ties_read_off_the_diagonal(orc):
    """At a tie t = (j + 1/2)/256 on a segment that starts in row 1, nearest
    rounding sends x up to (j+1)/256 and the row weight 1 - t up to
    (256-j)/256: the filter reads the bilinear patch of the segment's four
    texels at (u, v) = ((j+1)/256, (256-j)/256), off its diagonal -- checked
    against the oracle's tensor-product patch."""
    chain, grid = _chain_grid(orc, 16)
    ks, js = [1, 3, 5, 7], [0, 10, 100, 254]
    T = np.array([k + (j + 0.5) / 256 for k in ks for j in js], np.float32)
    got = orc.chain_texemu_eval(grid, T, 8, "nearest")
    P = []
    uv = []
    for k in ks:
        for j in js:
            # P_ij = texel (column k + i, row j): u along columns, v along rows
            P.append(np.stack([grid[k, 0], grid[k, 1], grid[k + 1, 0], grid[k + 1, 1]], axis=1))
            uv.append([[(j + 1) / 256, (256 - j) / 256]])
    ref = orc.tensor_points(np.array(P), 1, 1, 0, np.array(uv))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)
    # and that is not the chain at any rounded parameter on the diagonal
    diag = orc.chain_eval(chain, np.array([k + (j + 1) / 256 for k in ks for j in js], np.float32))
    assert np.abs(got - diag).max() > 1e-7


def test_chain_error_bound(orc):
    """Nearest rounding away from ties: both weights round to the same w, the
    read stays on the diagonal and |err| <= 2^-9 max|C'| + O(2^-24), C' of
    segment k bounded by 2 max(|M_k - A_k|, |A_k+1 - M_k|).  At ties (common:
    an FP32 T near 200 has 17 fractional bits) an odd segment is read off its
    diagonal and the error grows with the free texels."""
    chain, grid = _chain_grid(orc, 200)
    rng = np.random.default_rng(402)
    T = rng.uniform(0, 200, 20000).astype(np.float32)
    Td = T.astype(np.float64)
    tie = ((Td - np.floor(Td)) * 256) % 1 == 0.5
    assert 10 < tie.sum() < 400
    got = orc.chain_texemu_eval(grid, T, 8, "nearest")
    ref = orc.chain_eval(chain, T)
    err = np.abs(got - ref).max(axis=0)
    c = chain.astype(np.float64)
    dmax = 2 * np.abs(np.diff(c, axis=0)).max()
    assert err[~tie].max() <= dmax * (2 ** -9 + 2 ** -23) + 1e-6
    assert err[~tie].max() > 1e-6
    odd = (np.floor(Td).astype(np.int64) & 1) == 1
    assert err[tie & ~odd].max() <= dmax * (2 ** -9 + 2 ** -23) + 1e-6
    assert err[tie & odd].max() > err[~tie].max()


def test_hybrid_error_is_two_thirds_of_trilinear_error(orc):
    """To first order in d = w - t the trilinear read errs by C'(t) d and the
    hybrid read by ((1-t) Q0'(t) + t Q1'(t)) d = (2/3) C'(t) d (the Bernstein
    derivative of the cubic is 3 sum B_i^2 (b_i+1 - b_i), that of the lerped
    quadratics 2 sum B_i^2 (b_i+1 - b_i)); the rest is O(d^2) with
    |C''| <= 6 max|b_i+2 - 2 b_i+1 + b_i|."""
    rng = np.random.default_rng(390)
    ctrl = _curves(300, 3, 1, 391)
    t = rng.random(128).astype(np.float32)
    ref = orc.bezier_decasteljau(ctrl, t)
    e_dc = orc.tex_eval(orc.tex_build(ctrl, "decasteljau").astype(np.float32), 3, "decasteljau", t) - ref
    e_hy = orc.tex_eval(orc.tex_build(ctrl, "hybrid").astype(np.float32), 3, "hybrid", t) - ref
    c = ctrl[:, 0].astype(np.float64)
    d2 = np.abs(c[:, 2:] - 2 * c[:, 1:-1] + c[:, :-2]).max(axis=1)
    d = 2.0 ** -9 + 2.0 ** -24
    slack = (6 * d2 * d * d)[:, None] + 1e-12
    assert (np.abs(e_hy - 2.0 / 3.0 * e_dc).reshape(300, 128) <= slack).all()
    assert np.abs(e_dc).max() > 1e-4


# ------------------------------------------------------------ degree 7 in 2x2x2
def _poly_mul(a, b):
    return np.convolve(a, b)


def _trilinear_span_rank(y, z):
    """Rank of {1, x, y, z, xy, xz, yz, xyz} with x = t as integer
    polynomials in t (coefficient vectors, degree <= 9)."""
    x = np.array([0, 1])
    one = np.array([1])
    prods = [one, x, y, z, _poly_mul(x, y), _poly_mul(x, z), _poly_mul(y, z), _poly_mul(_poly_mul(x, y), z)]
    M = np.zeros((8, 10))
    for r, p in enumerate(prods):
        M[r, :len(p)] = p
    return np.linalg.matrix_rank(M), max(len(p) for p in prods) - 1


def test_conjecture_by_dimension_count():
    """A 2x2x2 read at (t, st, st) (the layout of degrees 4 and 5) spans only
    the polynomials of degree <= 5 -- two of its eight products coincide --
    while (t, st, (st)^2) spans all polynomials of degree <= 7: eight texels
    for eight control points, as the conclusion anticipates."""
    st = np.array([0, 1, -1])  # t - t^2
    st2 = _poly_mul(st, st)
    assert _trilinear_span_rank(st, st) == (6, 5)
    assert _trilinear_span_rank(st, st2) == (8, 7)


@pytest.mark.parametrize("d", [6, 7])
def test_degree_6_7_layout_exact(orc, d):
    """The 2x2x2 Seiler layout read at (t, st, (st)^2) in exact rational
    arithmetic equals the curve's Bernstein sum."""
    from fractions import Fraction
    from tests import _exact as ex
    ctrl = _curves(3, d, 1, 395 + d)
    tex = orc.tex_build(ctrl, "seiler")
    for c in range(3):
        T = [Fraction(v) for v in tex[c, 0]]
        b = [ex.F(v) for v in ctrl[c, 0]]
        for t in (Fraction(0), Fraction(1), Fraction(1, 3), Fraction(5, 7), Fraction(1, 2)):
            y, z = (1 - t) * t, ((1 - t) * t) ** 2

            def lx(a, bb):
                return (1 - t) * a + t * bb
            v = (1 - z) * ((1 - y) * lx(T[0], T[1]) + y * lx(T[2], T[3])) + \
                z * ((1 - y) * lx(T[4], T[5]) + y * lx(T[6], T[7]))
            assert abs(v - ex.bezier(b, t)) < Fraction(1, 2 ** 40)


# ------------------------------------------------------------ surfaces
PATCH_CASES = [(du, dv) for du in (2, 3) for dv in (1, 2, 3, 4)]


def _patches(n, du, dv, dim, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, dim, (du + 1) * (dv + 1))).astype(np.float32)


def test_patch_texel_counts(orc):
    assert orc.tex_patch_texels(3, 3, "decasteljau") == 32 and orc.tex_patch_texels(3, 3, "seiler") == 16
    assert orc.tex_patch_texels(2, 4, "decasteljau") == 20 and orc.tex_patch_texels(2, 1, "seiler") == 8


@pytest.mark.parametrize("du,dv", PATCH_CASES)
@pytest.mark.parametrize("mode", ["decasteljau", "seiler"])
def test_patch_unrounded_weights_give_the_surface(orc, du, dv, mode):
    """F = 0: both surface textures read the tensor-product surface itself
    (the separable oracle, pinned on its own)."""
    rng = np.random.default_rng(700 + 10 * du + dv)
    P = _patches(11, du, dv, 3, 710 + du + dv)
    uv = rng.random((11, 50, 2)).astype(np.float32)
    uv[:, :4] = [[0, 0], [1, 1], [0, 1], [1, 0]]
    tex = orc.tex_patch_build(P, du, dv, mode).astype(np.float32)
    got = orc.tex_patch_eval(tex, du, dv, mode, uv, frac_bits=0)
    ref = orc.tensor_points(P, du, dv, 0, uv)
    assert np.abs(got - ref).max() <= 4e-6 * _ext(P)


@pytest.mark.parametrize("du,dv", PATCH_CASES)
def test_patch_decasteljau_is_the_surface_at_the_rounded_u(orc, du, dv):
    """De Casteljau surface textures round only u (all of the u reads share
    one weight w); v is the shader's: the result is S(w(u), v) exactly."""
    rng = np.random.default_rng(720 + 10 * du + dv)
    P = _patches(9, du, dv, 2, 730 + du + dv)
    uv = rng.random((9, 40, 2)).astype(np.float32)
    tex = orc.tex_patch_build(P, du, dv, "decasteljau").astype(np.float32)
    got = orc.tex_patch_eval(tex, du, dv, "decasteljau", uv, 8, "nearest")
    w = orc.tex_axis_weights(uv[:, :, 0].ravel(), 8).reshape(9, 40)
    ref = orc.tensor_points(P, du, dv, 0, np.stack([w, uv[:, :, 1].astype(np.float64)], axis=-1))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("du,dv", PATCH_CASES)
def test_patch_seiler_dyadic_parameters_are_exact(orc, du, dv):
    """Seiler surface textures round u, su and v: where all three are on the
    8-bit grid the read is the surface."""
    us = np.array([0.0, 1.0, 0.5, 0.25, 0.75, 0.125, 1 / 16], np.float64)
    vs = np.array([0.0, 1.0, 0.5, 37 / 256, 200 / 256], np.float64)
    assert (((1 - us) * us * 256) % 1 == 0).all()
    uv = np.array([[[u, v] for u in us for v in vs]] * 6, np.float32)
    P = _patches(6, du, dv, 3, 740 + du + dv)
    tex = orc.tex_patch_build(P, du, dv, "seiler").astype(np.float32)
    got = orc.tex_patch_eval(tex, du, dv, "seiler", uv, 8, "nearest")
    ref = orc.tensor_points(P, du, dv, 0, uv)
    assert np.abs(got - ref).max() <= 4e-6 * _ext(P)
    # elsewhere the rounding shows
    uv2 = np.random.default_rng(750).random((6, 64, 2)).astype(np.float32)
    e = np.abs(orc.tex_patch_eval(tex, du, dv, "seiler", uv2, 8) - orc.tensor_points(P, du, dv, 0, uv2)).max()
    assert 1e-5 < e < 0.1 * _ext(P)
