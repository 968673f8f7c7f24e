"""Pins for the FP64 oracle's curve evaluators (de Casteljau, Bernstein,
Seiler): exact rational brute force, the paper's printed Seiler formulas and
texel layouts, and the defining invariants of Bezier curves."""
import os
from fractions import Fraction
from math import comb

import numpy as np
import pytest

from tests import _exact as ex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_curves(rng, n, d, dim):
    return rng.uniform(-1, 1, size=(n, dim, d + 1)).astype(np.float32)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("form", ["decasteljau", "bernstein"])
def test_bezier_matches_exact_rational(orc, d, form):
    """Brute force: the exact Bernstein sum in rationals on float32 inputs."""
    rng = np.random.default_rng(10 + d)
    ctrl = _rand_curves(rng, 3, d, 2)
    t = np.concatenate([[0.0, 1.0, 0.5], rng.random(6)]).astype(np.float32)
    fn = orc.bezier_decasteljau if form == "decasteljau" else orc.bezier_bernstein
    out = fn(ctrl, t)
    nt = t.size
    for c in range(3):
        for k in range(2):
            b = [ex.F(x) for x in ctrl[c, k]]
            for j in range(nt):
                exact = ex.bezier(b, ex.F(t[j]))
                assert abs(Fraction(out[k, c * nt + j]) - exact) <= Fraction(8 * (d + 1), 2 ** 53)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 9, 15])
def test_endpoints_bit_exact(orc, d):
    """C(0) = b_0 and C(1) = b_d exactly, in every form."""
    rng = np.random.default_rng(20 + d)
    ctrl = _rand_curves(rng, 16, d, 3)
    t = np.array([0.0, 1.0], np.float32)
    for fn in (orc.bezier_decasteljau, orc.bezier_bernstein):
        out = fn(ctrl, t).reshape(3, 16, 2)
        np.testing.assert_array_equal(out[:, :, 0], ctrl[:, :, 0].T.astype(np.float64))
        np.testing.assert_array_equal(out[:, :, 1], ctrl[:, :, d].T.astype(np.float64))
    s = orc.seiler_eval(orc.seiler_from_bezier(ctrl), t).reshape(3, 16, 2)
    np.testing.assert_array_equal(s[:, :, 0], ctrl[:, :, 0].T.astype(np.float64))
    np.testing.assert_array_equal(s[:, :, 1], ctrl[:, :, d].T.astype(np.float64))


@pytest.mark.parametrize("d", [1, 2, 4, 7, 15])
def test_partition_of_unity(orc, d):
    """All control points equal to P gives P for every t."""
    rng = np.random.default_rng(30 + d)
    P = rng.uniform(-3, 3, size=(5, 3, 1))
    ctrl = np.repeat(P, d + 1, axis=2)
    t = rng.random(33)
    for fn in (orc.bezier_decasteljau, orc.bezier_bernstein):
        out = fn(ctrl, t).reshape(3, 5, 33)
        np.testing.assert_allclose(out, np.repeat(P[:, :, 0].T[:, :, None], 33, axis=2), rtol=0, atol=4e-15 * d)
    out = orc.seiler_eval(orc.seiler_from_bezier(ctrl), t).reshape(3, 5, 33)
    np.testing.assert_allclose(out, np.repeat(P[:, :, 0].T[:, :, None], 33, axis=2), rtol=0, atol=1e-13)


@pytest.mark.parametrize("d", [1, 3, 6, 11])
def test_linear_precision(orc, d):
    """b_i = p + (i/d)(q - p) gives p + t(q - p)."""
    rng = np.random.default_rng(40 + d)
    p, q = rng.uniform(-1, 1, size=(2, 4, 2, 1))
    ctrl = p + (np.arange(d + 1) / d) * (q - p)
    t = rng.random(17)
    expect = (p[:, :, 0].T[:, :, None] + t * (q - p)[:, :, 0].T[:, :, None]).reshape(2, -1)
    for fn in (orc.bezier_decasteljau, orc.bezier_bernstein):
        np.testing.assert_allclose(fn(ctrl, t), expect, rtol=0, atol=1e-14)
    np.testing.assert_allclose(orc.seiler_eval(orc.seiler_from_bezier(ctrl), t), expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3, 8])
def test_reversal_symmetry(orc, d):
    """C(t; b_0..b_d) = C(1-t; b_d..b_0); t on a dyadic grid so 1-t is exact."""
    rng = np.random.default_rng(50 + d)
    ctrl = _rand_curves(rng, 6, d, 3)
    t = np.arange(0, 65) / 64.0
    a = orc.bezier_decasteljau(ctrl, t)
    b = orc.bezier_decasteljau(ctrl[:, :, ::-1].copy(), 1.0 - t)
    np.testing.assert_allclose(a, b, rtol=0, atol=2e-15 * d)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 9])
def test_degree_elevation_invariance(orc, d):
    """Elevating b to degree d+1 (exactly, in rationals) leaves C unchanged."""
    rng = np.random.default_rng(60 + d)
    ctrl = _rand_curves(rng, 4, d, 2)
    elev = np.empty((4, 2, d + 2))
    for c in range(4):
        for k in range(2):
            b = [ex.F(x) for x in ctrl[c, k]]
            e = [b[0]] + [Fraction(i, d + 1) * b[i - 1] + (1 - Fraction(i, d + 1)) * b[i]
                          for i in range(1, d + 1)] + [b[d]]
            elev[c, k] = [float(x) for x in e]
    t = rng.random(25)
    np.testing.assert_allclose(orc.bezier_decasteljau(ctrl, t), orc.bezier_decasteljau(elev, t), rtol=0,
                               atol=1e-14)
    np.testing.assert_allclose(orc.seiler_eval(orc.seiler_from_bezier(elev), t),
                               orc.bezier_bernstein(ctrl, t), rtol=0, atol=1e-13)


@pytest.mark.parametrize("d", range(1, 16))
def test_three_forms_agree(orc, d):
    """de Casteljau = Bernstein = Seiler (algebraically equal forms)."""
    rng = np.random.default_rng(70 + d)
    ctrl = _rand_curves(rng, 32, d, 3)
    t = rng.random((32, 9))
    a = orc.bezier_decasteljau(ctrl, t, per_object=True)
    b = orc.bezier_bernstein(ctrl, t, per_object=True)
    s = orc.seiler_eval(orc.seiler_from_bezier(ctrl), t, per_object=True)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    np.testing.assert_allclose(a, s, rtol=0, atol=1e-11)


def _seiler_index(d):
    """Position of each named term in the stored order [b0, bd, d1, d_{d-1}, d2, ...]."""
    idx = {"B0": 0, "B%d" % d: 1}
    pos, i = 2, 1
    while pos <= d:
        idx["d%d" % i] = pos
        pos += 1
        if d - i != i and pos <= d:
            idx["d%d" % (d - i)] = pos
            pos += 1
        i += 1
    return idx


def _exact_seiler_outer(b):
    """The paper's printed difference terms (Sec. 3.1) in exact arithmetic."""
    d = len(b) - 1
    out = {1: d * (b[1] - b[0]) - (b[d] - b[0]), d - 1: d * (b[d - 1] - b[d]) - (b[0] - b[d])}
    if d >= 4:
        out[2] = (comb(d, 2) * (b[2] - b[1]) - comb(d - 2, 2) * (b[1] - b[0]) - (d - 3) * (b[d - 1] - b[d])
                  - 3 * (b[d - 1] - b[1]))
        out[d - 2] = (comb(d, 2) * (b[d - 2] - b[d - 1]) - comb(d - 2, 2) * (b[d - 1] - b[d])
                      - (d - 3) * (b[1] - b[0]) - 3 * (b[1] - b[d - 1]))
    return out


@pytest.mark.parametrize("d", range(2, 16))
def test_seiler_terms_match_paper_formulas(orc, d):
    """d_1, d_{d-1} for every degree; d_2, d_{d-2} where the paper prints them
    (degrees 4 and 5; they also hold at 6 and 7, checked here as well)."""
    rng = np.random.default_rng(80 + d)
    ctrl = _rand_curves(rng, 4, d, 1)
    sc = orc.seiler_from_bezier(ctrl)
    idx = _seiler_index(d)
    for c in range(4):
        b = [ex.F(x) for x in ctrl[c, 0]]
        terms = _exact_seiler_outer(b)
        for i, val in terms.items():
            if i in (2, d - 2) and d > 7:
                continue
            got = sc[c, 0, idx["d%d" % i]]
            assert abs(Fraction(got) - val) <= Fraction(1, 2 ** 40) * (1 + abs(val)), (d, i)
        assert sc[c, 0, 0] == ctrl[c, 0, 0] and sc[c, 0, 1] == ctrl[c, 0, d]


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_seiler_outer_recursion_is_exact(orc, d):
    """C(t) - L(b0,bd,t) = st*D_1(t) with D_1 given by the stored terms,
    checked in exact arithmetic against the Bernstein sum."""
    rng = np.random.default_rng(90 + d)
    ctrl = _rand_curves(rng, 2, d, 1)
    sc = orc.seiler_from_bezier(ctrl)
    for c in range(2):
        b = [ex.F(x) for x in ctrl[c, 0]]
        terms = [Fraction(x) for x in sc[c, 0]]
        for tj in (Fraction(1, 3), Fraction(5, 7), Fraction(1, 1024)):
            # the named terms from the stored order
            idx = _seiler_index(d)
            dd = {i: terms[idx["d%d" % i]] for i in range(1, d)}

            def D(i, t):
                if 2 * i == d + 1:
                    return Fraction(0)
                if 2 * i == d:
                    return dd[i]
                return (1 - t) * dd[i] + t * dd[d - i] + (1 - t) * t * D(i + 1, t)

            C = (1 - tj) * terms[0] + tj * terms[1] + (1 - tj) * tj * D(1, tj)
            assert abs(C - ex.bezier(b, tj)) < Fraction(1, 2 ** 44)


def _L(a, b, t):
    return (1 - t) * a + t * b


def test_seiler_cubic_pure_lerp_and_quintic_eq6(orc):
    """Cubic: L(L(b0,b3,t), L(b0+d1, b3+d2, t), st) (Sec. 4, Eq. 3-5).
    Quintic Eq. 6: L(b05, L(b05+d14, b05+d14+d23, st), st)."""
    rng = np.random.default_rng(100)
    c3 = _rand_curves(rng, 3, 3, 1)
    c5 = _rand_curves(rng, 3, 5, 1)
    s3, s5 = orc.seiler_from_bezier(c3), orc.seiler_from_bezier(c5)
    for c in range(3):
        b0, b3, d1, d2 = [Fraction(x) for x in s3[c, 0]]
        q = [Fraction(x) for x in s5[c, 0]]
        i5 = _seiler_index(5)
        B0, B5 = q[0], q[1]
        e1, e4, e2, e3 = q[i5["d1"]], q[i5["d4"]], q[i5["d2"]], q[i5["d3"]]
        for t in (Fraction(0), Fraction(1), Fraction(2, 9), Fraction(7, 8)):
            st = (1 - t) * t
            eq5 = _L(_L(b0, b3, t), _L(b0 + d1, b3 + d2, t), st)
            assert abs(eq5 - ex.bezier([ex.F(x) for x in c3[c, 0]], t)) < Fraction(1, 2 ** 45)
            b05, d14, d23 = _L(B0, B5, t), _L(e1, e4, t), _L(e2, e3, t)
            eq6 = _L(b05, _L(b05 + d14, b05 + d14 + d23, st), st)
            assert abs(eq6 - ex.bezier([ex.F(x) for x in c5[c, 0]], t)) < Fraction(1, 2 ** 44)


def _parse_table1():
    rows = {}
    with open(os.path.join(GOLDEN, "seiler_table1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            d = int(parts[0][2:])
            z = int(parts[1][2:])
            cells = dict(p.split("=") for p in parts[2:])
            rows.setdefault(d, {})[z] = cells
    return rows


def test_table1_layouts_emulated_sampling(orc):
    """Emulated bilinear (t, st) / trilinear (t, st, st) sampling of the
    Table 1 texel layouts, filled from the oracle's Seiler terms, reproduces
    the exact curve."""
    table = _parse_table1()
    assert sorted(table) == [2, 3, 4, 5]
    rng = np.random.default_rng(110)
    for d, layers in table.items():
        ctrl = _rand_curves(rng, 2, d, 1)
        sc = orc.seiler_from_bezier(ctrl)
        idx = _seiler_index(d)
        for c in range(2):
            terms = {name: Fraction(sc[c, 0, pos]) for name, pos in idx.items()}

            def cell(expr):
                return sum(terms[tok] for tok in expr.split("+"))

            for t in (Fraction(0), Fraction(1), Fraction(3, 11), Fraction(1, 2)):
                st = (1 - t) * t

                def bilinear(layer, x, y):
                    top = _L(cell(layer["TL"]), cell(layer["TR"]), x)
                    bot = _L(cell(layer["BL"]), cell(layer["BR"]), x)
                    return _L(top, bot, y)

                if len(layers) == 1:
                    val = bilinear(layers[0], t, st)
                else:
                    val = _L(bilinear(layers[0], t, st), bilinear(layers[1], t, st), st)
                exact = ex.bezier([ex.F(x) for x in ctrl[c, 0]], t)
                assert abs(val - exact) < Fraction(1, 2 ** 44), (d, t)
