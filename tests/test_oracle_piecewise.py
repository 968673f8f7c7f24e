"""Pins for the oracle's C0 piecewise quadratic chain with the shared
diagonal (zig-zag) encoding (Sec. 2.1, Eq. 1-2, Fig. 2)."""
from fractions import Fraction

import numpy as np
import pytest

import bz_synth
from tests import _exact as ex


def _chain(n_seg, dim=3, seed=5):
    chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=seed)
    return chain


def test_bilinear_expansion_eq1_eq2():
    """(As+Bt)s + (Cs+Dt)t = As^2 + (B+C)st + Dt^2 (Eq. 1), equal to
    As^2 + 2Est + Dt^2 (Eq. 2) iff E = (B+C)/2, checked in exact arithmetic."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        A, B, C, D = (ex.F(x) for x in rng.uniform(-5, 5, 4))
        for t in (Fraction(0), Fraction(1), Fraction(1, 3), Fraction(7, 10)):
            s = 1 - t
            lhs = (A * s + B * t) * s + (C * s + D * t) * t
            assert lhs == A * s * s + (B + C) * s * t + D * t * t
            E = (B + C) / 2
            assert lhs == A * s * s + 2 * E * s * t + D * t * t
            if 0 < t < 1:
                assert lhs != A * s * s + 2 * (E + 1) * s * t + D * t * t


def test_storage_count():
    """N chained quadratics occupy 2(N+1) texels, e.g. 3 curves in a 4x2
    texture rather than 6x2 (Fig. 2)."""
    import oracle
    for n in (1, 3, 10):
        grid = oracle.piecewise_encode(_chain(n))
        assert grid.shape[:2] == (n + 1, 2)
        assert grid.shape[0] * grid.shape[1] == 2 * (n + 1)
    assert oracle.piecewise_encode(_chain(3)).shape[:2] == (4, 2)


def test_encode_constraints(orc):
    """On-path texels are the shared endpoints in zig-zag rows; the two
    texels off the path of segment k average to M_k (N constraints, N+1
    free texels, x_0 = M_0)."""
    chain = _chain(50)
    grid = orc.piecewise_encode(chain)
    n = 50
    for k in range(n + 1):
        r = k & 1
        np.testing.assert_array_equal(grid[k, r], chain[2 * k])
    x = np.array([grid[k, 1 - (k & 1)] for k in range(n + 1)])
    np.testing.assert_array_equal(x[0], chain[1])
    mid = (x[:-1] + x[1:]) / 2
    np.testing.assert_allclose(mid, chain[1::2][:n], rtol=0, atol=1e-13)


def test_grid_eval_equals_chain_definition(orc):
    """Zig-zag grid evaluation equals the chain's plain definition (each
    segment the quadratic (A_k, M_k, A_{k+1}))."""
    chain = _chain(200)
    rng = np.random.default_rng(2)
    T = np.concatenate([rng.uniform(0, 200, 3000), np.arange(201.0)]).astype(np.float32)
    a = orc.piecewise_eval(orc.piecewise_encode(chain), T)
    b = orc.chain_eval(chain, T)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_chain_brute_force_exact(orc):
    """Exact rational evaluation of each queried segment's quadratic."""
    chain = _chain(8, dim=2, seed=9)
    T = np.array([0.0, 0.25, 1.0, 1.5, 3.75, 7.99, 8.0, 5.0, 2.125], np.float32)
    out = orc.piecewise_eval(orc.piecewise_encode(chain), T)
    for q, Tq in enumerate(T):
        k = min(int(np.floor(Tq)), 7)
        t = ex.F(Tq) - k
        for c in range(2):
            b = [ex.F(chain[2 * k, c]), ex.F(chain[2 * k + 1, c]), ex.F(chain[2 * k + 2, c])]
            assert abs(Fraction(out[c, q]) - ex.bezier(b, t)) < Fraction(1, 2 ** 45)


def test_c0_continuity_and_endpoints(orc):
    """At integer T the chain passes exactly through A_T; T = N gives A_N."""
    chain = _chain(64)
    grid = orc.piecewise_encode(chain)
    T = np.arange(65, dtype=np.float64)
    out = orc.piecewise_eval(grid, T)
    np.testing.assert_array_equal(out.T, chain[0::2].astype(np.float64))
    # the end of segment k (local t = 1) equals the start of k+1
    eps_below = np.nextafter(T[1:-1], -np.inf)
    left = orc.piecewise_eval(grid, eps_below)
    np.testing.assert_allclose(left.T, chain[2:-1:2], rtol=0, atol=1e-12)


def test_clamp_and_nan(orc):
    chain = _chain(4)
    grid = orc.piecewise_encode(chain)
    out = orc.piecewise_eval(grid, np.array([-3.0, 0.0, 4.0, 9.0, np.nan]))
    np.testing.assert_array_equal(out[:, 0], chain[0])
    np.testing.assert_array_equal(out[:, 1], chain[0])
    np.testing.assert_array_equal(out[:, 2], chain[8])
    np.testing.assert_array_equal(out[:, 3], chain[8])
    assert np.isnan(out[:, 4]).all()


def test_tensor_diagonal_is_shared_diagonal(orc):
    """A bilinear patch [[P00, P01], [P10, P11]] restricted to u = v = t is
    the quadratic with middle point (P01 + P10)/2 -- the shared diagonal
    E = (B + C)/2 of Eq. 2 (Sec. 2, Fig. 1)."""
    rng = np.random.default_rng(3)
    P = rng.uniform(-1, 1, size=(10, 3, 4))
    t = rng.random(40)
    uv = np.repeat(np.stack([t, t], axis=1)[None], 10, axis=0)
    surf = orc.tensor_points(P, 1, 1, 0, uv)
    quad = np.stack([P[:, :, 0], (P[:, :, 1] + P[:, :, 2]) / 2, P[:, :, 3]], axis=2)
    curve = orc.bezier_decasteljau(quad, t)
    np.testing.assert_allclose(surf, curve, rtol=0, atol=1e-14)


# ------------------------------------------------ stacked zig-zag cubic chain
def _cubic_chain(n_seg, dim=3, seed=11):
    chain, _ = bz_synth.cubic_chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=seed)
    return chain


def test_stacked_layers_identity_exact():
    """(1-t)(A s^2 + 2 E0 s t + A' t^2) + t(A s^2 + 2 E1 s t + A' t^2) is the
    cubic Bezier (A, B, C, A') when E0 = (3B - A)/2 and E1 = (3C - A')/2
    (exact rational arithmetic); any other E0 changes the curve."""
    rng = np.random.default_rng(12)
    for _ in range(10):
        A, B, C, A1 = (ex.F(x) for x in rng.uniform(-3, 3, 4))
        E0, E1 = (3 * B - A) / 2, (3 * C - A1) / 2
        for t in (Fraction(0), Fraction(1), Fraction(2, 7), Fraction(1, 2)):
            s = 1 - t
            q0 = A * s * s + 2 * E0 * s * t + A1 * t * t
            q1 = A * s * s + 2 * E1 * s * t + A1 * t * t
            assert (1 - t) * q0 + t * q1 == ex.bezier([A, B, C, A1], t)
            if 0 < t < 1:
                q0b = A * s * s + 2 * (E0 + 1) * s * t + A1 * t * t
                assert (1 - t) * q0b + t * q1 != ex.bezier([A, B, C, A1], t)


def test_cubic_chain_encoding_layout(orc):
    """Two layers, each a zig-zag quadratic chain over the shared endpoints:
    4(N+1) texels in all (a 2x2x2 block per segment would need 8N)."""
    n = 40
    chain = _cubic_chain(n)
    grid = orc.cubic_chain_encode(chain)
    assert grid.shape == (n + 1, 2, 2, 3)
    for k in range(n + 1):
        for layer in (0, 1):
            np.testing.assert_array_equal(grid[k, layer, k & 1], chain[3 * k])
    c64 = chain.astype(np.float64)
    for layer, pick in ((0, lambda k: (3 * c64[3 * k + 1] - c64[3 * k]) / 2),
                        (1, lambda k: (3 * c64[3 * k + 2] - c64[3 * k + 3]) / 2)):
        x = np.array([grid[k, layer, 1 - (k & 1)] for k in range(n + 1)])
        mid = np.array([pick(k) for k in range(n)], np.float64)
        np.testing.assert_allclose((x[:-1] + x[1:]) / 2, mid, rtol=0, atol=1e-12)


def test_cubic_chain_grid_equals_definition(orc):
    chain = _cubic_chain(300)
    rng = np.random.default_rng(13)
    T = np.concatenate([rng.uniform(0, 300, 4000), np.arange(301.0), [-1.0, 305.0, np.nan]]).astype(np.float32)
    a = orc.cubic_chain_grid_eval(orc.cubic_chain_encode(chain), T)
    b = orc.cubic_chain_eval(chain, T)
    ok = ~np.isnan(T)
    np.testing.assert_allclose(a[:, ok], b[:, ok], rtol=0, atol=1e-11)
    assert np.isnan(a[:, ~ok]).all() and np.isnan(b[:, ~ok]).all()
    # C0: integer T gives the shared endpoint exactly (definition side)
    np.testing.assert_array_equal(orc.cubic_chain_eval(chain, np.arange(301.0)).T, chain[0::3])


def test_cubic_chain_brute_force_exact(orc):
    chain = _cubic_chain(6, dim=2, seed=14)
    T = np.array([0.0, 0.3, 1.0, 2.5, 5.875, 6.0], np.float32)
    out = orc.cubic_chain_grid_eval(orc.cubic_chain_encode(chain), T)
    for q, Tq in enumerate(T):
        k = min(int(np.floor(Tq)), 5)
        t = ex.F(Tq) - k
        for c in range(2):
            b = [ex.F(chain[3 * k + i, c]) for i in range(4)]
            assert abs(Fraction(out[c, q]) - ex.bezier(b, t)) < Fraction(1, 2 ** 40)
