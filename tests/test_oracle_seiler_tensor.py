"""Pins for the oracle's Seiler surfaces and volumes: per-axis Seiler terms
(Sec. 3 applied to each axis of the tensor product of Sec. 2.2)."""
import numpy as np
import pytest

DEGS = [(1, 1, 0), (3, 3, 0), (2, 4, 0), (4, 4, 0), (3, 3, 3), (1, 2, 3), (4, 4, 4), (2, 1, 1)]


def _net(rng, n, dim, du, dv, dw):
    return rng.uniform(-1, 1, size=(n, dim, (du + 1) * (dv + 1) * (dw + 1))).astype(np.float32)


@pytest.mark.parametrize("degs", DEGS)
def test_seiler_tensor_equals_bernstein_tensor(orc, degs):
    """Nested per-axis Seiler evaluation of the converted net equals the
    oracle's separable de Casteljau tensor evaluation (pinned on its own)."""
    du, dv, dw = degs
    rng = np.random.default_rng(600 + du + 5 * dv + 25 * dw)
    P = _net(rng, 9, 3, du, dv, dw)
    uvw = rng.random((9, 40, 3 if dw else 2))
    uvw[:, :4] = [[0, 0, 0][:uvw.shape[2]], [1, 1, 1][:uvw.shape[2]], [0, 1, 0][:uvw.shape[2]],
                  [1, 0, 1][:uvw.shape[2]]]
    sc = orc.tensor_to_seiler(P, du, dv, dw)
    got = orc.tensor_seiler_points(sc, du, dv, dw, uvw)
    ref = orc.tensor_points(P, du, dv, dw, uvw)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_one_axis_is_the_curve_conversion(orc):
    """With dv = 1 the u-fibres at v = 0 and v = 1 are plain curves: the
    corresponding terms are the curve Seiler terms of those fibres."""
    rng = np.random.default_rng(610)
    du = 5
    P = _net(rng, 4, 2, du, 1, 0)
    sc = orc.tensor_to_seiler(P, du, 1, 0).reshape(4, 2, du + 1, 2)
    for j in (0, 1):
        fib = np.ascontiguousarray(P.reshape(4, 2, du + 1, 2)[:, :, :, j])
        np.testing.assert_allclose(sc[:, :, :, j], orc.seiler_from_bezier(fib), rtol=0, atol=1e-13)


def test_corners_survive_conversion(orc):
    """b0 and bd keep their places on every axis, so the terms at the
    corner indices are the corner control points, and the surface passes
    through them exactly."""
    rng = np.random.default_rng(620)
    du, dv, dw = 3, 2, 4
    P = _net(rng, 5, 3, du, dv, dw)
    sc = orc.tensor_to_seiler(P, du, dv, dw).reshape(5, 3, du + 1, dv + 1, dw + 1)
    Pr = P.reshape(5, 3, du + 1, dv + 1, dw + 1)
    for (i, si) in ((0, 0), (du, 1)):
        for (j, sj) in ((0, 0), (dv, 1)):
            for (k, sk) in ((0, 0), (dw, 1)):
                np.testing.assert_array_equal(sc[:, :, si, sj, sk], Pr[:, :, i, j, k])
    uvw = np.array([[[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)]] * 5, np.float64)
    got = orc.tensor_seiler_points(orc.tensor_to_seiler(P, du, dv, dw), du, dv, dw, uvw).reshape(3, 5, 8)
    want = np.stack([Pr[:, :, a * du, b * dv, c * dw] for a in (0, 1) for b in (0, 1) for c in (0, 1)], axis=2)
    np.testing.assert_array_equal(got, want.transpose(1, 0, 2))


def test_grid_helper_matches_points(orc):
    rng = np.random.default_rng(630)
    P = _net(rng, 3, 3, 3, 3, 0)
    sc = orc.tensor_to_seiler(P, 3, 3)
    np.testing.assert_allclose(orc.tensor_seiler_grid(sc, 3, 3, 5, 7), orc.tensor_grid(P, 3, 3, 5, 7), rtol=0,
                               atol=1e-13)
