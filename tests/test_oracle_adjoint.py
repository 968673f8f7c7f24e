"""Pins for the oracle's adjoint (hodograph derivative, dL/dP, dL/dw,
dL/dt), the fitting loss and Adam: central finite differences, the
dot-product test and closed-form first Adam steps."""
import numpy as np
import pytest

import bz_synth


def _fd(f, x, h):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("d", [1, 3, 6])
@pytest.mark.parametrize("rational", [False, True])
def test_adjoint_matches_finite_differences(orc, d, rational):
    rng = np.random.default_rng(d + 10 * rational)
    n, dim, nt = 3, 3, 5
    ctrl = rng.uniform(-1, 1, size=(n, dim, d + 1))
    w = rng.uniform(0.5, 2.0, size=(n, d + 1)) if rational else None
    t = rng.uniform(0.05, 0.95, size=(n, nt))
    gout = rng.normal(size=(dim, n * nt))

    def ev(c=ctrl, ww=w, tt=t):
        if rational:
            return orc.rational_eval(c, ww, tt, True)
        return orc.bezier_decasteljau(c, tt, True)

    def L(c=ctrl, ww=w, tt=t):
        return float(np.sum(ev(c, ww, tt) * gout))

    gc, gw, gt = orc.bezier_adjoint(ctrl, t, gout, w=w)
    h = 1e-6
    np.testing.assert_allclose(gc, _fd(lambda c: L(c=c), ctrl, h), rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(gt, _fd(lambda tt: L(tt=tt), t, h), rtol=1e-6, atol=1e-7)
    if rational:
        np.testing.assert_allclose(gw, _fd(lambda ww: L(ww=ww), w, h), rtol=1e-6, atol=1e-8)


def test_adjoint_dot_product(orc):
    """C is linear in the control points: <J v, g> = <v, J^T g>."""
    rng = np.random.default_rng(3)
    n, d, dim, nt = 20, 5, 3, 7
    t = rng.random((n, nt))
    v = rng.normal(size=(n, dim, d + 1))
    g = rng.normal(size=(dim, n * nt))
    Jv = orc.bezier_decasteljau(v, t, True)
    JTg, _, _ = orc.bezier_adjoint(v, t, g)
    assert abs(np.sum(Jv * g) - np.sum(v * JTg)) < 1e-10 * np.sum(np.abs(Jv * g))


def test_hodograph_closed_form(orc):
    """For b_i = (i/d)^2 (a parabola t^2 in Bernstein form for d >= 2) the
    derivative is 2t."""
    for d in (2, 3, 7):
        ctrl = np.zeros((1, 1, d + 1))
        # t^2 = sum_i [i(i-1)/(d(d-1))] B_{i,d}(t)
        ctrl[0, 0] = [i * (i - 1) / (d * (d - 1)) for i in range(d + 1)]
        t = np.linspace(0, 1, 11)[None]
        _, _, gt = orc.bezier_adjoint(ctrl, t, np.ones((1, 11)))
        np.testing.assert_allclose(gt[0], 2 * t[0], atol=1e-14)


def test_fit_loss_and_gradient(orc):
    gt_ctrl, tau, eps = bz_synth.fit_problem(n_curves=6, n_samples=16, seed=4)
    y = orc.bezier_decasteljau(gt_ctrl, tau, True) + eps
    rng = np.random.default_rng(5)
    ctrl = rng.uniform(-1, 1, size=gt_ctrl.shape)
    t = rng.random(tau.shape)
    L, gc, gtt = orc.fit_loss_grad(ctrl, t, y)
    r = orc.bezier_decasteljau(ctrl, t, True) - y
    assert abs(L - np.sum(r * r) / t.size) < 1e-13
    f = lambda c: orc.fit_loss_grad(c, t, y)[0]
    np.testing.assert_allclose(gc, _fd(f, ctrl, 1e-6), rtol=1e-5, atol=1e-9)
    f = lambda tt: orc.fit_loss_grad(ctrl, tt, y)[0]
    np.testing.assert_allclose(gtt, _fd(f, t, 1e-6), rtol=1e-5, atol=1e-9)
    # at the ground truth with no noise the loss and gradients vanish
    L0, g0, gt0 = orc.fit_loss_grad(gt_ctrl, tau, orc.bezier_decasteljau(gt_ctrl, tau, True))
    assert L0 < 1e-28 and np.abs(g0).max() < 1e-14 and np.abs(gt0).max() < 1e-14


def test_adam_first_step_is_signed_lr(orc):
    """With zero moments the first bias-corrected step is lr*g/(|g|+eps)."""
    rng = np.random.default_rng(6)
    g = rng.normal(size=50)
    p = rng.random(50)
    p0 = p.copy()
    m, v = np.zeros(50), np.zeros(50)
    orc.adam(p, m, v, g, 1, lr=0.01)
    np.testing.assert_allclose(p, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    q = np.full(4, 0.999)
    orc.adam(q, np.zeros(4), np.zeros(4), -np.ones(4), 1, lr=0.01, lo=0.0, hi=1.0)
    np.testing.assert_array_equal(q, 1.0)


def test_fit_reference_converges(orc):
    """Fitting noisy samples of a cubic drives the loss down toward the
    noise floor (3 sigma^2 per sample for 3D Gaussian noise).  200 Adam steps
    at lr 1e-2 from the chord start only get within 20x of it (the control
    points and the 128 parameters per curve are strongly coupled, so Adam's
    fixed step converges slowly); 3000 steps get within 3x."""
    gt_ctrl, tau, eps = bz_synth.fit_problem(n_curves=16, n_samples=128, seed=7)
    _, _, losses = orc.fit_reference(gt_ctrl, tau, eps, steps=200)
    assert losses[-1] < 0.2 * losses[0]
    assert losses[-1] < 20 * 3 * 0.01 ** 2
    assert np.mean(np.diff(losses) < 0) > 0.8
    _, _, long_run = orc.fit_reference(gt_ctrl, tau, eps, steps=3000)
    assert long_run[-1] < 3 * 3 * 0.01 ** 2
    assert long_run[-1] < 0.2 * losses[-1]


def test_fit_loss_at_the_ground_truth_is_the_noise(orc):
    """At the ground-truth control points and parameters the residuals are
    the noise itself, so the loss is its mean square (about 3 sigma^2) and
    the gradient with respect to the control points is the noise's
    projection on the basis."""
    gt_ctrl, tau, eps = bz_synth.fit_problem(n_curves=16, n_samples=128, seed=7)
    y = orc.bezier_decasteljau(gt_ctrl, tau, True) + eps.astype(np.float64)
    L, gc, _ = orc.fit_loss_grad(gt_ctrl, tau, y)
    e = eps.astype(np.float64)
    assert abs(L - (e * e).sum() / tau.size) < 1e-15
    assert abs(L / (3 * 0.01 ** 2) - 1) < 0.05
    from math import comb
    t = tau.astype(np.float64)
    Bm = np.stack([comb(3, i) * (1 - t) ** (3 - i) * t ** i for i in range(4)], -1)  # n nt 4
    want = -2.0 / tau.size * np.einsum("dcj,cji->cdi", e.reshape(3, *tau.shape), Bm)
    np.testing.assert_allclose(gc, want, rtol=1e-9, atol=1e-15)
