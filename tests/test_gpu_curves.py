"""GPU parity: integral and rational Bezier curves (de Casteljau, Bernstein,
Seiler) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import TOL_F32, bbox_err, dev, extents, host, to_dev

pytestmark = pytest.mark.gpu

METHODS = ["decasteljau", "bernstein", "seiler"]


@pytest.mark.parametrize("degree", range(1, 16))
@pytest.mark.parametrize("method", METHODS)
def test_curves_all_degrees(orc, degree, method):
    """Every degree 1..15, dims 1..4, ragged counts, shared and per-curve t."""
    for dim, per_object in ((3, False), (1, True), (2, False), (4, True)):
        ctrl, t = bz_synth.random_curves(37, degree, dim, 67, seed=100 * degree + dim, per_object=per_object)
        got = host(bz.eval_bezier(to_dev(ctrl), to_dev(t), method))
        ref = orc.bezier_decasteljau(ctrl, t, per_object)
        err = bbox_err(got, ref, extents(ctrl), 67)
        assert err <= TOL_F32, (degree, dim, method, err)


def test_auto_method_is_the_bernstein_form():
    """BZ_AUTO resolves to the Bernstein form: bit-identical results for
    integral and rational curves (low and high degree) and for a batch plan."""
    for degree in (3, 12):
        ctrl, t = bz_synth.random_curves(29, degree, 3, 40, seed=77 + degree)
        c, tt = to_dev(ctrl), to_dev(t)
        np.testing.assert_array_equal(host(bz.eval_bezier(c, tt, "auto")), host(bz.eval_bezier(c, tt, "bernstein")))
        w = to_dev(np.random.default_rng(degree).uniform(0.5, 2.0, (29, degree + 1)))
        np.testing.assert_array_equal(host(bz.eval_rational(c, w, tt, "auto")),
                                      host(bz.eval_rational(c, w, tt, "bernstein")))
    b = bz_synth.mixed_batch(n_bezier=300, n_nurbs=20, n_t=8, seed=5)
    dv = lambda x: torch.from_numpy(x).cuda()  # noqa: E731
    outs = []
    for m in ("auto", "bernstein"):
        plan = bz.BatchPlan(dv(b.kind_degree.astype(np.int16)), dv(b.cp_offset), to_dev(b.ctrl), to_dev(b.w), 3,
                            dv(b.knot_offset), to_dev(b.knots), 8, m)
        outs.append(host(plan(to_dev(b.t))))
        plan.close()
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("method", METHODS)
def test_config_plain_full_size(orc, method):
    """4096 cubic 3D curves x 256 shared t (1M points), every point checked."""
    ctrl, t = bz_synth.plain_curves()
    got = host(bz.eval_bezier(to_dev(ctrl), to_dev(t), method))
    ref = orc.bezier_decasteljau(ctrl, t)
    err = bbox_err(got, ref, extents(ctrl), 256)
    assert err <= TOL_F32, err


@pytest.mark.parametrize("method", METHODS)
def test_endpoints_bit_exact(method):
    for degree in (1, 2, 3, 7, 15):
        ctrl, _ = bz_synth.random_curves(50, degree, 3, 1, seed=7)
        t = np.array([0.0, 1.0], np.float32)
        got = bz.eval_bezier(to_dev(ctrl), to_dev(t), method).cpu().numpy().reshape(3, 50, 2)
        np.testing.assert_array_equal(got[:, :, 0], ctrl[:, :, 0].T)
        np.testing.assert_array_equal(got[:, :, 1], ctrl[:, :, degree].T)


def test_nan_and_extrapolation(orc):
    ctrl, _ = bz_synth.random_curves(8, 3, 3, 1, seed=8)
    t = np.array([np.nan, -0.5, 1.5, 0.25], np.float32)
    for m in METHODS:
        got = host(bz.eval_bezier(to_dev(ctrl), to_dev(t), m)).reshape(3, 8, 4)
        assert np.isnan(got[:, :, 0]).all()
        ref = orc.bezier_decasteljau(ctrl, t[1:]).reshape(3, 8, 3)
        np.testing.assert_allclose(got[:, :, 1:], ref, rtol=0, atol=1e-5)


@pytest.mark.parametrize("n_t", [64, 192, 256, 512, 768])
@pytest.mark.parametrize("method", METHODS)
def test_curves_wave_uniform_modes(orc, n_t, method):
    """n_t a multiple of 64 (one curve per wavefront) or of 256 (256 queries of
    one curve per wavefront, four per lane): degrees 1..15, dims 1..4, shared
    and per-curve t, FP32 / FP16 / BF16 storage, a curve count that leaves the
    last workgroup partly empty."""
    cases = ((1, 3, False, None), (3, 1, True, None), (7, 2, False, torch.float16), (15, 4, True, None),
             (3, 3, False, torch.bfloat16), (5, 3, True, torch.float16))
    for degree, dim, per_object, dtype in cases:
        ctrl, t = bz_synth.random_curves(21, degree, dim, n_t, seed=n_t + 16 * degree + dim, per_object=per_object)
        dc = to_dev(ctrl) if dtype is None else to_dev(ctrl).to(dtype)
        pts = dc.float().cpu().numpy()
        got = host(bz.eval_bezier(dc, to_dev(t), method))
        ref = orc.bezier_decasteljau(pts, t, per_object)
        assert bbox_err(got, ref, extents(pts), n_t) <= TOL_F32, (n_t, degree, dim, per_object, dtype, method)


def test_curves_across_launch_chunks(orc):
    """2^18 + 5 cubic curves x 4096 t: more than 2^30 queries, so the call is
    split into launches of whole curves and the last 5 curves come in a second
    launch with its own control-point offset and global query offset (12.9 GB
    of output; per-curve t indexed by the global query).  Curves on both sides
    of the boundary and at the ends are checked, shared and per-curve t."""
    n_t = 4096
    per = (1 << 30) // n_t
    n = per + 5
    rng = np.random.default_rng(91)
    ctrl = rng.uniform(-1, 1, size=(n, 3, 4)).astype(np.float32)
    pick = np.array([0, 1, per - 1, per, per + 1, n - 1])
    idx = torch.from_numpy(pick).cuda()
    cd = to_dev(ctrl)
    out = torch.empty((3, n * n_t), dtype=torch.float32, device=cd.device)
    t_shared = rng.random(n_t, dtype=np.float32)
    t_per = rng.random((n, n_t), dtype=np.float32)
    for t, per_object in ((t_shared, False), (t_per, True)):
        td = to_dev(t)
        ref = orc.bezier_decasteljau(ctrl[pick], t[pick] if per_object else t, per_object)
        for m in METHODS:
            out.fill_(float("nan"))
            bz.eval_bezier(cd, td, m, out=out)
            got = out.view(3, n, n_t)[:, idx].reshape(3, -1).cpu().numpy()
            assert bbox_err(got, ref, extents(ctrl[pick]), n_t) <= TOL_F32, (m, per_object)
        del td
    del out, cd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_low_precision_storage(orc, dtype):
    """FP16/BF16 control points, FP32 arithmetic: exact-to-FP32 on the rounded
    points, and within max_i|b_i - round(b_i)| of the FP32 curve (convexity of
    the Bernstein weights)."""
    ctrl, t = bz_synth.random_curves(300, 5, 3, 40, seed=9)
    dc = to_dev(ctrl).to(dtype)
    rounded = dc.float().cpu().numpy()
    for m in METHODS:
        got = host(bz.eval_bezier(dc, to_dev(t), m))
        ref_r = orc.bezier_decasteljau(rounded, t, True)
        assert bbox_err(got, ref_r, extents(rounded), 40) <= TOL_F32
        ref = orc.bezier_decasteljau(ctrl, t, True)
        bound = np.abs(rounded - ctrl).max() + 2e-6
        assert np.abs(got - ref).max() <= bound


@pytest.mark.parametrize("degree", [2, 3, 5, 8, 15])
@pytest.mark.parametrize("n_t", [33, 256])
def test_seiler_terms_and_eval(orc, degree, n_t):
    ctrl, t = bz_synth.random_curves(70, degree, 3, n_t, seed=10 + degree)
    sc = bz.bezier_to_seiler(to_dev(ctrl))
    ref_sc = orc.seiler_from_bezier(ctrl)
    scale = np.abs(ref_sc).max(axis=2, keepdims=True) + 1.0
    assert (np.abs(host(sc) - ref_sc) / scale).max() < 2e-6
    got = host(bz.eval_seiler(sc, to_dev(t)))
    ref = orc.bezier_decasteljau(ctrl, t, True)
    assert bbox_err(got, ref, extents(ctrl), n_t) <= TOL_F32


@pytest.mark.parametrize("degree", [1, 2, 3, 6, 11, 15])
@pytest.mark.parametrize("method", METHODS)
def test_rational_parity(orc, degree, method):
    ctrl, w, t = bz_synth.rational_curves(53, degree, 3, 29, seed=20 + degree)
    nf = torch.zeros(1, dtype=torch.int32, device=dev())
    got = host(bz.eval_rational(to_dev(ctrl), to_dev(w), to_dev(t), method, n_fixed=nf))
    ref = orc.rational_eval(ctrl, w, t, True)
    assert bbox_err(got, ref, extents(ctrl), 29) <= TOL_F32
    assert int(nf.item()) == 0  # positive weights: conditioning 1, never recomputed


def test_rational_quarter_circle():
    ctrl = np.array([[[1.0, 1.0, 0.0], [0.0, 1.0, 1.0]]], np.float32)
    w = np.array([[1.0, np.sqrt(0.5), 1.0]], np.float32)
    t = np.linspace(0, 1, 1001).astype(np.float32)
    for m in METHODS:
        out = host(bz.eval_rational(to_dev(ctrl), to_dev(w), to_dev(t), m))
        assert np.abs(np.hypot(out[0], out[1]) - 1.0).max() < 1e-6


def test_rational_fp64_recompute(orc):
    """Weights close to (1,-1,1,-1) give W(t) close to (1-2t)^3 while
    sum|w_i|B_i stays near 1: near t = 1/2 the FP32 weight sum cancels.  Those
    points (conditioning above kappa) are recomputed in FP64 and the worst
    error drops far below the plain FP32 path's."""
    rng = np.random.default_rng(11)
    n, d = 64, 3
    ctrl = rng.uniform(-1, 1, size=(n, 2, d + 1)).astype(np.float32)
    w = np.array([1.0, -1.0, 1.0, -1.0]) * (1.0 + 0.01 * rng.uniform(-1, 1, (n, d + 1)))
    w = np.ascontiguousarray(w.astype(np.float32))
    t = rng.random((n, 31)).astype(np.float32)
    nf = torch.zeros(1, dtype=torch.int32, device=dev())
    got = host(bz.eval_rational(to_dev(ctrl), to_dev(w), to_dev(t), "decasteljau", kappa=64.0, n_fixed=nf))
    ref = orc.rational_eval(ctrl, w, t, True)
    assert int(nf.item()) > 0
    nofix = host(bz.eval_rational(to_dev(ctrl), to_dev(w), to_dev(t), "decasteljau", kappa=0.0))
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    rel_nofix = np.abs(nofix - ref) / np.maximum(np.abs(ref), 1.0)
    # kept FP32 points have conditioning <= 64: a few ulps times 64
    assert rel.max() < 64 * 8 * 2.0 ** -24
    assert rel.max() < 0.1 * rel_nofix.max()


def test_empty_and_single():
    d = dev()
    ctrl = torch.zeros((0, 3, 4), device=d)
    t = torch.zeros(5, device=d)
    assert bz.eval_bezier(ctrl, t).shape == (3, 0)
    ctrl1, t1 = bz_synth.random_curves(1, 3, 3, 1, seed=1, per_object=False)
    out = host(bz.eval_bezier(to_dev(ctrl1), to_dev(t1)))
    assert out.shape == (3, 1) and np.isfinite(out).all()
