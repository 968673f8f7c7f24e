"""GPU parity: mixed batches (integral / rational Bezier of degree 1..15 and
cubic NURBS) in one persistent launch, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._batch import _extents, _lp_bound
from tests._gpu import TOL_F32, host, to_dev

pytestmark = pytest.mark.gpu


def _err(got, ref, ext, n_t):
    d = np.abs(got - ref)
    if np.isnan(d).any():
        return np.inf
    return float((d.max(axis=0).reshape(-1, n_t).max(axis=1) / ext).max())


def _plan(b, dtype=torch.float32, method="bernstein"):
    dev = {
        "kind_degree": torch.from_numpy(b.kind_degree.astype(np.int16)).cuda(),
        "cp_offset": torch.from_numpy(b.cp_offset).cuda(),
        "ctrl": to_dev(b.ctrl).to(dtype),
        "w": to_dev(b.w).to(dtype),
        "knot_offset": torch.from_numpy(b.knot_offset).cuda(),
        "knots": to_dev(b.knots if b.knots.size else np.zeros(1, np.float32)),
    }
    plan = bz.BatchPlan(dev["kind_degree"], dev["cp_offset"], dev["ctrl"], dev["w"], b.dim, dev["knot_offset"],
                        dev["knots"], b.n_t, method)
    return plan, dev


def _subbatch(b, n):
    """The first n objects of a batch, re-based."""
    cp = b.cp_offset[:n + 1]
    ko = b.knot_offset[:n + 1]
    return bz_synth.Batch(dim=b.dim, n_t=b.n_t, kind_degree=b.kind_degree[:n], cp_offset=cp,
                          ctrl=b.ctrl[:cp[-1] * b.dim], w=b.w[:cp[-1]], knot_offset=ko, knots=b.knots[:ko[-1]],
                          t=b.t[:n])


@pytest.mark.parametrize("method", ["bernstein", "decasteljau"])
@pytest.mark.parametrize("n_t", [16, 1, 37])
def test_mixed_batch(orc, method, n_t):
    b = bz_synth.mixed_batch(n_bezier=3000, n_nurbs=400, n_t=n_t, deg_lo=1, seed=11 + n_t)
    plan, dev = _plan(b, method=method)
    info = plan.info()
    assert info["n_classes"] == len(set(b.kind_degree.tolist()))
    t = to_dev(b.t)
    got = host(plan(t))
    ref = orc.batch_eval(b)
    assert _err(got, ref, _extents(b), n_t) <= TOL_F32
    # repeated launches reuse the self-resetting work counter
    again = host(plan(t))
    np.testing.assert_array_equal(again, got)


@pytest.mark.parametrize("n_t", [8, 16])
def test_mixed_batch_dims_and_kinds(orc, n_t):
    """n_t = 16 takes the DPP row-broadcast path (one object per 16-lane
    row), other n_t the per-lane loads; every dim, degrees 1..15."""
    for dim in (1, 2, 4):
        b = bz_synth.mixed_batch(n_bezier=500, n_nurbs=60, dim=dim, n_t=n_t, deg_lo=1, seed=dim + n_t)
        plan, _ = _plan(b)
        got = host(plan(to_dev(b.t)))
        assert _err(got, orc.batch_eval(b), _extents(b), n_t) <= TOL_F32
    b = bz_synth.mixed_batch(n_bezier=700, n_nurbs=0, n_t=5, seed=4)  # no NURBS, no knots needed
    plan, _ = _plan(b)
    assert _err(host(plan(to_dev(b.t))), orc.batch_eval(b), _extents(b), 5) <= TOL_F32
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=333, n_t=7, knots_lo=8, knots_hi=8, seed=5)  # single-span NURBS
    plan, _ = _plan(b)
    assert _err(host(plan(to_dev(b.t))), orc.batch_eval(b), _extents(b), 7) <= TOL_F32


def test_nurbs_clamp_and_ends(orc):
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=50, n_t=4, seed=6)
    b.t[:, 0] = -0.5
    b.t[:, 1] = 0.0
    b.t[:, 2] = 1.0
    b.t[:, 3] = 7.0
    plan, _ = _plan(b)
    got = host(plan(to_dev(b.t))).reshape(3, 50, 4)
    ref = orc.batch_eval(b).reshape(3, 50, 4)
    for o in range(50):
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        P = b.ctrl[a0 * 3:a1 * 3].reshape(3, a1 - a0)
        np.testing.assert_allclose(got[:, o, :2], P[:, :1].repeat(2, 1), atol=2e-6)
        np.testing.assert_allclose(got[:, o, 2:], P[:, -1:].repeat(2, 1), atol=2e-6)
    np.testing.assert_allclose(got, ref, atol=2e-6)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_nurbs_clustered_knots(orc, dtype):
    """Interior knots packed into a narrow cluster put many breakpoints in one
    bucket of the span lookup (FP32 storage: the bucket table's binary-search
    fallback; 16-bit storage: the search over all breakpoints); parameters at,
    just beside and between the clustered breakpoints, and at random.  16-bit
    plans against the oracle on their rounded control points and weights."""
    b = bz_synth.mixed_batch(n_bezier=0, n_nurbs=240, n_t=16, seed=12)
    rng = np.random.default_rng(13)
    for o in range(b.n_obj):
        a, e = b.knot_offset[o], b.knot_offset[o + 1]
        n_in = e - a - 8
        if n_in < 2:
            continue
        if o % 3 == 0:  # all interior knots in [0.5, 0.5 + 2^-10)
            v = 0.5 + rng.choice(256, n_in, replace=False) * 2.0 ** -18
        elif o % 3 == 1:  # half uniform, half clustered
            h = n_in // 2
            v = np.concatenate([rng.uniform(0.01, 0.99, n_in - h), 0.25 + rng.choice(64, h, replace=False) * 2.0 ** -20])
        else:
            continue
        b.knots[a + 4:e - 4] = np.sort(v).astype(np.float32)
        inner = b.knots[a + 4:e - 4]
        pick = rng.integers(0, n_in, 16)
        t = inner[pick].copy()
        t[4:8] = np.nextafter(t[4:8], np.float32(0))
        t[8:12] = np.nextafter(t[8:12], np.float32(1))
        t[12:] = rng.uniform(0.0, 1.0, 4)
        b.t[o] = t
    plan, dev = _plan(b, dtype=dtype)
    got = host(plan(to_dev(b.t)))
    rb = bz_synth.Batch(**{**b.__dict__})
    rb.ctrl = dev["ctrl"].float().cpu().numpy()
    rb.w = dev["w"].float().cpu().numpy()
    assert _err(got, orc.batch_eval(rb), _extents(rb), 16) <= TOL_F32


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_low_precision_storage(orc, dtype):
    """FP16/BF16 control points and weights, FP32 arithmetic: within FP32
    rounding of the oracle on the rounded inputs."""
    b = bz_synth.mixed_batch(n_bezier=2000, n_nurbs=200, n_t=16, seed=7)
    plan, dev = _plan(b, dtype=dtype)
    got = host(plan(to_dev(b.t)))
    rb = bz_synth.Batch(**{**b.__dict__})
    rb.ctrl = dev["ctrl"].float().cpu().numpy()
    rb.w = dev["w"].float().cpu().numpy()
    ref = orc.batch_eval(rb)
    assert _err(got, ref, _extents(rb), 16) <= TOL_F32
    for vq, window in ((1, 0), (4, 300), (1, 300)):  # both lane mappings, window-major order
        plan.configure(500, 2, "static", vq, window)
        assert _err(host(plan(to_dev(b.t))), ref, _extents(rb), 16) <= TOL_F32, (vq, window)


@pytest.mark.parametrize("n_t", [16, 8, 4, 12])
def test_every_launch_configuration(orc, n_t):
    """Both lane mappings (1 query per lane; 4 consecutive parameters of one
    object per lane), every tile size, both schedules, small and large
    grids, class-major and window-major tile orders (windows of one object,
    and of 700 objects, which cut classes into partial tiles): within the
    tolerance of the oracle, and bit-identical across schedules, tile sizes,
    orders and grids of one mapping."""
    b = bz_synth.mixed_batch(n_bezier=3000, n_nurbs=300, n_t=n_t, deg_lo=1, seed=40 + n_t)
    plan, _ = _plan(b)
    t = to_dev(b.t)
    ref = orc.batch_eval(b)
    for vq in (1, 4):
        first = None  # schedules and tile sizes must not change a bit; the
        # two lane mappings contract their FMAs differently (1 ulp apart)
        for sub in (1, 2, 4):
            for sched in ("dynamic", "static"):
                for wg, window in ((7, 0), (600, 0), (600, 1), (7, 700), (600, 700)):
                    plan.configure(wg, sub, sched, vq, window)
                    out = torch.full((3, b.n_obj * n_t), float("nan"), device=t.device)
                    got = host(plan(t, out=out))  # every query must be written
                    assert _err(got, ref, _extents(b), n_t) <= TOL_F32, (vq, sub, sched, wg, window)
                    if first is None:
                        first = got
                    else:
                        np.testing.assert_array_equal(got, first)
    b2 = bz_synth.mixed_batch(n_bezier=50, n_nurbs=5, n_t=6, seed=49)
    plan2, _ = _plan(b2)
    with pytest.raises(bz.BzError) as e:
        plan2.configure(64, 1, "dynamic", 4)
    assert e.value.code == bz.ERR_UNSUPPORTED


def test_autotune_keeps_results(orc):
    b = bz_synth.mixed_batch(n_bezier=20000, n_nurbs=2000, n_t=16, seed=8)
    plan, _ = _plan(b)
    t = to_dev(b.t)
    out = torch.empty((3, b.n_obj * 16), device=t.device)
    best = plan.autotune(t, out)
    assert best["workgroups"] >= 1 and best["tile_multiple"] in (1, 2, 4) and best["queries_per_lane"] in (1, 4)
    assert best["window"] == 0  # every window candidate covers the 22000 objects
    out.fill_(float("nan"))
    got = host(plan(t, out=out))
    assert _err(got, orc.batch_eval(b), _extents(b), 16) <= TOL_F32


def test_plan_errors():
    b = bz_synth.mixed_batch(n_bezier=10, n_nurbs=3, n_t=2, seed=9)
    bad = b.knots.copy()
    k0 = b.knot_offset[np.nonzero(b.kind_degree >> 8 == 2)[0][0]]
    bad[k0] = -1.0  # breaks the clamped start
    b2 = bz_synth.Batch(**{**b.__dict__, "knots": bad})
    with pytest.raises(bz.BzError) as e:
        _plan(b2)
    assert e.value.code == bz.ERR_SHAPE
    kd = b.kind_degree.copy()
    kd[np.nonzero(kd >> 8 == 2)[0][0]] = (2 << 8) | 2
    with pytest.raises(bz.BzError) as e:
        _plan(bz_synth.Batch(**{**b.__dict__, "kind_degree": kd}))
    assert e.value.code == bz.ERR_UNSUPPORTED


def test_config_batched_full_size_sampled(orc):
    """2^20 Bezier curves (degree 2..15, half rational) + 2^16 cubic NURBS,
    16 random t each, FP32 and FP16 storage, one persistent launch each:
    65536 objects drawn at random from the whole batch (with the first and
    last object and the last NURBS) checked against the oracle.  FP32: within
    1e-5 of each object's box.  FP16: within FP32 rounding of the oracle on the
    rounded inputs, and against the FP32 inputs within the rounding bound
    (_lp_bound) plus 1e-5 of the box."""
    b = bz_synth.mixed_batch()
    kinds = b.kind_degree >> 8
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([rng.choice(b.n_obj, 65536, replace=False),
                                    [0, b.n_obj - 1, np.nonzero(kinds == 2)[0][-1]]]))
    sub = b.subset(idx)
    ref = orc.batch_eval(sub)
    ext = _extents(sub)
    idx_d = torch.from_numpy(idx).cuda()
    for dtype in (torch.float32, torch.float16):
        plan, dev = _plan(b, dtype=dtype)
        got = host(plan(to_dev(b.t)).view(3, b.n_obj, 16)[:, idx_d].reshape(3, -1))
        if dtype == torch.float32:
            assert _err(got, ref, ext, 16) <= TOL_F32
        else:
            rsub = bz_synth.Batch(**{**sub.__dict__})
            rsub.ctrl = torch.from_numpy(sub.ctrl).to(dtype).float().numpy()
            rsub.w = torch.from_numpy(sub.w).to(dtype).float().numpy()
            assert _err(got, orc.batch_eval(rsub), _extents(rsub), 16) <= TOL_F32
            d = np.abs(got - ref).max(axis=0).reshape(-1, 16).max(axis=1)
            bound = _lp_bound(sub, rsub, ext) + TOL_F32 * ext
            assert (d <= bound).all(), float((d / bound).max())
        plan.close()


def _signed_batch(n_rat=600, n_t=16, seed=31):
    """Rational curves of degree 2..9 with weights of both signs, parameters
    placed next to the roots of the weight sum sum w_i B_i(t) (where the
    conditioning number sum|w_i|B_i / |sum w_i B_i| is large) and at random;
    plus integral curves and positive-weight rationals."""
    b = bz_synth.mixed_batch(n_bezier=n_rat, n_nurbs=0, n_t=n_t, deg_lo=2, deg_hi=9, seed=seed)
    rng = np.random.default_rng(seed + 1)
    kinds = b.kind_degree >> 8
    from math import comb
    n_signed = 0
    for o in range(b.n_obj):
        if kinds[o] != 1 or o % 3 == 0:
            continue
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        d = a1 - a0 - 1
        w = rng.uniform(0.5, 2.0, d + 1)
        w[1:d] *= -1.0  # inner weights negative: the sum changes sign inside (0, 1)
        b.w[a0:a1] = w.astype(np.float32)
        wf = b.w[a0:a1].astype(np.float64)
        poly = np.zeros(d + 1)  # the weight sum in the power basis (numpy: highest power first)
        for i in range(d + 1):
            bi = np.zeros(d + 1)
            for j in range(d - i + 1):  # C(d,i) t^i (1-t)^(d-i)
                bi[d - (i + j)] += comb(d, i) * comb(d - i, j) * (-1) ** j
            poly += wf[i] * bi
        roots = [r.real for r in np.roots(poly) if abs(r.imag) < 1e-12 and 0.0 < r.real < 1.0]
        ts = list(rng.random(n_t))
        for k, r in enumerate(roots[:2]):
            for j, off in enumerate((1e-4, -1e-4, 1e-6, -1e-6, 0.0)):
                ts[5 * k + j] = r + off
        b.t[o] = np.clip(np.asarray(ts[:n_t]), 0.0, 1.0).astype(np.float32)
        n_signed += 1
    return b, n_signed


def _kappa(b):
    """FP64 conditioning number of every query of the rational objects."""
    from math import comb
    kap = np.ones((b.n_obj, b.n_t))
    for o in range(b.n_obj):
        if (b.kind_degree[o] >> 8) != 1:
            continue
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        d = a1 - a0 - 1
        w = b.w[a0:a1].astype(np.float64)
        t = b.t[o].astype(np.float64)[:, None]
        B = np.array([comb(d, i) for i in range(d + 1)]) * t ** np.arange(d + 1) * (1 - t) ** (d - np.arange(d + 1))
        kap[o] = (np.abs(w) * B).sum(1) / np.maximum(np.abs((w * B).sum(1)), 1e-300)
    return kap


@pytest.mark.parametrize("method", ["bernstein", "decasteljau"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_signed_weight_rationals(orc, method, dtype):
    """Rational objects with weights of both signs get their own classes
    with the conditioning test: points next to a root of the weight sum
    (conditioning numbers far above 64) are recomputed in FP64, so every
    point matches the oracle to 1e-5 of the larger of the object's box and
    the point's own size (near a pole the point itself is huge, and its FP32
    rounding alone is 2^-24 of it)."""
    b, n_signed = _signed_batch()
    kap = _kappa(b)
    assert n_signed > 150 and (kap > 1e3).sum() > 300  # the test reaches the recomputation
    plan, dev = _plan(b, dtype=dtype, method=method)
    assert plan.info()["n_classes"] > len(set(b.kind_degree.tolist()))  # signed classes of their own
    got = host(plan(to_dev(b.t)))
    rb = bz_synth.Batch(**{**b.__dict__})
    rb.ctrl = dev["ctrl"].float().cpu().numpy()
    rb.w = dev["w"].float().cpu().numpy()
    ref = orc.batch_eval(rb)
    scale = np.maximum(np.repeat(_extents(rb), b.n_t)[None, :], np.abs(ref))
    assert np.isfinite(got).all() or np.array_equal(np.isfinite(got), np.isfinite(ref))
    assert (np.abs(got - ref) / scale).max() <= TOL_F32
    # the signed classes' launch follows the persistent one in every configuration
    for cfg in ((64, 1, "dynamic", 1, 0), (512, 4, "static", 4, 300)):
        plan.configure(*cfg)
        got = host(plan(to_dev(b.t)))
        assert (np.abs(got - ref) / scale).max() <= TOL_F32, cfg
    # the same objects through bz_eval_rational (its own FP64 recomputation) agree
    for o in np.nonzero(b.kind_degree >> 8 == 1)[0][:50]:
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        c = dev["ctrl"][a0 * 3:a1 * 3].reshape(1, 3, a1 - a0).contiguous()
        w = dev["w"][a0:a1].reshape(1, a1 - a0).contiguous()
        single = host(bz.eval_rational(c, w, to_dev(b.t[o:o + 1]), method=method))
        sc = np.maximum(_extents(rb)[o], np.abs(ref[:, o * b.n_t:(o + 1) * b.n_t]))
        assert (np.abs(single - ref[:, o * b.n_t:(o + 1) * b.n_t]) / sc).max() <= TOL_F32


def test_signed_nurbs_weights_are_refused():
    b = bz_synth.mixed_batch(n_bezier=20, n_nurbs=4, n_t=4, seed=32)
    o = np.nonzero(b.kind_degree >> 8 == 2)[0][1]
    b.w[b.cp_offset[o] + 2] = -0.5
    with pytest.raises(bz.BzError) as e:
        _plan(b)
    assert e.value.code == bz.ERR_UNSUPPORTED


def _plan_uv(b, dtype=torch.float32, method="bernstein"):
    plan, dev = _plan(b, dtype=dtype, method=method)
    return plan, dev, to_dev(b.t), to_dev(b.v)


@pytest.mark.parametrize("method", ["bernstein", "decasteljau"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
@pytest.mark.parametrize("n_t", [16, 5])
def test_batch_with_patches(orc, method, dtype, n_t):
    """Surface patches of degree (1..3, 1..3) in the same persistent launch as
    curves, rational curves and NURBS (Sec. 2.2): every point against the
    oracle (on the rounded inputs for FP16 storage), for both lane mappings,
    both schedules and the window-major order."""
    b = bz_synth.mixed_batch(n_bezier=2000, n_nurbs=200, n_patches=900, n_t=n_t, patch_deg_lo=1, patch_deg_hi=3,
                             seed=60 + n_t)
    plan, dev, t, v = _plan_uv(b, dtype, method)
    rb = bz_synth.Batch(**{**b.__dict__})
    rb.ctrl = dev["ctrl"].float().cpu().numpy()
    rb.w = dev["w"].float().cpu().numpy()
    ref = orc.batch_eval(rb)
    ext = _extents(rb)
    assert plan.info()["n_classes"] == len(set(b.kind_degree.tolist()))
    assert _err(host(plan(t, v=v)), ref, ext, n_t) <= TOL_F32
    configs = [(300, 1, "static", 1, 0), (64, 2, "dynamic", 1, 500), (512, 4, "static", 1, 400)]
    if n_t % 4 == 0:
        configs += [(300, 4, "static", 4, 0), (512, 1, "dynamic", 4, 700)]
    for cfg in configs:
        plan.configure(*cfg)
        out = torch.full((3, b.n_obj * n_t), float("nan"), device=t.device)
        assert _err(host(plan(t, out=out, v=v)), ref, ext, n_t) <= TOL_F32, cfg


def test_batch_patches_need_v_and_degrees():
    b = bz_synth.mixed_batch(n_bezier=20, n_nurbs=2, n_patches=5, n_t=4, seed=61)
    plan, dev, t, v = _plan_uv(b)
    with pytest.raises(bz.BzError) as e:
        plan(t)  # no v for the patches
    assert e.value.code == bz.ERR_NULL
    plan(t, v=v)
    kd = b.kind_degree.copy()
    kd[np.nonzero(kd >> 8 == 3)[0][0]] = (3 << 8) | (4 << 4) | 1  # du = 4
    with pytest.raises(bz.BzError) as e:
        _plan(bz_synth.Batch(**{**b.__dict__, "kind_degree": kd}))
    assert e.value.code == bz.ERR_UNSUPPORTED


def test_autotune_with_patches(orc):
    b = bz_synth.mixed_batch(n_bezier=20000, n_nurbs=2000, n_patches=4000, n_t=16, seed=62)
    plan, dev, t, v = _plan_uv(b)
    out = torch.empty((3, b.n_obj * 16), device=t.device)
    plan.autotune(t, out)
    out.fill_(float("nan"))
    assert _err(host(plan(t, out=out, v=v)), orc.batch_eval(b), _extents(b), 16) <= TOL_F32


def test_config_batched_with_patches_sampled(orc):
    """The mixed workload plus 2^16 bicubic patches at 16 random (u, v) each,
    in one launch: a random sample of 16384 objects against the oracle."""
    b = bz_synth.mixed_batch(n_patches=1 << 16)
    kinds = b.kind_degree >> 8
    rng = np.random.default_rng(63)
    idx = np.unique(np.concatenate([rng.choice(b.n_obj, 16384, replace=False), [0, b.n_obj - 1],
                                    np.nonzero(kinds == 3)[0][[0, -1]]]))
    sub = b.subset(idx)
    plan, dev, t, v = _plan_uv(b)
    got = host(plan(t, v=v).view(3, b.n_obj, 16)[:, torch.from_numpy(idx).cuda()].reshape(3, -1))
    assert _err(got, orc.batch_eval(sub), _extents(sub), 16) <= TOL_F32
