"""GPU parity: tensor-product surfaces (grid and random points, VALU and
MFMA engines) and volumes against the FP64 oracle."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import TOL_F32, bbox_err, extents, host, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("du,dv", [(1, 1), (2, 3), (3, 3), (4, 2), (4, 4), (1, 4)])
@pytest.mark.parametrize("nu,nv", [(32, 32), (5, 16), (9, 7), (3, 33), (1, 1), (300, 8), (129, 2)])
def test_grid_valu(orc, du, dv, nu, nv):
    for dim in (3, 1, 4):
        P = bz_synth.patches(n_obj=19, du=du, dv=dv, dim=dim, seed=du * 10 + dv + dim)
        got = host(bz.eval_tensor_patch(to_dev(P), du, dv, nu=nu, nv=nv))
        ref = orc.tensor_grid(P, du, dv, nu, nv)
        assert bbox_err(got, ref, extents(P), nu * nv) <= TOL_F32, (dim, du, dv, nu, nv)


def test_grid_corners_exact():
    P = bz_synth.patches(n_obj=33, seed=3)
    got = host(bz.eval_tensor_patch(to_dev(P), 3, 3, nu=32, nv=32)).reshape(3, 33, 32, 32)
    for (a, b, idx) in ((0, 0, 0), (0, 31, 3), (31, 0, 12), (31, 31, 15)):
        np.testing.assert_array_equal(got[:, :, a, b], P[:, :, idx].T)


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_grid_low_precision_storage(orc, dtype):
    P = bz_synth.patches(n_obj=40, seed=4)
    Pd = to_dev(P).to(dtype)
    rounded = Pd.float().cpu().numpy()
    got = host(bz.eval_tensor_patch(Pd, 3, 3, nu=32, nv=32))
    assert bbox_err(got, orc.tensor_grid(rounded, 3, 3, 32, 32), extents(rounded), 1024) <= TOL_F32
    assert np.abs(got - orc.tensor_grid(P, 3, 3, 32, 32)).max() <= np.abs(rounded - P).max() + 2e-6


# bound for basis-matrix contraction with both operands rounded to a format of
# unit roundoff u: |sum (P+dP)(K+dK) - sum P K| <= 2u max|P| (sum K = 1),
# plus FP32 accumulation of 16 terms.
# FP16x3 keeps hi*hi + hi*lo + lo*hi: it is held to the FP32 tolerance.
MFMA_BOUNDS = {"mfma_f32": None, "mfma_bf16": 2 * 2.0 ** -9, "mfma_f16": 2 * 2.0 ** -11, "mfma_f16x3": None}


@pytest.mark.parametrize("engine", ["mfma_f32", "mfma_bf16", "mfma_f16", "mfma_f16x3"])
@pytest.mark.parametrize("n_obj,dim", [(1, 3), (11, 3), (43, 3), (64, 2), (9, 1), (17, 4)])
def test_grid_mfma(orc, engine, n_obj, dim):
    P = bz_synth.patches(n_obj=n_obj, dim=dim, seed=n_obj + 100 * dim)
    got = host(bz.eval_tensor_patch(to_dev(P), 3, 3, nu=32, nv=32, engine=engine))
    ref = orc.tensor_grid(P, 3, 3, 32, 32)
    u = MFMA_BOUNDS[engine]
    if u is None:
        assert bbox_err(got, ref, extents(P), 1024) <= TOL_F32
    else:
        assert np.abs(got - ref).max() <= u * np.abs(P).max() + 1e-5


@pytest.mark.parametrize("scale", [1e6, 1e-6, 3e30])
def test_grid_mfma_f16x3_row_scaling(orc, scale):
    """Control points far outside FP16's range (or deep in its subnormals):
    the per-row power-of-two scaling keeps the FP16x3 engine at FP32-class
    accuracy; each (patch, coordinate) row gets its own magnitude."""
    n, dim = 37, 3
    P = bz_synth.patches(n_obj=n, dim=dim, seed=77).astype(np.float64)
    rng = np.random.default_rng(78)
    P *= scale * np.exp2(rng.integers(-6, 7, size=(n, dim, 1)))
    P = P.astype(np.float32)
    got = host(bz.eval_tensor_patch(to_dev(P), 3, 3, nu=32, nv=32, engine="mfma_f16x3"))
    ref = orc.tensor_grid(P, 3, 3, 32, 32)
    assert np.isfinite(got).all()
    assert bbox_err(got, ref, extents(P), 1024) <= TOL_F32


def test_grid_config_full_size_sampled(orc):
    """2^18 bicubic patches on 32x32 grids (2^28 points): VALU and every MFMA
    engine (FP32, BF16, FP16, FP16x3) checked on 2048 sampled patches (every
    grid point); BF16 and FP16 against their rounding bound."""
    n = 1 << 18
    P = bz_synth.patches(n_obj=n)
    Pd = to_dev(P)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(n, size=2048, replace=False))
    ref = orc.tensor_grid(P[pick], 3, 3, 32, 32).reshape(3, 2048, 1024)
    out = torch.empty((3, n * 1024), dtype=torch.float32, device=Pd.device)
    for engine in ("valu", "mfma_f32", "mfma_bf16", "mfma_f16", "mfma_f16x3"):
        out.fill_(float("nan"))
        bz.eval_tensor_patch(Pd, 3, 3, nu=32, nv=32, engine=engine, out=out)
        got = out.view(3, n, 1024)[:, torch.from_numpy(pick).to(Pd.device)].cpu().numpy().astype(np.float64)
        if engine in ("mfma_bf16", "mfma_f16"):
            assert np.abs(got - ref).max() <= MFMA_BOUNDS[engine] * np.abs(P[pick]).max() + 1e-5, engine
        else:
            assert bbox_err(got.reshape(3, -1), ref.reshape(3, -1), extents(P[pick]), 1024) <= TOL_F32, engine
    del out


def test_grid_across_launch_chunks(orc):
    """2^22 + 40 bicubic patches: the grid engines launch at most 2^22 patches
    at a time, so the last 40 (a partial block of 32 and 8) come in a second
    launch with its own offsets into the control points and the 51.5 GB
    output planes.  Patches on both sides of the boundary and at the ends are
    checked for the VALU, FP32 and BF16 (four workgroups per block) engines."""
    n = (1 << 22) + 40
    P = bz_synth.patches(n_obj=n, seed=77)
    Pd = to_dev(P)
    pick = np.array([0, 1, 31, 32, (1 << 22) - 33, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, (1 << 22) + 31,
                     (1 << 22) + 32, n - 1])
    ref = orc.tensor_grid(P[pick], 3, 3, 32, 32).reshape(3, len(pick), 1024)
    idx = torch.from_numpy(pick).to(Pd.device)
    out = torch.empty((3, n * 1024), dtype=torch.float32, device=Pd.device)
    for engine in ("valu", "mfma_f32", "mfma_bf16"):
        out.fill_(float("nan"))
        bz.eval_tensor_patch(Pd, 3, 3, nu=32, nv=32, engine=engine, out=out)
        got = out.view(3, n, 1024)[:, idx].cpu().numpy().astype(np.float64)
        if engine == "mfma_bf16":
            assert np.abs(got - ref).max() <= MFMA_BOUNDS[engine] + 1e-5, engine
        else:
            assert bbox_err(got.reshape(3, -1), ref.reshape(3, -1), extents(P[pick]), 1024) <= TOL_F32, engine
    del out, Pd
    torch.cuda.empty_cache()


def test_points_across_launch_chunks(orc):
    """2^22 + 5 objects: random-point evaluation launches at most 2^22 objects
    at a time, so the last 5 come in a second launch with its own offsets into
    the control points, the parameters and the output planes (stride n *
    n_per).  Bicubic patches and tricubic volumes (Bernstein and per-axis
    Seiler form), objects on both sides of the boundary and at the ends."""
    n = (1 << 22) + 5
    rng = np.random.default_rng(55)
    pick = np.array([0, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, n - 1])
    idx = torch.from_numpy(pick).cuda()
    for du, dv, dw, n_per in ((3, 3, 0, 3), (3, 3, 3, 1)):
        ncp = (du + 1) * (dv + 1) * (dw + 1)
        P = rng.random((n, 3, ncp), dtype=np.float32) * 2.0 - 1.0
        uvw = rng.random((n, n_per, 3 if dw else 2), dtype=np.float32)
        ref = orc.tensor_points(P[pick], du, dv, dw, uvw[pick])
        Pd, ud = to_dev(P), to_dev(uvw)
        got = bz.eval_tensor_patch(Pd, du, dv, dw, uvw=ud).view(3, n, n_per)[:, idx].reshape(3, -1).cpu().numpy()
        assert bbox_err(got, ref, extents(P[pick]), n_per) <= TOL_F32, (du, dv, dw)
        if dw:
            sc = bz.tensor_to_seiler(Pd, du, dv, dw)
            got = bz.eval_tensor_seiler(sc, du, dv, dw, uvw=ud).view(3, n, n_per)[:, idx].reshape(3, -1).cpu().numpy()
            assert bbox_err(got, ref, extents(P[pick]), n_per) <= TOL_F32, "seiler"
            del sc
        del Pd, ud, P
    torch.cuda.empty_cache()


@pytest.mark.parametrize("degs", [(3, 3, 0), (1, 1, 0), (2, 4, 0), (3, 3, 3), (1, 1, 1), (4, 2, 3), (2, 2, 2)])
@pytest.mark.parametrize("n_per", [1, 100, 256, 300])
def test_points(orc, degs, n_per):
    du, dv, dw = degs
    ncp = (du + 1) * (dv + 1) * (dw + 1)
    rng = np.random.default_rng(du + 7 * dv + 49 * dw + n_per)
    for dim in (3, 2):
        P = rng.uniform(-1, 1, size=(13, dim, ncp)).astype(np.float32)
        uvw = rng.random((13, n_per, 3 if dw else 2)).astype(np.float32)
        got = host(bz.eval_tensor_patch(to_dev(P), du, dv, dw, uvw=to_dev(uvw)))
        ref = orc.tensor_points(P, du, dv, dw, uvw)
        assert bbox_err(got, ref, extents(P), n_per) <= TOL_F32


def test_volume_config_full_size_sampled(orc):
    """2^16 tricubic volumes at 2^24 random (u,v,w): the first 1024 volumes'
    256 queries each checked against the oracle."""
    ctrl, uvw = bz_synth.volumes()
    got = bz.eval_tensor_patch(to_dev(ctrl), 3, 3, 3, uvw=to_dev(uvw))
    g = host(got.view(3, 1 << 16, 256)[:, :1024]).reshape(3, -1)
    ref = orc.tensor_points(ctrl[:1024], 3, 3, 3, uvw[:1024])
    assert bbox_err(g, ref, extents(ctrl[:1024]), 256) <= TOL_F32


def test_tensor_errors():
    P = to_dev(bz_synth.patches(n_obj=2))
    with pytest.raises(bz.BzError) as e:
        bz.eval_tensor_patch(P, 3, 3, nu=16, nv=16, engine="mfma_bf16")
    assert e.value.code == bz.ERR_UNSUPPORTED
    with pytest.raises(bz.BzError) as e:
        bz.eval_tensor_patch(P, 5, 3, nu=4, nv=4)
    assert e.value.code == bz.ERR_SHAPE
