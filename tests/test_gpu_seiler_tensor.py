"""GPU parity: Seiler surfaces and volumes (per-axis Seiler terms, Sec. 3 on
each axis of the Sec. 2.2 tensor product) against the FP64 oracle."""
import numpy as np
import pytest

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import TOL_F32, bbox_err, extents, host, to_dev

pytestmark = pytest.mark.gpu

DEGS = [(1, 1, 0), (3, 3, 0), (2, 4, 0), (4, 4, 0), (3, 3, 3), (1, 2, 3), (4, 4, 4), (2, 1, 1), (4, 1, 2)]


def _net(rng, n, dim, du, dv, dw):
    return rng.uniform(-1, 1, size=(n, dim, (du + 1) * (dv + 1) * (dw + 1))).astype(np.float32)


@pytest.mark.parametrize("degs", DEGS)
def test_conversion_parity(orc, degs):
    du, dv, dw = degs
    rng = np.random.default_rng(700 + du + 5 * dv + 25 * dw)
    P = _net(rng, 300, 3, du, dv, dw)
    got = host(bz.tensor_to_seiler(to_dev(P), du, dv, dw))
    ref = orc.tensor_to_seiler(P, du, dv, dw)
    # FP64 terms rounded once: within one FP32 spacing of the oracle's
    assert (np.abs(got - ref) <= np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)).all()


@pytest.mark.parametrize("degs", DEGS)
@pytest.mark.parametrize("n_per", [1, 100, 256, 300])
def test_points_parity(orc, degs, n_per):
    du, dv, dw = degs
    rng = np.random.default_rng(710 + du + 5 * dv + 25 * dw + n_per)
    for dim in (3, 1):
        P = _net(rng, 13, dim, du, dv, dw)
        sc = orc.tensor_to_seiler(P, du, dv, dw).astype(np.float32)
        uvw = rng.random((13, n_per, 3 if dw else 2)).astype(np.float32)
        got = host(bz.eval_tensor_seiler(to_dev(sc), du, dv, dw, uvw=to_dev(uvw)))
        ref = orc.tensor_seiler_points(sc, du, dv, dw, uvw)
        assert bbox_err(got, ref, extents(P), n_per) <= TOL_F32
        # and the surface / volume itself (Bernstein oracle on the control points)
        assert bbox_err(got, orc.tensor_points(P, du, dv, dw, uvw), extents(P), n_per) <= TOL_F32


@pytest.mark.parametrize("du,dv,nu,nv", [(3, 3, 32, 32), (2, 4, 7, 9), (1, 1, 2, 2), (4, 3, 16, 64), (3, 2, 5, 300)])
def test_grid_parity(orc, du, dv, nu, nv):
    rng = np.random.default_rng(720 + du + 5 * dv)
    P = _net(rng, 11, 3, du, dv, 0)
    sc = bz.tensor_to_seiler(to_dev(P), du, dv)
    got = host(bz.eval_tensor_seiler(sc, du, dv, nu=nu, nv=nv))
    ref = orc.tensor_seiler_grid(host(sc).astype(np.float32), du, dv, nu, nv)
    assert bbox_err(got, ref, extents(P), nu * nv) <= TOL_F32
    assert bbox_err(got, orc.tensor_grid(P, du, dv, nu, nv), extents(P), nu * nv) <= TOL_F32


def test_volume_config_full_size_sampled(orc):
    """2^16 tricubic volumes at 2^24 random (u,v,w) in Seiler form: the first
    1024 volumes' 256 queries each against the oracle."""
    ctrl, uvw = bz_synth.volumes()
    sc = bz.tensor_to_seiler(to_dev(ctrl), 3, 3, 3)
    got = bz.eval_tensor_seiler(sc, 3, 3, 3, uvw=to_dev(uvw))
    g = host(got.view(3, 1 << 16, 256)[:, :1024]).reshape(3, -1)
    ref = orc.tensor_points(ctrl[:1024], 3, 3, 3, uvw[:1024])
    assert bbox_err(g, ref, extents(ctrl[:1024]), 256) <= TOL_F32


def test_errors():
    P = to_dev(bz_synth.patches(n_obj=2))
    with pytest.raises(bz.BzError) as e:
        bz.tensor_to_seiler(P, 5, 3)
    assert e.value.code == bz.ERR_SHAPE
    sc = bz.tensor_to_seiler(P, 3, 3)
    with pytest.raises(bz.BzError) as e:
        bz.eval_tensor_seiler(sc.reshape(2, 3, 16), 3, 3, 0, nu=0, nv=4)
    assert e.value.code == bz.ERR_SHAPE
