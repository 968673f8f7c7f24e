"""GPU parity: one frame of the particle ring (Sec. 5's particle test) in
each of the four position methods, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import host, to_dev

pytestmark = pytest.mark.gpu

METHODS = ["polynomial", "seiler", "seiler_texture", "table"]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("n,iters,dt", [(1, 0, 0.01), (1000, 3, 0.3), (70001, 64, 0.01), (4099, 300, 1.7)])
def test_frame_parity(orc, method, n, iters, dt):
    seg, T, speed = bz_synth.particle_ring(n_particles=n, seed=900 + n)
    seg_d = to_dev(seg)
    ring = bz.particle_ring_data(seg_d, method, 64)
    T_d = to_dev(T)
    pos, shade = bz.particles_step(method, ring, 16, T_d, to_dev(speed), dt, iters, 64)
    Tr, posr, shader = orc.particles_step(seg, T, speed, dt, method, iters, 64)
    # the phase update is the same FP32 arithmetic on both sides: bit-exact
    np.testing.assert_array_equal(host(T_d).astype(np.float32), Tr)
    assert np.abs(host(pos) - posr).max() <= 1e-5 * 2.0  # ring extent ~2
    assert np.abs(host(shade) - shader).max() <= 1e-5 * 2.0


def test_many_frames_stay_on_the_ring(orc):
    """60 frames: the GPU and oracle phases stay bit-identical frame by
    frame (same FP32 updates), and the polynomial positions stay on the ring."""
    seg, T, speed = bz_synth.particle_ring(n_particles=5000, seed=950)
    ring = bz.particle_ring_data(to_dev(seg), "polynomial")
    T_d, s_d = to_dev(T), to_dev(speed)
    Tr = T.copy()
    for _ in range(60):
        pos, _ = bz.particles_step("polynomial", ring, 16, T_d, s_d, 1 / 60, 0)
        Tr, posr, _ = orc.particles_step(seg, Tr, speed, 1 / 60, "polynomial", 0)
    np.testing.assert_array_equal(host(T_d).astype(np.float32), Tr)
    assert np.abs(host(pos) - posr).max() <= 2e-5


def test_full_size_frame(orc):
    """10M particles (the paper's largest count), K = 64, every method; a
    sample of 65536 particles checked against the oracle."""
    seg, T, speed = bz_synth.particle_ring(n_particles=10_000_000, seed=960)
    pick = np.random.default_rng(961).choice(T.shape[0], 65536, replace=False)
    for method in METHODS:
        ring = bz.particle_ring_data(to_dev(seg), method, 64)
        T_d = to_dev(T)
        pos, shade = bz.particles_step(method, ring, 16, T_d, to_dev(speed), 0.01, 64, 64)
        pidx = torch.from_numpy(pick).to(T_d.device)
        _, posr, shader = orc.particles_step(seg, T[pick], speed[pick], 0.01, method, 64, 64)
        assert np.abs(host(pos[:, pidx]) - posr).max() <= 2e-5, method
        assert np.abs(host(shade[pidx]) - shader).max() <= 2e-5, method


def test_errors():
    seg, T, speed = bz_synth.particle_ring(n_particles=10)
    ring = bz.particle_ring_data(to_dev(seg), "polynomial")
    T_d, s_d = to_dev(T), to_dev(speed)
    pos = torch.empty((3, 10), device=T_d.device)
    shade = torch.empty(10, device=T_d.device)
    with pytest.raises(bz.BzError) as e:
        bz.check(bz.lib().bz_particles_step(4, ring.data_ptr(), 16, 64, T_d.data_ptr(), s_d.data_ptr(), 0.01, 10, 0,
                                            pos.data_ptr(), shade.data_ptr(), None))
    assert e.value.code == bz.ERR_UNSUPPORTED
    with pytest.raises(bz.BzError) as e:
        bz.check(bz.lib().bz_particles_step(3, ring.data_ptr(), 16, 0, T_d.data_ptr(), s_d.data_ptr(), 0.01, 10, 0,
                                            pos.data_ptr(), shade.data_ptr(), None))
    assert e.value.code == bz.ERR_SHAPE


def test_ring_table_matches_curve_evaluation(orc):
    """The table entry point holds segment k at t = j/samples: against the
    oracle within 1e-5 of the ring's box, and within two FP32 ulps of the
    curve evaluator at the same parameters."""
    seg, _, _ = bz_synth.particle_ring(n_particles=16)
    ext = float((seg.max(axis=(0, 2)) - seg.min(axis=(0, 2))).max())
    for samples in (1, 7, 64):
        sd = to_dev(seg)
        got = host(bz.particle_ring_table(sd, samples))
        t = (np.arange(samples, dtype=np.float32) / np.float32(samples)).astype(np.float32)
        ref = orc.bezier_decasteljau(seg, t)
        assert np.abs(got - ref).max() <= 1e-5 * ext
        gpu = host(bz.eval_bezier(sd, to_dev(t)))
        np.testing.assert_allclose(got, gpu, rtol=0, atol=2 * 2.0 ** -23 * np.abs(gpu).max())
