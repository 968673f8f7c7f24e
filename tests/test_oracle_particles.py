"""Pins for the oracle's particle-ring frame (Sec. 5's particle test:
particles moving along cubic Bezier curves chained into a ring)."""
import numpy as np
import pytest

import bz_synth

A, B, C, D = 23 / 32, 0.25, -0.125, 0.0625


def _frame(orc, method, iters=8, n=4000, samples=64, dt=0.01):
    seg, T, speed = bz_synth.particle_ring(n_particles=n)
    Tn, pos, shade = orc.particles_step(seg, T, speed, dt, method, iters, samples)
    return seg, T, speed, Tn, pos, shade


def _on_ring(orc, seg, Tn):
    """The ring's definition at the new phases: segment floor(T), local T - k."""
    k = np.minimum(np.floor(Tn.astype(np.float64)).astype(np.int64), seg.shape[0] - 1)
    t = Tn.astype(np.float64) - k
    out = np.empty((3, Tn.shape[0]))
    for s in np.unique(k):
        m = k == s
        out[:, m] = orc.bezier_decasteljau(seg[s:s + 1], t[m])
    return out


def test_ring_is_closed_and_c0():
    seg, _, _ = bz_synth.particle_ring(n_seg=16, n_particles=1)
    for k in range(16):
        np.testing.assert_array_equal(seg[k, :, 3], seg[(k + 1) % 16, :, 0])
    np.testing.assert_allclose(np.linalg.norm(seg[:, :, 0], axis=1), 1.0, rtol=1e-6)


def test_phase_update_wraps(orc):
    seg, T, speed, Tn, _, _ = _frame(orc, "polynomial", dt=0.37)
    assert (Tn >= 0).all() and (Tn < 16).all()
    step = (T.astype(np.float64) + speed.astype(np.float64) * 0.37) % 16
    d = np.abs(Tn - step)
    assert np.minimum(d, 16 - d).max() < 1e-5
    assert ((T.astype(np.float64) + speed * 0.37) >= 16).any()  # some particles did wrap


@pytest.mark.parametrize("method", ["polynomial", "seiler"])
def test_exact_methods_are_the_ring(orc, method):
    seg, _, _, Tn, pos, _ = _frame(orc, method)
    np.testing.assert_allclose(pos, _on_ring(orc, seg, Tn), rtol=0, atol=1e-13)


def test_consumer_closed_form(orc):
    """v_K = drive (1 - a^K) / (1 - a), drive = b x + c y + d z."""
    for K in (0, 1, 7, 64):
        _, _, _, _, pos, shade = _frame(orc, "polynomial", iters=K)
        drive = B * pos[0] + C * pos[1] + D * pos[2]
        np.testing.assert_allclose(shade, drive * (1 - A ** K) / (1 - A), rtol=0, atol=1e-13)


def test_table_method(orc):
    """The sampled table is exact at its samples and within the linear
    interpolation bound |C''| h^2 / 8 (h = 1/S, |C''| <= 6 max |second
    difference|) elsewhere; it wraps around the ring."""
    seg, T, speed = bz_synth.particle_ring(n_particles=1)
    S = 64
    Tg = (np.arange(16 * S) / S).astype(np.float32)
    Tn, pos, _ = orc.particles_step(seg, Tg, np.zeros_like(Tg), 0.0, "table", 0, S)
    np.testing.assert_array_equal(Tn, Tg)
    np.testing.assert_allclose(pos, _on_ring(orc, seg, Tn), rtol=0, atol=1e-13)
    seg, _, _, Tn, pos, _ = _frame(orc, "table", samples=S, n=20000)
    d2 = np.abs(seg[:, :, 2:] - 2 * seg[:, :, 1:-1] + seg[:, :, :-2]).max()
    err = np.abs(pos - _on_ring(orc, seg, Tn)).max()
    assert 1e-6 < err <= 6 * d2 / (8 * S * S) + 1e-6
    Tw = np.array([16 - 1e-4, 15.99, 0.0], np.float32)
    Tw2, pw, _ = orc.particles_step(seg, Tw, np.zeros(3, np.float32), 0.0, "table", 0, S)
    np.testing.assert_allclose(pw[:, 0], pw[:, 2], atol=1e-3)  # the last sample interval closes the ring


def test_seiler_texture_method_is_the_emulated_read(orc):
    """Method 2 is the segment's Seiler texture read through the emulated
    8-bit filter (the texture-emulation oracle, pinned on its own)."""
    seg, _, _, Tn, pos, _ = _frame(orc, "seiler_texture")
    k = np.minimum(np.floor(Tn).astype(np.int64), 15)
    t = (Tn - k.astype(np.float32)).astype(np.float32)
    tex = orc.tex_build(seg, "seiler").astype(np.float64)
    for s in range(16):
        m = k == s
        ref = orc.tex_eval(tex[s:s + 1], 3, "seiler", t[m], frac_bits=8)
        np.testing.assert_allclose(pos[:, m], ref, rtol=0, atol=2e-7)
    err = np.abs(pos - _on_ring(orc, seg, Tn)).max()
    assert 1e-4 < err < 0.02
