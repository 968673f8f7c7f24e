"""GPU parity: texture-filter emulation (Sec. 2, Sec. 2.3, Sec. 4 with
Table 1, Fig. 3) and the zig-zag chain read through the emulated bilinear
filter (Sec. 2.1), against the FP64 oracle with the same FP32 weight rule."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import TOL_F32, bbox_err, extents, host, to_dev

pytestmark = pytest.mark.gpu

CASES = [("decasteljau", d) for d in range(2, 9)] + [("hybrid", d) for d in range(2, 9)] + \
        [("seiler", d) for d in range(2, 8)]


def _curves(n, d, dim, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, dim, d + 1)).astype(np.float32)


@pytest.mark.parametrize("mode,d", CASES)
def test_build_parity(orc, mode, d):
    ctrl = _curves(257, d, 3, 500 + d)
    got = host(bz.build_texture(to_dev(ctrl), mode))
    ref = orc.tex_build(ctrl, mode)
    assert got.shape == ref.shape == (257, 3, bz.texture_texels(d, mode))
    if mode != "seiler":
        np.testing.assert_array_equal(got, ref)
    else:  # FP64 texels rounded once to FP32: within one FP32 spacing
        assert (np.abs(got - ref) <= np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)).all()


@pytest.mark.parametrize("mode,d", CASES)
@pytest.mark.parametrize("frac_bits,rounding", [(8, "nearest"), (8, "truncate"), (0, "nearest"), (4, "nearest")])
def test_eval_parity(orc, mode, d, frac_bits, rounding):
    """Same FP32 textures on both sides; every weight decision must agree
    (one flip would cost ~2^-8 of the curve's extent, far above the
    tolerance).  Parameter counts ragged against the 256-thread blocks, and
    multiples of 64 (one curve per wavefront, scalar texel loads)."""
    n = 67
    rng = np.random.default_rng(510 + d + 20 * frac_bits)
    for dim, nt, nt_obj in ((3, 130, 7), (1, 130, 7), (3, 128, 64), (2, 64, 192)):
        ctrl = _curves(n, d, dim, 520 + d + dim)
        tex = orc.tex_build(ctrl, mode).astype(np.float32)
        t = np.concatenate([[0.0, 1.0, 0.5], rng.random(nt - 3)]).astype(np.float32)
        got = host(bz.eval_texture(to_dev(tex), d, mode, to_dev(t), frac_bits, rounding))
        ref = orc.tex_eval(tex, d, mode, t, False, frac_bits, rounding)
        assert bbox_err(got, ref, extents(ctrl), nt) <= TOL_F32, (dim, nt)
        tp = rng.random((n, nt_obj)).astype(np.float32)  # per-object parameters
        got = host(bz.eval_texture(to_dev(tex), d, mode, to_dev(tp), frac_bits, rounding))
        ref = orc.tex_eval(tex, d, mode, tp, True, frac_bits, rounding)
        assert bbox_err(got, ref, extents(ctrl), nt_obj) <= TOL_F32, (dim, nt_obj)


def test_eval_across_launch_chunks(orc):
    """2^18 + 5 cubic curve textures x 4096 t: more than 2^30 reads, so the
    call is split into launches of whole curves; the last 5 curves come in a
    second launch with its own texture and query offsets (12.9 GB of output).
    Curves on both sides of the boundary and at the ends, shared and
    per-curve t, de Casteljau and Seiler textures."""
    import torch
    n_t = 4096
    per = (1 << 30) // n_t
    n = per + 5
    rng = np.random.default_rng(93)
    ctrl = rng.random((n, 3, 4), dtype=np.float32) * 2.0 - 1.0
    pick = np.array([0, per - 1, per, per + 1, n - 1])
    idx = torch.from_numpy(pick).cuda()
    out = torch.empty((3, n * n_t), dtype=torch.float32, device="cuda")
    t_shared = rng.random(n_t, dtype=np.float32)
    t_per = rng.random((n, n_t), dtype=np.float32)
    for mode in ("decasteljau", "seiler"):
        tex = bz.build_texture(to_dev(ctrl), mode)
        tex_p = tex[idx].cpu().numpy()
        for t, per_object in ((t_shared, False), (t_per, True)):
            td = to_dev(t)
            out.fill_(float("nan"))
            bz.eval_texture(tex, 3, mode, td, 8, "nearest", out=out)
            got = out.view(3, n, n_t)[:, idx].reshape(3, -1).cpu().numpy()
            ref = orc.tex_eval(tex_p, 3, mode, t[pick] if per_object else t, per_object, 8, "nearest")
            assert bbox_err(got, ref, extents(ctrl[pick]), n_t) <= TOL_F32, (mode, per_object)
            del td
        del tex
    del out
    torch.cuda.empty_cache()


def test_eval_edges(orc):
    """Clamp-to-edge outside [0,1], endpoints, ties of the weight rule, NaN."""
    ctrl = _curves(9, 3, 2, 530)
    t = np.array([-1.0, 0.0, 1.0, 2.0, np.inf, -np.inf, np.nan, 0.5 / 256, 128.5 / 256, 255.5 / 256],
                 np.float32)
    for mode in ("decasteljau", "hybrid", "seiler"):
        tex = orc.tex_build(ctrl, mode).astype(np.float32)
        for rounding in ("nearest", "truncate"):
            got = host(bz.eval_texture(to_dev(tex), 3, mode, to_dev(t), 8, rounding))
            ref = orc.tex_eval(tex, 3, mode, t, False, 8, rounding)
            ok = ~np.isnan(ref)
            assert np.isnan(got[~ok]).all()
            assert np.abs(got[ok] - ref[ok]).max() <= 1e-6
            g = got.reshape(2, 9, -1)
            np.testing.assert_allclose(g[:, :, 0], g[:, :, 1], rtol=0, atol=1e-7)


def test_eval_fig3_errors_match_oracle(orc):
    """Fig. 3 workload shape: cubic curves, 8-bit nearest weights.  The GPU's
    deviation from the exact curve, per mode, is the oracle's (same weights),
    and the modes keep the oracle's order: hybrid < trilinear < Seiler."""
    ctrl = _curves(2048, 3, 3, 540)
    t = (np.arange(256) / 255).astype(np.float32)
    exact = orc.bezier_decasteljau(ctrl, t)
    ext = extents(ctrl)
    errs = {}
    for mode in ("decasteljau", "hybrid", "seiler"):
        tex = bz.build_texture(to_dev(ctrl), mode)
        got = host(bz.eval_texture(tex, 3, mode, to_dev(t), 8, "nearest"))
        ref = orc.tex_eval(host(tex).astype(np.float32), 3, mode, t, False, 8, "nearest")
        assert bbox_err(got, ref, ext, 256) <= TOL_F32
        errs[mode] = bbox_err(got, exact, ext, 256)
    assert errs["hybrid"] < errs["decasteljau"] < errs["seiler"]
    assert errs["seiler"] < 2 ** -6


def test_degree7_single_read_errors(orc):
    """Degree-7 curves from one 2x2x2 read at (t, st, (st)^2): exact with
    unrounded weights (to FP32), and the 8-bit rounding error the oracle
    predicts."""
    ctrl = _curves(512, 7, 3, 545)
    t = (np.arange(256) / 255).astype(np.float32)
    exact = orc.bezier_decasteljau(ctrl, t)
    tex = bz.build_texture(to_dev(ctrl), "seiler")
    for F in (0, 8):
        got = host(bz.eval_texture(tex, 7, "seiler", to_dev(t), F, "nearest"))
        ref = orc.tex_eval(host(tex).astype(np.float32), 7, "seiler", t, False, F, "nearest")
        assert bbox_err(got, ref, extents(ctrl), 256) <= TOL_F32
        if F == 0:
            assert bbox_err(got, exact, extents(ctrl), 256) <= 4 * TOL_F32


def test_errors():
    ctrl = to_dev(_curves(4, 3, 3, 550))
    tex = bz.build_texture(ctrl, "decasteljau")
    t = to_dev(np.zeros(8, np.float32))
    assert bz.texture_texels(8, "seiler") == 0 and bz.texture_texels(9, "decasteljau") == 0
    with pytest.raises(bz.BzError) as e:
        bz.build_texture(to_dev(_curves(4, 8, 3, 551)), "seiler")
    assert e.value.code == bz.ERR_UNSUPPORTED
    with pytest.raises(bz.BzError) as e:
        bz.eval_texture(tex, 3, "decasteljau", t, frac_bits=21)
    assert e.value.code == bz.ERR_SHAPE
    with pytest.raises(bz.BzError) as e:
        bz.check(bz.lib().bz_eval_texture(tex.data_ptr() + 4, 4, 3, 3, 0, t.data_ptr(), 8, 0, 8, 0,
                                          torch.empty(3 * 32, device=tex.device).data_ptr(), None))
    assert e.value.code == bz.ERR_ALIGN
    empty = bz.eval_texture(tex, 3, "decasteljau", to_dev(np.zeros(0, np.float32)))
    assert empty.shape == (3, 0)


# ------------------------------------------------------------ chain
@pytest.mark.parametrize("n_seg,dim,n_q", [(1, 3, 100), (7, 1, 1000), (1000, 3, 5003), (2048, 2, 70001),
                                           (777, 4, 4099)])
@pytest.mark.parametrize("frac_bits,rounding", [(8, "nearest"), (8, "truncate"), (0, "nearest")])
def test_chain_texemu_parity(orc, n_seg, dim, n_q, frac_bits, rounding):
    """Grid and cache-line tiles: the oracle's emulated filter, and the two
    placements bit-identical (same texels, same arithmetic)."""
    chain, T = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=n_q, seed=7 * n_seg + dim)
    grid = orc.piecewise_encode(chain).astype(np.float32)
    T = np.concatenate([T, np.arange(n_seg + 1, dtype=np.float32), [np.nan, -1.0, n_seg + 3.0]]).astype(np.float32)
    got = host(bz.eval_piecewise_texemu(to_dev(grid), to_dev(T), frac_bits, rounding))
    ref = orc.chain_texemu_eval(grid, T, frac_bits, rounding)
    ok = ~np.isnan(T)
    scale = max(float((chain.max(axis=0) - chain.min(axis=0)).max()), float(np.abs(grid).max()))
    assert np.abs(got[:, ok] - ref[:, ok]).max() <= TOL_F32 * scale
    assert np.isnan(got[:, ~ok]).all()
    tiles = bz.tile_piecewise(to_dev(grid))
    got_t = host(bz.eval_piecewise_texemu_tiled(tiles, n_seg, dim, to_dev(T), frac_bits, rounding))
    np.testing.assert_array_equal(got_t, got)


def test_chain_texemu_edges(orc):
    n_seg = 64
    chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=3, n_q=1, seed=560)
    grid = bz.encode_piecewise(to_dev(chain))
    T = np.array([-5.0, 0.0, 64.0, 70.0, np.inf, -np.inf, np.nan, 1 + 0.5 / 256, 3 + 100.5 / 256] +
                 list(range(65)), np.float32)
    got = host(bz.eval_piecewise_texemu(grid, to_dev(T)))
    ref = orc.chain_texemu_eval(host(grid).astype(np.float32), T)
    assert np.isnan(got[:, 6]).all()
    ok = np.arange(T.size) != 6
    assert np.abs(got[:, ok] - ref[:, ok]).max() <= 1e-5
    np.testing.assert_array_equal(got[:, 9:].T, chain[0::2])


def test_chain_texemu_full_size(orc):
    """2^20 segments, 2^24 random T, 8-bit nearest weights: every query
    against the oracle's emulated filter."""
    chain, T = bz_synth.chain_walk()
    grid = bz.encode_piecewise(to_dev(chain))
    got = host(bz.eval_piecewise_texemu(grid, to_dev(T)))
    gh = host(grid).astype(np.float32)
    ref = orc.chain_texemu_eval(gh, T)
    scale = max(float((chain.max(axis=0) - chain.min(axis=0)).max()), float(np.abs(gh).max()))
    assert np.abs(got - ref).max() / scale <= TOL_F32
    tiles = bz.tile_piecewise(grid)
    np.testing.assert_array_equal(host(bz.eval_piecewise_texemu_tiled(tiles, chain.shape[0] // 2, 3, to_dev(T))), got)


# ------------------------------------------------------------ surfaces
PATCH_CASES = [(du, dv) for du in (2, 3) for dv in (1, 2, 3, 4)]


def _patches(n, du, dv, dim, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, size=(n, dim, (du + 1) * (dv + 1))).astype(np.float32)


@pytest.mark.parametrize("du,dv", PATCH_CASES)
@pytest.mark.parametrize("mode", ["decasteljau", "seiler"])
def test_patch_build_parity(orc, du, dv, mode):
    P = _patches(123, du, dv, 3, 800 + du + 5 * dv)
    got = host(bz.build_texture_patch(to_dev(P), du, dv, mode))
    ref = orc.tex_patch_build(P, du, dv, mode)
    assert got.shape == ref.shape
    if mode == "decasteljau":
        np.testing.assert_array_equal(got, ref)
    else:
        assert (np.abs(got - ref) <= np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)).all()


@pytest.mark.parametrize("du,dv", PATCH_CASES)
@pytest.mark.parametrize("mode", ["decasteljau", "seiler"])
@pytest.mark.parametrize("frac_bits,rounding", [(8, "nearest"), (8, "truncate"), (0, "nearest")])
def test_patch_eval_parity(orc, du, dv, mode, frac_bits, rounding):
    rng = np.random.default_rng(810 + du + 5 * dv + frac_bits)
    for dim, n_per in ((3, 77), (1, 300), (4, 256)):
        P = _patches(19, du, dv, dim, 820 + du + dv + dim)
        tex = orc.tex_patch_build(P, du, dv, mode).astype(np.float32)
        uv = rng.random((19, n_per, 2)).astype(np.float32)
        uv[:, :3] = [[0, 0], [1, 1], [0.5, 0.25]]
        got = host(bz.eval_texture_patch(to_dev(tex), du, dv, mode, to_dev(uv), frac_bits, rounding))
        ref = orc.tex_patch_eval(tex, du, dv, mode, uv, frac_bits, rounding)
        assert bbox_err(got, ref, extents(P), n_per) <= TOL_F32, (dim, n_per)


def test_patch_fig3_style_errors(orc):
    """Bicubic patches, 8-bit nearest weights: the GPU's deviation from the
    exact surface per mode is the oracle's; de Casteljau (u rounded, v exact
    in the shader) errs less than Seiler (u, su and v rounded)."""
    P = bz_synth.patches(n_obj=1024)
    uv = np.random.default_rng(830).random((1024, 64, 2)).astype(np.float32)
    exact = orc.tensor_points(P, 3, 3, 0, uv)
    errs = {}
    for mode in ("decasteljau", "seiler"):
        tex = bz.build_texture_patch(to_dev(P), 3, 3, mode)
        got = host(bz.eval_texture_patch(tex, 3, 3, mode, to_dev(uv)))
        ref = orc.tex_patch_eval(host(tex).astype(np.float32), 3, 3, mode, uv)
        assert bbox_err(got, ref, extents(P), 64) <= TOL_F32
        errs[mode] = bbox_err(got, exact, extents(P), 64)
    assert errs["decasteljau"] < errs["seiler"] < 2 ** -5


def test_patch_errors():
    P = to_dev(_patches(3, 3, 3, 3, 840))
    assert bz.lib().bz_texture_patch_texels(4, 3, 0) == 0 and bz.lib().bz_texture_patch_texels(3, 3, 1) == 0
    with pytest.raises(bz.BzError) as e:
        bz.build_texture_patch(P, 3, 3, "hybrid")
    assert e.value.code == bz.ERR_UNSUPPORTED
    tex = bz.build_texture_patch(P, 3, 3, "seiler")
    with pytest.raises(bz.BzError) as e:
        bz.eval_texture_patch(tex, 3, 3, "seiler", to_dev(np.zeros((3, 4, 2), np.float32)), frac_bits=30)
    assert e.value.code == bz.ERR_SHAPE
