"""GPU parity: zig-zag encoding and random-access evaluation of C0
quadratic chains (Sec. 2.1) against the FP64 oracle."""
import numpy as np
import pytest

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import TOL_F32, host, to_dev

pytestmark = pytest.mark.gpu


def _chain_extent(chain):
    c = np.asarray(chain, np.float64)
    return float((c.max(axis=0) - c.min(axis=0)).max())


@pytest.mark.parametrize("n_seg,dim", [(1, 3), (2, 1), (1000, 3), (4097, 2), (3001, 4)])
def test_encode_parity(orc, n_seg, dim):
    chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=n_seg)
    grid = host(bz.encode_piecewise(to_dev(chain)))
    ref = orc.piecewise_encode(chain)
    assert grid.shape == (n_seg + 1, 2, dim)
    ext = _chain_extent(chain)
    # on-path texels are copies: bit-exact
    for k in range(n_seg + 1):
        np.testing.assert_array_equal(grid[k, k & 1], chain[2 * k])
    # free texels: one FP32 rounding of an FP64 alternating sum
    assert np.abs(grid - ref).max() <= 1e-6 * max(ext, np.abs(ref).max())
    x = np.array([grid[k, 1 - (k & 1)] for k in range(n_seg + 1)])
    np.testing.assert_allclose((x[:-1] + x[1:]) / 2, chain[1::2][:n_seg], rtol=0,
                               atol=2e-7 * max(1.0, np.abs(x).max()))


@pytest.mark.parametrize("n_seg,dim,n_q", [(1, 3, 100), (5, 1, 1000), (1000, 3, 5003), (2048, 2, 70001),
                                           (777, 4, 4099)])
def test_eval_parity(orc, n_seg, dim, n_q):
    chain, T = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=n_q, seed=3 * n_seg + dim)
    grid = orc.piecewise_encode(chain).astype(np.float32)
    got = host(bz.eval_piecewise(to_dev(grid), to_dev(T)))
    ref = orc.piecewise_eval(grid, T)
    ext = _chain_extent(chain)
    assert np.abs(got - ref).max() <= TOL_F32 * ext
    # same answer as the chain's plain definition
    ref2 = orc.chain_eval(chain, T)
    assert np.abs(got - ref2).max() <= TOL_F32 * ext


def test_eval_edges(orc):
    """Clamping, T = N, integer T (exact vertices), NaN."""
    n_seg = 64
    chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=3, n_q=1, seed=5)
    grid = bz.encode_piecewise(to_dev(chain))
    T = np.array([-5.0, 0.0, 64.0, 70.0, np.inf, -np.inf, np.nan, 0.5, 63.999996] + list(range(65)), np.float32)
    got = host(bz.eval_piecewise(grid, to_dev(T)))
    np.testing.assert_array_equal(got[:, 0], chain[0])
    np.testing.assert_array_equal(got[:, 1], chain[0])
    np.testing.assert_array_equal(got[:, 2], chain[2 * n_seg])
    np.testing.assert_array_equal(got[:, 3], chain[2 * n_seg])
    np.testing.assert_array_equal(got[:, 4], chain[2 * n_seg])
    np.testing.assert_array_equal(got[:, 5], chain[0])
    assert np.isnan(got[:, 6]).all()
    # C0: at every integer T the chain passes exactly through the shared vertex
    np.testing.assert_array_equal(got[:, 9:].T, chain[0::2])
    ref = orc.piecewise_eval(host(grid), T[7:9])
    np.testing.assert_allclose(got[:, 7:9], ref, rtol=0, atol=1e-5)


def test_encode_then_eval_full_chain_config(orc):
    """2^20 segments, 2^24 random global parameters: GPU encode + GPU eval
    against the oracle's chain definition at every query."""
    chain, T = bz_synth.chain_walk()
    grid = bz.encode_piecewise(to_dev(chain))
    got = host(bz.eval_piecewise(grid, to_dev(T)))
    ref = orc.chain_eval(chain, T)
    ext = _chain_extent(chain)
    err = np.abs(got - ref).max() / ext
    assert err <= TOL_F32, err
    del got, ref
    # storage: 2(N+1) texels
    assert grid.shape[0] * grid.shape[1] == 2 * ((chain.shape[0] - 1) // 2 + 1)


def _tiles_reference(grid):
    """Host re-tiling of a grid (plain index arithmetic): 128-byte tiles of
    C = 128/(8*dim) columns overlapping by one column, zero padded."""
    n_seg, dim = grid.shape[0] - 1, grid.shape[2]
    C = 128 // (8 * dim)
    S = C - 1
    n_tiles = -(-n_seg // S)
    tiles = np.zeros((n_tiles, 32), np.float32)
    flat = grid.reshape(n_seg + 1, 2 * dim)
    for j in range(n_tiles):
        cols = flat[j * S: j * S + C]
        tiles[j, :cols.size] = cols.reshape(-1)
    return tiles.reshape(-1)


@pytest.mark.parametrize("n_seg,dim", [(1, 3), (4, 3), (5, 3), (1000, 3), (77, 1), (300, 2), (129, 4)])
def test_tiled_layout_and_eval(orc, n_seg, dim):
    chain, T = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=3001, seed=7 * n_seg + dim)
    grid = bz.encode_piecewise(to_dev(chain))
    tiles = bz.tile_piecewise(grid)
    np.testing.assert_array_equal(host(tiles), _tiles_reference(host(grid)))
    T = np.concatenate([T, np.array([0, n_seg, -1, n_seg + 3, np.nan], np.float32),
                        np.arange(n_seg + 1, dtype=np.float32)])
    got = host(bz.eval_piecewise_tiled(tiles, n_seg, dim, to_dev(T)))
    ref_grid = host(bz.eval_piecewise(grid, to_dev(T)))
    np.testing.assert_array_equal(got, ref_grid)  # same texels, same arithmetic
    ok = ~np.isnan(T)
    ref = orc.chain_eval(chain, T[ok])
    assert np.abs(got[:, ok] - ref).max() <= TOL_F32 * _chain_extent(chain)
    assert np.isnan(got[:, ~ok]).all()


def test_tiled_full_chain_config(orc):
    chain, T = bz_synth.chain_walk()
    grid = bz.encode_piecewise(to_dev(chain))
    tiles = bz.tile_piecewise(grid)
    got = host(bz.eval_piecewise_tiled(tiles, grid.shape[0] - 1, 3, to_dev(T)))
    ref = orc.chain_eval(chain, T)
    assert np.abs(got - ref).max() / _chain_extent(chain) <= TOL_F32


# ---------------------------------------------------------------- 16-bit texels
UNIT16 = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}  # unit roundoff of round-to-nearest-even


def _round16(x, dtype):
    """FP32 values rounded to FP16 / BF16 (nearest even), as FP64; and the bits."""
    x = np.asarray(x, np.float32)
    if dtype == "f16":
        h = x.astype(np.float16)
        return h.astype(np.float64), h.view(np.uint16)
    u = x.view(np.uint32).astype(np.uint64)
    b = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64), b


def _tiles16_reference(grid, dtype):
    """Expected 16-bit tile bits: columns j*S .. j*S+S of the grid, S = 32/dim - 1."""
    n_seg, _, dim = grid.shape[0] - 1, 2, grid.shape[2]
    S = 32 // dim - 1
    n_tiles = -(-n_seg // S)
    bits = _round16(grid, dtype)[1]
    tiles = np.zeros((n_tiles, 64), np.uint16)
    for j in range(n_tiles):
        cols = bits[j * S: min(j * S + S + 1, n_seg + 1)]
        tiles[j, :cols.size] = cols.reshape(-1)
    return tiles.reshape(-1)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("n_seg,dim", [(1, 3), (9, 3), (10, 3), (1000, 3), (77, 1), (300, 2), (129, 4)])
def test_tiled16_layout_and_eval(orc, dtype, n_seg, dim):
    """16-bit texel tiles: layout bit-exact; results against the oracle's
    chain evaluation on its own grid rounded to the texel type (they differ
    only where the FP64 texel sits on an FP32 rounding tie, by at most one
    16-bit unit of a free texel, whose weight is at most 1/4), and the
    stated bound against the exact chain: u times the largest |texel|."""
    import torch
    chain, T = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=3001, seed=11 * n_seg + dim)
    grid = bz.encode_piecewise(to_dev(chain))
    tiles = bz.tile_piecewise16(grid, torch.float16 if dtype == "f16" else torch.bfloat16)
    torch.cuda.synchronize()
    bits = tiles.view(torch.int16).cpu().numpy().view(np.uint16)  # the raw texel bits
    np.testing.assert_array_equal(bits, _tiles16_reference(host(grid), dtype))
    T = np.concatenate([T, np.array([0, n_seg, -1, n_seg + 3, np.nan], np.float32),
                        np.arange(n_seg + 1, dtype=np.float32)])
    got = host(bz.eval_piecewise_tiled16(tiles, n_seg, dim, to_dev(T)))
    ok = ~np.isnan(T)
    rg = _round16(orc.piecewise_encode(chain).astype(np.float32), dtype)[0]
    u, xmax, ext = UNIT16[dtype], float(np.abs(rg).max()), _chain_extent(chain)
    ref_r = orc.piecewise_eval(rg, T[ok])
    assert np.abs(got[:, ok] - ref_r).max() <= 0.5 * u * xmax + TOL_F32 * ext
    ref = orc.chain_eval(chain, T[ok])
    assert np.abs(got[:, ok] - ref).max() <= u * xmax + TOL_F32 * ext
    assert np.isnan(got[:, ~ok]).all()


def test_tiled16_full_chain_config(orc):
    """The bench's chain (2^20 segments, 2^24 random T) with FP16 texels:
    every query against the FP32 tiles (the difference is the texel
    rounding alone, within u times the largest |texel| of the chain), and a
    seeded sample of 2^18 queries against the oracle's chain."""
    import torch
    chain, T = bz_synth.chain_walk()
    n_seg = (chain.shape[0] - 1) // 2
    grid = bz.encode_piecewise(to_dev(chain))
    T_d = to_dev(T)
    got = bz.eval_piecewise_tiled16(bz.tile_piecewise16(grid, torch.float16), n_seg, 3, T_d)
    f32 = bz.eval_piecewise_tiled(bz.tile_piecewise(grid), n_seg, 3, T_d)
    xmax = float(grid.abs().max().item())
    assert float((got - f32).abs().max().item()) <= UNIT16["f16"] * xmax + 1e-6 * xmax
    pick = np.random.default_rng(5).choice(T.size, 1 << 18, replace=False)
    ref = orc.chain_eval(chain, T[pick])
    g = host(got)[:, pick]
    assert np.abs(g - ref).max() <= UNIT16["f16"] * xmax + TOL_F32 * _chain_extent(chain)


def test_chains_across_launch_chunks(orc):
    """2^30 + 777 queries in 2D: the chain evaluators launch at most 2^30
    queries at a time, so the last 777 come in a second launch that reads T
    and writes both output planes (stride n_q) at its own offset.  The
    quadratic chain (grid and tiled layouts, and the tiles through the
    emulated texture filter) and the two-layer cubic chain (tiled) are checked at queries on both sides of the boundary and at the
    ends.  T is drawn on the GPU from a seeded generator and the sampled
    values are read back for the oracle."""
    import torch
    n_seg, dim = 1000, 2
    n_q = (1 << 30) + 777
    g = torch.Generator(device="cuda")
    g.manual_seed(123)
    T = torch.rand(n_q, generator=g, device="cuda", dtype=torch.float32) * n_seg
    pick = np.array([0, 1, (1 << 30) - 2, (1 << 30) - 1, 1 << 30, (1 << 30) + 1, n_q - 1])
    idx = torch.from_numpy(pick).cuda()
    Tp = T[idx].cpu().numpy()
    out = torch.empty((dim, n_q), dtype=torch.float32, device="cuda")
    chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=5)
    grid = bz.encode_piecewise(to_dev(chain))
    tiles = bz.tile_piecewise(grid)
    ref = orc.chain_eval(chain, Tp)
    for name, run in (("grid", lambda: bz.eval_piecewise(grid, T, out=out)),
                      ("tiled", lambda: bz.eval_piecewise_tiled(tiles, n_seg, dim, T, out=out))):
        out.fill_(float("nan"))
        run()
        got = out[:, idx].cpu().numpy()
        assert np.abs(got - ref).max() / _chain_extent(chain) <= TOL_F32, name
    # the same tiles read through the emulated 8-bit bilinear filter
    gh = host(grid).astype(np.float32)
    tref = orc.chain_texemu_eval(gh, Tp, 8, "nearest")
    out.fill_(float("nan"))
    bz.eval_piecewise_texemu_tiled(tiles, n_seg, dim, T, 8, "nearest", out=out)
    got = out[:, idx].cpu().numpy()
    scale = max(_chain_extent(chain), float(np.abs(gh).max()))
    assert np.abs(got - tref).max() <= TOL_F32 * scale, "texture emulation"
    cchain, _ = bz_synth.cubic_chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=6)
    ctiles = bz.tile_piecewise_cubic(bz.encode_piecewise_cubic(to_dev(cchain)))
    out.fill_(float("nan"))
    bz.eval_piecewise_cubic_tiled(ctiles, n_seg, dim, T, out=out)
    got = out[:, idx].cpu().numpy()
    cref = orc.cubic_chain_eval(cchain, Tp)
    assert np.abs(got - cref).max() / _chain_extent(cchain) <= TOL_F32, "cubic"
    del out, T
    torch.cuda.empty_cache()
