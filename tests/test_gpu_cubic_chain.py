"""GPU parity: C0 piecewise cubic chains as two stacked zig-zag layers
(Sec. 2.1, two C0 quadratic textures interpolated in depth) against the
FP64 oracle."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import TOL_F32, host, to_dev

pytestmark = pytest.mark.gpu


def _extent(chain):
    c = np.asarray(chain, np.float64)
    return float((c.max(axis=0) - c.min(axis=0)).max())


@pytest.mark.parametrize("n_seg,dim", [(1, 3), (2, 1), (1000, 3), (4097, 2), (3001, 4)])
def test_cubic_encode_parity(orc, n_seg, dim):
    chain, _ = bz_synth.cubic_chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=n_seg + 7)
    grid = host(bz.encode_piecewise_cubic(to_dev(chain)))
    ref = orc.cubic_chain_encode(chain)
    assert grid.shape == (n_seg + 1, 2, 2, dim)
    # shared endpoints are copies in both layers: bit-exact
    for k in range(n_seg + 1):
        for layer in (0, 1):
            np.testing.assert_array_equal(grid[k, layer, k & 1], chain[3 * k])
    # free texels: one FP32 rounding of an FP64 alternating sum
    assert np.abs(grid - ref).max() <= 1e-6 * max(_extent(chain), np.abs(ref).max())


@pytest.mark.parametrize("n_seg,dim,n_q", [(1, 3, 100), (5, 1, 1000), (1000, 3, 5003), (2048, 2, 70001),
                                           (777, 4, 4099)])
def test_cubic_eval_parity(orc, n_seg, dim, n_q):
    chain, T = bz_synth.cubic_chain_walk(n_seg=n_seg, dim=dim, n_q=n_q, seed=5 * n_seg + dim)
    grid = orc.cubic_chain_encode(chain).astype(np.float32)
    got = host(bz.eval_piecewise_cubic(to_dev(grid), to_dev(T)))
    ext = _extent(chain)
    ref = orc.cubic_chain_grid_eval(grid, T)
    assert np.abs(got - ref).max() <= TOL_F32 * ext
    ref2 = orc.cubic_chain_eval(chain, T)
    assert np.abs(got - ref2).max() <= TOL_F32 * ext


def test_cubic_eval_edges(orc):
    """Clamping, T = N, integer T (exact shared endpoints), NaN."""
    n_seg = 64
    chain, _ = bz_synth.cubic_chain_walk(n_seg=n_seg, dim=3, n_q=1, seed=21)
    grid = bz.encode_piecewise_cubic(to_dev(chain))
    T = np.array([-5.0, 0.0, 64.0, 70.0, np.inf, -np.inf, np.nan, 0.5, 63.999996] + list(range(65)), np.float32)
    got = host(bz.eval_piecewise_cubic(grid, to_dev(T)))
    for col, row in ((0, 0), (1, 0), (2, 3 * n_seg), (3, 3 * n_seg), (4, 3 * n_seg), (5, 0)):
        np.testing.assert_array_equal(got[:, col], chain[row])
    assert np.isnan(got[:, 6]).all()
    np.testing.assert_array_equal(got[:, 9:].T, chain[0::3])
    ref = orc.cubic_chain_eval(chain, T[7:9])
    np.testing.assert_allclose(got[:, 7:9], ref, rtol=0, atol=1e-5 * _extent(chain))


def test_cubic_empty_and_errors():
    chain, _ = bz_synth.cubic_chain_walk(n_seg=4, dim=3, n_q=1, seed=3)
    grid = bz.encode_piecewise_cubic(to_dev(chain))
    out = bz.eval_piecewise_cubic(grid, to_dev(np.zeros(0, np.float32)))
    assert out.shape == (3, 0)
    # zero segments, and a grid lacking 16-byte alignment, are rejected
    T = to_dev(np.zeros(4, np.float32))
    with pytest.raises(bz.BzError) as e:
        bz.eval_piecewise_cubic(grid[:1], T)
    assert e.value.code == bz.ERR_SHAPE
    flat = grid.reshape(-1)
    with pytest.raises(bz.BzError) as e:
        bz.check(bz.lib().bz_eval_piecewise_cubic(flat[1:].data_ptr(), 4, 3, T.data_ptr(), 4,
                                                   bz.eval_piecewise_cubic(grid, T).data_ptr(), None))
    assert e.value.code == bz.ERR_ALIGN


def test_cubic_full_size(orc):
    """2^20 cubic segments, 2^24 random global parameters: GPU encode + GPU
    eval against the oracle's chain definition at every query."""
    chain, T = bz_synth.cubic_chain_walk()
    grid = bz.encode_piecewise_cubic(to_dev(chain))
    got = host(bz.eval_piecewise_cubic(grid, to_dev(T)))
    ref = orc.cubic_chain_eval(chain, T)
    err = np.abs(got - ref).max() / _extent(chain)
    assert err <= TOL_F32, err


@pytest.mark.parametrize("n_seg,dim", [(1, 3), (2, 3), (3, 3), (1000, 3), (77, 1), (300, 2), (129, 4), (10, 1)])
def test_cubic_tiled_layout_and_eval(orc, n_seg, dim):
    """Tiles hold [A, x0, x1] per column, tiles overlap by one column; the
    tiled evaluator returns the two-layer grid evaluator's results bit for
    bit, and the oracle's."""
    chain, T = bz_synth.cubic_chain_walk(n_seg=n_seg, dim=dim, n_q=5000, seed=11 * n_seg + dim)
    T = np.concatenate([T, [0.0, float(n_seg), -1.0, n_seg + 3.0, np.nan], np.arange(n_seg + 1.0)]).astype(np.float32)
    grid = bz.encode_piecewise_cubic(to_dev(chain))
    tiles = bz.tile_piecewise_cubic(grid)
    W = 3 * dim
    S = 32 // W - 1
    assert tiles.numel() == -(-n_seg // S) * 32
    tl = host(tiles).reshape(-1, 32)
    g = host(grid)
    for k in range(n_seg + 1):
        r = k & 1
        for j in ({k // S, (k - 1) // S} if k > 0 else {0}):
            if j >= tl.shape[0] or not (j * S <= k <= j * S + S):
                continue
            c = k - j * S
            col = tl[j, c * W:(c + 1) * W]
            np.testing.assert_array_equal(col[:dim], g[k, 0, r])
            np.testing.assert_array_equal(col[dim:2 * dim], g[k, 0, 1 - r])
            np.testing.assert_array_equal(col[2 * dim:], g[k, 1, 1 - r])
            np.testing.assert_array_equal(g[k, 1, r], g[k, 0, r])  # the shared texel
    Td = to_dev(T)
    a = host(bz.eval_piecewise_cubic_tiled(tiles, n_seg, dim, Td))
    b = host(bz.eval_piecewise_cubic(grid, Td))
    np.testing.assert_array_equal(a, b)
    ok = ~np.isnan(T)
    ref = orc.cubic_chain_eval(chain, T[ok])
    assert np.abs(a[:, ok] - ref).max() <= TOL_F32 * _extent(chain)


def test_cubic_tiled_full_size(orc):
    chain, T = bz_synth.cubic_chain_walk()
    grid = bz.encode_piecewise_cubic(to_dev(chain))
    tiles = bz.tile_piecewise_cubic(grid)
    Td = to_dev(T)
    a = bz.eval_piecewise_cubic_tiled(tiles, 1 << 20, 3, Td)
    b = bz.eval_piecewise_cubic(grid, Td)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    got = host(a)
    ref = orc.cubic_chain_eval(chain, T)
    assert np.abs(got - ref).max() / _extent(chain) <= TOL_F32
