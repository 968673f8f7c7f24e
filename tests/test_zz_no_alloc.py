"""GPU: the allocation-free chain encoder (bz_encode_piecewise_noalloc)
against the allocating one (bz_encode_piecewise), through the C ABI: bit
for bit on two calls in a row, the second with a smaller chain (the fixed
workspace keeps the first call's partials, which must not leak into the
second), and its size limit."""
import ctypes

import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import host, to_dev

pytestmark = pytest.mark.gpu


def _both(chain):
    c = to_dev(chain)
    m, dim = chain.shape
    nseg = (m - 1) // 2
    ref = bz.encode_piecewise(c)
    got = torch.full((nseg + 1, 2, dim), float("nan"), device=c.device)
    bz.encode_piecewise_noalloc(c, got)
    return host(got), host(ref)


def test_noalloc_encoder_matches_allocating_encoder(orc):
    for n_seg, dim, seed in ((1 << 20, 3, 1), (3001, 2, 2), (1, 1, 3)):
        chain, _ = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=1, seed=seed)
        got, ref = _both(chain)
        np.testing.assert_array_equal(got, ref)
        if n_seg <= 4096:  # and the oracle's encoding, to the encoder's FP64-then-round accuracy
            want = orc.piecewise_encode(chain)
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-6 * max(1.0, np.abs(want).max()))


def test_noalloc_encoder_size_limit():
    L = bz.lib()
    for dim, limit in ((1, 536870911), (2, 268435455), (3, 178956287), (4, 134217727)):
        # beyond the limit: refused before anything is launched (no pointer is read)
        rc = L.bz_encode_piecewise_noalloc(ctypes.c_void_p(0x10000), limit + 1, dim, ctypes.c_void_p(0x10000), None)
        assert rc == bz.ERR_SHAPE, (dim, rc)
        assert "workspace" in bz.last_error()
    assert L.bz_encode_piecewise_noalloc(None, 0, 3, None, None) == bz.OK
    assert L.bz_encode_piecewise_noalloc(None, 5, 3, None, None) == bz.ERR_NULL
