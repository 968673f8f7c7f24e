"""GPU checks of the HBM probe kernels (measurement utility)."""
import pytest
import torch

import paper_2603_15447_amd as bz

pytestmark = pytest.mark.gpu


def test_probe_modes():
    n = (1 << 20) + 4 * 37  # not a multiple of the grid's stride
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros(n, dtype=torch.float32, device="cuda")
    bz.hbm_probe("copy", src, dst, 4)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    bz.hbm_probe("write", src, dst, 2)
    torch.cuda.synchronize()
    assert bool((dst == 1.0).all())
    bz.hbm_probe("read", src, dst, 8)  # non-negative data: dst untouched
    torch.cuda.synchronize()
    assert bool((dst == 1.0).all())
    dst.zero_()
    bz.hbm_probe("copy", src, dst, 0)  # one vector per thread
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    dst.zero_()
    bz.hbm_probe("write", src, dst, 0)
    torch.cuda.synchronize()
    assert bool((dst == 1.0).all())
    with pytest.raises(bz.BzError) as e:
        bz.check(bz.lib().bz_hbm_probe(2, src.data_ptr(), dst.data_ptr(), 6, 4, None))
    assert e.value.code == bz.ERR_SHAPE


@pytest.mark.parametrize("vec16", [1, 2, 3, 4])
def test_gather_probe(vec16):
    n_lines = 1000  # not a power of two: the line map is a multiply-high, not a mask
    src = torch.ones(n_lines * 32, dtype=torch.float32, device="cuda")
    sink = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    bz.gather_probe(src, (1 << 16) + 5, vec16, sink)  # ragged last block
    torch.cuda.synchronize()
    assert float(sink[0]) == 7.0  # non-negative data: never written
