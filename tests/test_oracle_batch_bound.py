"""CPU pin of the low-precision storage bound of mixed batches, on the
oracle alone (no GPU): FP64 evaluation of FP32 inputs against FP64
evaluation of their FP16 / BF16 roundings."""
import numpy as np
import torch

import bz_synth
from tests._batch import _extents, _lp_bound


def test_lp_bound_holds_on_the_cpu(orc):
    """The rounding bound itself, on the oracle alone (FP64 evaluation of the
    FP32 inputs and of their FP16 / BF16 roundings): it holds for every object
    and is not vacuous (the worst object uses a good part of it)."""
    b = bz_synth.mixed_batch(n_bezier=3000, n_nurbs=300, n_t=16, seed=77)
    ref = orc.batch_eval(b)
    ext = _extents(b)
    for dtype in (torch.float16, torch.bfloat16):
        rb = bz_synth.Batch(**{**b.__dict__})
        rb.ctrl = torch.from_numpy(b.ctrl).to(dtype).float().numpy()
        rb.w = torch.from_numpy(b.w).to(dtype).float().numpy()
        d = np.abs(orc.batch_eval(rb) - ref).max(axis=0).reshape(-1, 16).max(axis=1)
        bound = _lp_bound(b, rb, ext)
        assert (d <= bound * (1 + 1e-9)).all()
        assert (d / bound).max() > 0.3
