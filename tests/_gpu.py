"""Helpers shared by the GPU parity tests."""
import numpy as np
import torch

TOL_F32 = 1e-5  # max error / control-point bounding-box extent, per object


def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def host(x):
    torch.cuda.synchronize()
    return x.detach().cpu().numpy().astype(np.float64)


# Below this fraction of an object's largest |coordinate| a box side cannot
# be resolved to TOL_F32 by FP32 results at all: two roundings of a result of
# that size (2u, u = 2^-24) already exceed TOL_F32 of such a box.
FP32_RESOLVABLE = 2.0 ** -23 / TOL_F32  # about 1.2%


def extents(ctrl):
    """Per-object error normaliser of ctrl[n][dim][m]: the largest side of the
    control-point bounding box, floored at FP32_RESOLVABLE of the object's
    largest |coordinate| (only a box smaller than about 1.2% of its distance
    from the origin reaches the floor)."""
    c = np.asarray(ctrl, dtype=np.float64)
    side = (c.max(axis=2) - c.min(axis=2)).max(axis=1)
    mag = np.abs(c).max(axis=(1, 2))
    return np.maximum(np.maximum(side, FP32_RESOLVABLE * mag), 1e-30)


def bbox_err(got, ref, ext, per_obj):
    """Largest per-object max|got - ref| / extent; got, ref are [dim, n*per_obj]."""
    d = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    if np.isnan(d).any():
        return np.inf
    e = d.max(axis=0).reshape(-1, per_obj).max(axis=1)
    return float((e / ext).max())
