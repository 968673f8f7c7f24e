"""Helpers for batch tests (CPU side): per-object error normaliser and the
low-precision storage bound."""
import numpy as np


def _extents(b, ctrl=None):
    """Per-object normaliser: the largest bounding-box side, floored at
    FP32_RESOLVABLE of the largest |coordinate|, as for single curves."""
    from tests._gpu import FP32_RESOLVABLE
    c = np.asarray(b.ctrl if ctrl is None else ctrl, np.float64)
    ext = np.empty(b.n_obj)
    for o in range(b.n_obj):
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        P = c[a0 * b.dim:a1 * b.dim].reshape(b.dim, a1 - a0)
        ext[o] = max((P.max(axis=1) - P.min(axis=1)).max(), FP32_RESOLVABLE * np.abs(P).max(), 1e-30)
    return ext


def _lp_bound(b, rb, ext):
    """Per-object bound on |C(rounded inputs) - C(inputs)| for positive
    weights: the points are convex combinations sum lam_i b_i with lam_i =
    w_i B_i / sum w_j B_j (B-spline basis for NURBS), so rounding the points
    moves C by at most max|b_i - rb_i|, and rounding the weights by relative
    e_i changes lam_i to lam_i (1+e_i)/(1+e_bar), which moves C by at most
    max|e_i| * (half the box side, doubled) / (1 - max|e_i|)."""
    out = np.empty(b.n_obj)
    for o in range(b.n_obj):
        a0, a1 = b.cp_offset[o], b.cp_offset[o + 1]
        db = np.abs(b.ctrl[a0 * b.dim:a1 * b.dim].astype(np.float64) - rb.ctrl[a0 * b.dim:a1 * b.dim]).max()
        w = b.w[a0:a1].astype(np.float64)
        e = float(np.abs((rb.w[a0:a1] - w) / w).max()) if (b.kind_degree[o] >> 8) else 0.0
        out[o] = db + e * ext[o] / (1.0 - e)
    return out
