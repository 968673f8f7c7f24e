"""Seeded synthetic inputs for the Bezier-family evaluators.

This module is shared by the FP64 oracle side and the GPU side.  It draws
random numbers and lays them out in the arrays both sides consume; it holds
none of the evaluation arithmetic (no curve is evaluated here, no encoding
is performed).  Everything is drawn with numpy's PCG64 in float64 and cast
to float32 once, so both sides see bit-identical FP32 inputs.

Workload shapes follow the evaluation scenarios the paper motivates
(Sec. 2: curves, C0 piecewise chains, surfaces, volumes and NURBS; Sec. 5:
many evaluations per frame).  The paper names no public dataset; every
input here is synthetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEEDS = {"plain": 1001, "chain": 1002, "batched": 1003, "patch": 1004,
         "volume": 1005, "fit": 1006, "particles": 1007}

KIND_BEZIER = 0
KIND_RATIONAL = 1
KIND_NURBS = 2
KIND_PATCH = 3


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


# ---------------------------------------------------------------- curves
def plain_curves(n_curves=4096, degree=3, dim=3, n_t=256, seed=SEEDS["plain"]):
    """Independent Bezier curves, control points i.i.d. U[-1,1]^dim.

    Returns ctrl[n_curves][dim][degree+1] (f32) and the shared parameter
    vector t_j = j/(n_t-1) (inclusive grid, so both endpoints are hit)."""
    rng = np.random.default_rng(seed)
    ctrl = _f32(rng.uniform(-1.0, 1.0, size=(n_curves, dim, degree + 1)))
    t = _f32(np.arange(n_t, dtype=np.float64) / max(n_t - 1, 1))
    return ctrl, t


def random_curves(n_curves, degree, dim, n_t, seed, per_object=True, lo=0.0, hi=1.0):
    """Bezier curves with U[-1,1] control points and uniform random t."""
    rng = np.random.default_rng(seed)
    ctrl = _f32(rng.uniform(-1.0, 1.0, size=(n_curves, dim, degree + 1)))
    shape = (n_curves, n_t) if per_object else (n_t,)
    t = _f32(rng.uniform(lo, hi, size=shape))
    return ctrl, t


def log_uniform_weights(rng, size, lo=0.25, hi=4.0):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def rational_curves(n_curves, degree, dim, n_t, seed, per_object=True):
    rng = np.random.default_rng(seed)
    ctrl = _f32(rng.uniform(-1.0, 1.0, size=(n_curves, dim, degree + 1)))
    w = _f32(log_uniform_weights(rng, (n_curves, degree + 1)))
    shape = (n_curves, n_t) if per_object else (n_t,)
    t = _f32(rng.uniform(0.0, 1.0, size=shape))
    return ctrl, w, t


# ---------------------------------------------------------------- C0 chain
def chain_walk(n_seg=1 << 20, dim=3, n_q=1 << 24, step=0.1, seed=SEEDS["chain"]):
    """C0 quadratic chain: 2*n_seg+1 points of a random walk started at 0
    with i.i.d. U[-step,step]^dim steps.  Point 2k is the shared endpoint
    A_k, point 2k+1 is the middle control point M_k of segment k.

    Returns chain[2*n_seg+1][dim] (f32) and n_q global parameters
    T = f32(U[0,1) * n_seg)."""
    rng = np.random.default_rng(seed)
    steps = rng.uniform(-step, step, size=(2 * n_seg, dim))
    walk = np.zeros((2 * n_seg + 1, dim), dtype=np.float64)
    np.cumsum(steps, axis=0, out=walk[1:])
    chain = _f32(walk)
    del walk, steps
    T = _f32(rng.uniform(0.0, 1.0, size=n_q) * n_seg)
    return chain, T


def cubic_chain_walk(n_seg=1 << 20, dim=3, n_q=1 << 24, step=0.1, seed=SEEDS["chain"] + 100):
    """C0 cubic chain: 3*n_seg+1 points of a random walk started at 0 with
    i.i.d. U[-step,step]^dim steps (points 3k are the shared endpoints), and
    n_q global parameters T = f32(U[0,1) * n_seg)."""
    rng = np.random.default_rng(seed)
    steps = rng.uniform(-step, step, size=(3 * n_seg, dim))
    walk = np.zeros((3 * n_seg + 1, dim), dtype=np.float64)
    np.cumsum(steps, axis=0, out=walk[1:])
    chain = _f32(walk)
    del walk, steps
    T = _f32(rng.uniform(0.0, 1.0, size=n_q) * n_seg)
    return chain, T


# ---------------------------------------------------------------- batched
@dataclass
class Batch:
    """Mixed batch of curves in one flat description.

    kind_degree[o] = kind << 8 | degree   (kind 0 Bezier, 1 rational, 2 NURBS,
                   3 tensor-product surface patch with degree du << 4 | dv)
    cp_offset[o]   first control point of object o; ctrl holds, for object o,
                   a [dim][ncp_o] block starting at float index cp_offset[o]*dim
                   (a patch's (du+1)(dv+1) points indexed i*(dv+1)+j)
    w              one weight per control point (1.0 for integral objects)
    knot_offset[o] first knot of object o (NURBS only; empty range otherwise)
    t              [n_obj][n_t] parameters in [0,1) (a patch's u)
    v              [n_obj][n_t] second parameters (a patch's v), or None
                   when the batch has no patch
    """
    dim: int
    n_t: int
    kind_degree: np.ndarray
    cp_offset: np.ndarray
    ctrl: np.ndarray
    w: np.ndarray
    knot_offset: np.ndarray
    knots: np.ndarray
    t: np.ndarray
    meta: dict = field(default_factory=dict)
    v: np.ndarray = None

    @property
    def n_obj(self):
        return int(self.kind_degree.shape[0])

    def subset(self, idx):
        """The objects idx (in that order) as a batch of their own: the same
        control points, weights, knots and parameters, re-packed with new
        offsets.  A layout gather only."""
        idx = np.asarray(idx, dtype=np.int64)
        ncp = (self.cp_offset[idx + 1] - self.cp_offset[idx])
        nk = (self.knot_offset[idx + 1] - self.knot_offset[idx])
        cp = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(ncp, out=cp[1:])
        ko = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(nk, out=ko[1:])
        def ranges(off, scale=1):
            parts = [np.arange(off[o] * scale, off[o + 1] * scale) for o in idx]
            return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
        pts, crd, kts = ranges(self.cp_offset), ranges(self.cp_offset, self.dim), ranges(self.knot_offset)
        return Batch(dim=self.dim, n_t=self.n_t, kind_degree=self.kind_degree[idx].copy(), cp_offset=cp,
                     ctrl=np.ascontiguousarray(self.ctrl[crd]), w=np.ascontiguousarray(self.w[pts]),
                     knot_offset=ko, knots=np.ascontiguousarray(self.knots[kts]),
                     t=np.ascontiguousarray(self.t[idx]), meta=dict(self.meta),
                     v=None if self.v is None else np.ascontiguousarray(self.v[idx]))


def mixed_batch(n_bezier=1 << 20, n_nurbs=1 << 16, dim=3, n_t=16, deg_lo=2, deg_hi=15,
                knots_lo=8, knots_hi=64, seed=SEEDS["batched"], n_patches=0, patch_deg_lo=3, patch_deg_hi=3):
    """Bezier curves of degree U{deg_lo..deg_hi} (half of them rational with
    log-uniform weights in [0.25,4]) plus cubic NURBS with a clamped knot
    vector of K ~ U{knots_lo..knots_hi} knots (interior knots sorted U(0,1)),
    K-4 control points and log-uniform weights, plus n_patches tensor-product
    surface patches of degrees du, dv ~ U{patch_deg_lo..patch_deg_hi} (default
    bicubic).  Objects are shuffled.  Control points are U[-1,1]^dim; n_t
    parameters U[0,1) per object, and for batches with patches a second
    parameter array v, U[0,1) (drawn last, so batches without patches are
    unchanged)."""
    rng = np.random.default_rng(seed)
    n_obj = n_bezier + n_nurbs + n_patches
    deg = rng.integers(deg_lo, deg_hi + 1, size=n_bezier)
    rational = rng.random(n_bezier) < 0.5
    kinds = np.where(rational, KIND_RATIONAL, KIND_BEZIER)
    K = rng.integers(knots_lo, knots_hi + 1, size=n_nurbs)
    if n_patches:
        pdu = rng.integers(patch_deg_lo, patch_deg_hi + 1, size=n_patches)
        pdv = rng.integers(patch_deg_lo, patch_deg_hi + 1, size=n_patches)
    perm = rng.permutation(n_obj)
    kind_degree = np.empty(n_obj, dtype=np.uint16)
    ncp = np.empty(n_obj, dtype=np.int64)
    nknot = np.zeros(n_obj, dtype=np.int64)
    is_b = perm < n_bezier
    is_n = (perm >= n_bezier) & (perm < n_bezier + n_nurbs)
    is_p = perm >= n_bezier + n_nurbs
    bidx = perm[is_b]
    nidx = perm[is_n] - n_bezier
    kind_degree[is_b] = (kinds[bidx] << 8 | deg[bidx]).astype(np.uint16)
    ncp[is_b] = deg[bidx] + 1
    kind_degree[is_n] = np.uint16(KIND_NURBS << 8 | 3)
    ncp[is_n] = K[nidx] - 4
    nknot[is_n] = K[nidx]
    if n_patches:
        pidx = perm[is_p] - n_bezier - n_nurbs
        kind_degree[is_p] = (KIND_PATCH << 8 | pdu[pidx] << 4 | pdv[pidx]).astype(np.uint16)
        ncp[is_p] = (pdu[pidx] + 1) * (pdv[pidx] + 1)
    cp_offset = np.zeros(n_obj + 1, dtype=np.int64)
    np.cumsum(ncp, out=cp_offset[1:])
    knot_offset = np.zeros(n_obj + 1, dtype=np.int64)
    np.cumsum(nknot, out=knot_offset[1:])
    total_cp = int(cp_offset[-1])
    # Control points: each object's block is [dim][ncp]; drawing all values
    # i.i.d. makes the block layout irrelevant to the distribution.
    ctrl = _f32(rng.uniform(-1.0, 1.0, size=total_cp * dim))
    w = log_uniform_weights(rng, total_cp)
    kind = kind_degree >> 8
    integral = np.repeat((kind == KIND_BEZIER) | (kind == KIND_PATCH), ncp)
    w[integral] = 1.0
    w = _f32(w)
    # Clamped knot vectors: 4 zeros, K-8 sorted uniforms, 4 ones.
    total_k = int(knot_offset[-1])
    knots = np.empty(total_k, dtype=np.float64)
    nurbs_objs = np.nonzero(kind == KIND_NURBS)[0]
    inner = rng.random(total_k)
    for o in nurbs_objs:
        a, b = knot_offset[o], knot_offset[o + 1]
        k = b - a
        # interior knots strictly inside (0, 1) also after rounding to FP32
        v = np.clip(np.sort(inner[a:a + k - 8]), np.finfo(np.float32).tiny, np.nextafter(np.float32(1), np.float32(0)))
        knots[a:a + 4] = 0.0
        knots[a + 4:b - 4] = v
        knots[b - 4:b] = 1.0
    knots = _f32(knots)
    t = _f32(rng.random((n_obj, n_t)))
    v = _f32(rng.random((n_obj, n_t))) if n_patches else None
    return Batch(dim=dim, n_t=n_t, kind_degree=kind_degree, cp_offset=cp_offset, ctrl=ctrl,
                 w=w, knot_offset=knot_offset, knots=knots, t=t,
                 meta={"n_bezier": n_bezier, "n_nurbs": n_nurbs, "n_patches": n_patches}, v=v)


# ---------------------------------------------------------------- tensor
def patches(n_obj=1 << 18, du=3, dv=3, dim=3, seed=SEEDS["patch"]):
    """Tensor-product surface patches, control points U[-1,1]^dim, stored
    ctrl[n_obj][dim][(du+1)*(dv+1)] with the u index major."""
    rng = np.random.default_rng(seed)
    return _f32(rng.uniform(-1.0, 1.0, size=(n_obj, dim, (du + 1) * (dv + 1))))


def volumes(n_obj=1 << 16, d=3, dim=3, n_q=1 << 24, seed=SEEDS["volume"]):
    """Tensor-product volumes of degree (d,d,d), control points U[-1,1]^dim,
    ctrl[n_obj][dim][(d+1)^3] (u major, w minor), and n_q random (u,v,w) in
    U[0,1)^3 split evenly over the volumes: uvw[n_obj][n_q/n_obj][3]."""
    rng = np.random.default_rng(seed)
    ctrl = _f32(rng.uniform(-1.0, 1.0, size=(n_obj, dim, (d + 1) ** 3)))
    n_per = n_q // n_obj
    uvw = _f32(rng.random((n_obj, n_per, 3)))
    return ctrl, uvw


# ---------------------------------------------------------------- fitting
def fit_problem(n_curves=65536, n_samples=128, dim=3, degree=3, noise=0.01, seed=SEEDS["fit"]):
    """Curve-fitting problem: ground-truth control points U[-1,1]^dim,
    sorted sample parameters tau ~ U(0,1) per curve and Gaussian noise of
    standard deviation `noise` (one draw per target coordinate, stored
    [dim][n_curves*n_samples]).  The targets are ground_truth(tau) + noise;
    each side evaluates the ground-truth curve itself."""
    rng = np.random.default_rng(seed)
    gt = _f32(rng.uniform(-1.0, 1.0, size=(n_curves, dim, degree + 1)))
    tau = _f32(np.sort(rng.random((n_curves, n_samples)), axis=1))
    eps = _f32(rng.normal(0.0, noise, size=(dim, n_curves * n_samples)))
    return gt, tau, eps


# ---------------------------------------------------------------- particle ring
def particle_ring(n_seg=16, n_particles=1 << 20, jitter=0.15, seed=SEEDS["particles"]):
    """A closed C0 ring of n_seg cubic Bezier segments and particles on it
    (Sec. 5's particle test: cubic curves chained into a ring, particles
    moving along them).  Shared endpoints lie on the unit circle at angles
    2 pi k / n_seg in the z = 0 plane; each inner control point is a third
    of the way along the chord plus U[-jitter, jitter]^3.  Returns
    segments[n_seg][3][4] (per-segment control points, endpoints repeated,
    the last segment ending at the first point), particle phases
    T ~ U[0, n_seg) and speeds ~ U[0.5, 1.5] segments per unit time."""
    rng = np.random.default_rng(seed)
    ang = 2.0 * np.pi * np.arange(n_seg) / n_seg
    A = np.stack([np.cos(ang), np.sin(ang), np.zeros(n_seg)], axis=1)
    seg = np.empty((n_seg, 3, 4))
    for k in range(n_seg):
        a, b = A[k], A[(k + 1) % n_seg]
        p1 = a + (b - a) / 3.0 + rng.uniform(-jitter, jitter, 3)
        p2 = a + 2.0 * (b - a) / 3.0 + rng.uniform(-jitter, jitter, 3)
        seg[k] = np.stack([a, p1, p2, b], axis=1)
    T = _f32(rng.uniform(0.0, 1.0, size=n_particles) * n_seg)
    speed = _f32(rng.uniform(0.5, 1.5, size=n_particles))
    return _f32(seg), T, speed
