"""FP64 CPU oracle for Bezier-family evaluation -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package imports nothing from it.

The arithmetic lives in ``bzo.c`` (plain C, double precision, OpenMP over
objects, built with ``-ffp-contract=off``).  This module only marshals numpy
arrays: every input is converted to float64 (exact for float32 data) and
every result comes back as float64.  Layouts follow the library interface:
curve control points ``ctrl[n][dim][deg+1]``, results ``out[dim][n*n_t]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bzo.c")
_LIB = os.path.join(_HERE, "libbzo.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def build(force=True):
    """Compile the oracle with gcc (plain C, FP64, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                           "-fPIC", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.bzo_max_threads.restype = ctypes.c_int
        L.bzo_set_threads.restype = ctypes.c_int
        L.bzo_set_threads.argtypes = [ctypes.c_int]
        L.bzo_fit_loss_grad.restype = ctypes.c_double
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def max_threads():
    return lib().bzo_max_threads()


def set_threads(n):
    """Thread count of the OpenMP loops from now on; returns the previous one."""
    return lib().bzo_set_threads(int(n))


def _curve_call(fn, ctrl, t, per_object):
    ctrl = _d(ctrl)
    n, dim, dp1 = ctrl.shape
    t = _d(t)
    nt = t.shape[-1]
    out = np.empty((dim, n * nt))
    fn(_ptr(ctrl), _I64(n), ctypes.c_int(dp1 - 1), ctypes.c_int(dim), _ptr(t), _I64(nt),
       ctypes.c_int(int(per_object)), _ptr(out))
    return out


def bezier_decasteljau(ctrl, t, per_object=False):
    """Bezier curves ctrl[n][dim][d+1] at t -> out[dim][n*n_t] (de Casteljau)."""
    return _curve_call(lib().bzo_bezier_decasteljau, ctrl, t, per_object)


def bezier_bernstein(ctrl, t, per_object=False):
    """Same curves by the Bernstein polynomial sum."""
    return _curve_call(lib().bzo_bezier_bernstein, ctrl, t, per_object)


def seiler_from_bezier(ctrl):
    """Seiler coefficients [b0, bd, d1, d_{d-1}, d2, ...] per curve/coordinate."""
    ctrl = _d(ctrl)
    n, dim, dp1 = ctrl.shape
    out = np.empty_like(ctrl)
    lib().bzo_seiler_from_bezier(_ptr(ctrl), _I64(n), ctypes.c_int(dp1 - 1), ctypes.c_int(dim), _ptr(out))
    return out


def seiler_eval(seiler, t, per_object=False):
    return _curve_call(lib().bzo_seiler_eval, seiler, t, per_object)


def piecewise_encode(chain):
    """chain[2N+1][dim] -> zig-zag grid[N+1][2][dim]."""
    chain = _d(chain)
    m, dim = chain.shape
    nseg = (m - 1) // 2
    grid = np.empty((nseg + 1, 2, dim))
    lib().bzo_piecewise_encode(_ptr(chain), _I64(nseg), ctypes.c_int(dim), _ptr(grid))
    return grid


def piecewise_eval(grid, T):
    grid = _d(grid)
    nseg = grid.shape[0] - 1
    dim = grid.shape[2]
    T = _d(T)
    out = np.empty((dim, T.shape[0]))
    lib().bzo_piecewise_eval(_ptr(grid), _I64(nseg), ctypes.c_int(dim), _ptr(T), _I64(T.shape[0]), _ptr(out))
    return out


def chain_eval(chain, T):
    chain = _d(chain)
    nseg = (chain.shape[0] - 1) // 2
    dim = chain.shape[1]
    T = _d(T)
    out = np.empty((dim, T.shape[0]))
    lib().bzo_chain_eval(_ptr(chain), _I64(nseg), ctypes.c_int(dim), _ptr(T), _I64(T.shape[0]), _ptr(out))
    return out


def cubic_chain_encode(chain):
    """Cubic chain[3N+1][dim] -> two stacked zig-zag layers grid[N+1][2][2][dim]."""
    chain = _d(chain)
    m, dim = chain.shape
    nseg = (m - 1) // 3
    grid = np.empty((nseg + 1, 2, 2, dim))
    lib().bzo_cubic_chain_encode(_ptr(chain), _I64(nseg), ctypes.c_int(dim), _ptr(grid))
    return grid


def cubic_chain_grid_eval(grid, T):
    grid = _d(grid)
    nseg, dim = grid.shape[0] - 1, grid.shape[3]
    T = _d(T)
    out = np.empty((dim, T.shape[0]))
    lib().bzo_cubic_chain_grid_eval(_ptr(grid), _I64(nseg), ctypes.c_int(dim), _ptr(T), _I64(T.shape[0]), _ptr(out))
    return out


def cubic_chain_eval(chain, T):
    chain = _d(chain)
    nseg, dim = (chain.shape[0] - 1) // 3, chain.shape[1]
    T = _d(T)
    out = np.empty((dim, T.shape[0]))
    lib().bzo_cubic_chain_eval(_ptr(chain), _I64(nseg), ctypes.c_int(dim), _ptr(T), _I64(T.shape[0]), _ptr(out))
    return out


def rational_eval(ctrl, w, t, per_object=False):
    ctrl = _d(ctrl)
    w = _d(w)
    n, dim, dp1 = ctrl.shape
    t = _d(t)
    nt = t.shape[-1]
    out = np.empty((dim, n * nt))
    lib().bzo_rational_eval(_ptr(ctrl), _ptr(w), _I64(n), ctypes.c_int(dp1 - 1), ctypes.c_int(dim), _ptr(t),
                            _I64(nt), ctypes.c_int(int(per_object)), _ptr(out))
    return out


def nurbs_eval(ctrl, w, knots, u, p=3):
    """One NURBS curve ctrl[dim][ncp], w[ncp], knots[ncp+p+1] at u -> out[dim][nu]."""
    ctrl = _d(ctrl)
    dim, ncp = ctrl.shape
    w, knots, u = _d(w), _d(knots), _d(u)
    assert knots.shape[0] == ncp + p + 1
    out = np.empty((dim, u.shape[0]))
    lib().bzo_nurbs_eval(_ptr(ctrl), _ptr(w), _ptr(knots), ctypes.c_int(ncp), ctypes.c_int(p), ctypes.c_int(dim),
                         _ptr(u), _I64(u.shape[0]), _ptr(out))
    return out


def batch_eval(batch):
    """Mixed batch (see bz_synth.Batch) -> out[dim][n_obj*n_t]."""
    kd = np.ascontiguousarray(batch.kind_degree, dtype=np.uint16)
    cpo = np.ascontiguousarray(batch.cp_offset, dtype=np.int64)
    ko = np.ascontiguousarray(batch.knot_offset, dtype=np.int64)
    ctrl, w, knots, t = _d(batch.ctrl), _d(batch.w), _d(batch.knots), _d(batch.t)
    v = getattr(batch, "v", None)
    if v is None:
        assert not ((kd >> 8) == 3).any(), "patches need the second parameters v"
    else:
        v = _d(v)
    n_obj = kd.shape[0]
    out = np.empty((batch.dim, n_obj * batch.n_t))
    lib().bzo_batch_eval(_I64(n_obj), _ptr(kd), _ptr(cpo), _ptr(ctrl), _ptr(w), _ptr(ko),
                         _ptr(knots if knots.size else np.zeros(1)), ctypes.c_int(batch.dim), _ptr(t), _ptr(v),
                         _I64(batch.n_t), _ptr(out))
    return out


def tensor_points(ctrl, du, dv, dw, uvw):
    """ctrl[n][dim][(du+1)(dv+1)(dw+1)], uvw[n][n_per][2|3] -> out[dim][n*n_per]."""
    ctrl = _d(ctrl)
    n, dim, _ = ctrl.shape
    uvw = _d(uvw)
    n_per = uvw.shape[1]
    out = np.empty((dim, n * n_per))
    lib().bzo_tensor_points(_ptr(ctrl), _I64(n), ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(dw),
                            ctypes.c_int(dim), _ptr(uvw), _I64(n_per), _ptr(out))
    return out


def tensor_grid(ctrl, du, dv, nu, nv):
    ctrl = _d(ctrl)
    n, dim, _ = ctrl.shape
    out = np.empty((dim, n * nu * nv))
    lib().bzo_tensor_grid(_ptr(ctrl), _I64(n), ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(dim),
                          ctypes.c_int(nu), ctypes.c_int(nv), _ptr(out))
    return out


def bezier_adjoint(ctrl, t, gout, w=None, per_object=True):
    """Analytic adjoint: returns (grad_ctrl, grad_w or None, grad_t or None)."""
    ctrl = _d(ctrl)
    n, dim, dp1 = ctrl.shape
    t = _d(t)
    nt = t.shape[-1]
    gout = _d(gout)
    w = _d(w) if w is not None else None
    gc = np.empty_like(ctrl)
    gw = np.empty((n, dp1)) if w is not None else None
    gt = np.empty((n, nt)) if per_object else None
    lib().bzo_bezier_adjoint(_ptr(ctrl), _ptr(w), _I64(n), ctypes.c_int(dp1 - 1), ctypes.c_int(dim), _ptr(t),
                             _I64(nt), ctypes.c_int(int(per_object)), _ptr(gout), _ptr(gc), _ptr(gw), _ptr(gt))
    return gc, gw, gt


def fit_loss_grad(ctrl, t, y, m_total=None):
    """L2 fitting loss (sum of squared distances over M, M = number of samples
    unless m_total is given) and its gradients."""
    ctrl = _d(ctrl)
    n, dim, dp1 = ctrl.shape
    t, y = _d(t), _d(y)
    nt = t.shape[-1]
    gc = np.empty_like(ctrl)
    gt = np.empty((n, nt))
    L = lib().bzo_fit_loss_grad(_ptr(ctrl), _I64(n), ctypes.c_int(dp1 - 1), ctypes.c_int(dim), _ptr(t), _I64(nt),
                                _ptr(y), ctypes.c_double(m_total or 0.0), _ptr(gc), _ptr(gt))
    return L, gc, gt


def adam(p, m, v, g, step, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8, lo=1.0, hi=0.0):
    """In-place Adam update of float64 arrays p, m, v (clamp to [lo,hi] if lo<=hi)."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _d(g)
    lib().bzo_adam(_ptr(p), _ptr(m), _ptr(v), _ptr(g), _I64(p.size), ctypes.c_int(step), ctypes.c_double(lr),
                   ctypes.c_double(b1), ctypes.c_double(b2), ctypes.c_double(eps), ctypes.c_double(lo),
                   ctypes.c_double(hi))


def fit_init(gt_ctrl, tau, eps):
    """Targets y = G(tau) + eps and the starting point of the fit: t_j =
    j/(n_t-1) and the straight line from y_0 to y_{n_t-1} (control point i at
    i/d).  Returns (y, ctrl0, t0) in float64."""
    n, dim, dp1 = gt_ctrl.shape
    deg = dp1 - 1
    nt = tau.shape[1]
    y = bezier_decasteljau(gt_ctrl, tau, per_object=True) + _d(eps)
    y3 = y.reshape(dim, n, nt)
    first, last = y3[:, :, 0].T, y3[:, :, -1].T
    frac = np.arange(dp1) / deg
    ctrl = np.ascontiguousarray(first[:, :, None] * (1.0 - frac) + last[:, :, None] * frac)
    t = np.ascontiguousarray(np.tile(np.arange(nt) / (nt - 1), (n, 1)))
    return y, ctrl, t


def fit_steps(y, ctrl, t, steps, lr=1e-2, m_total=None, first_step=1):
    """Adam steps on (ctrl, t) in place (t clamped to [0,1]); returns losses."""
    mc, vc = np.zeros_like(ctrl), np.zeros_like(ctrl)
    mt, vt = np.zeros_like(t), np.zeros_like(t)
    losses = []
    for s in range(first_step, first_step + steps):
        L, gc, gtt = fit_loss_grad(ctrl, t, y, m_total)
        losses.append(L)
        adam(ctrl, mc, vc, gc, s, lr)
        adam(t, mt, vt, gtt, s, lr, lo=0.0, hi=1.0)
    return losses


def fit_reference(gt_ctrl, tau, eps, steps, lr=1e-2):
    """The whole fitting experiment in FP64: targets y = G(tau) + eps, start
    from t_j = j/(n_t-1) and the straight line from y_0 to y_{n_t-1} (control
    point i at i/d), then `steps` Adam steps on control points and t (t
    clamped to [0,1]).  Returns (ctrl, t, losses)."""
    y, ctrl, t = fit_init(gt_ctrl, tau, eps)
    losses = fit_steps(y, ctrl, t, steps, lr)
    return ctrl, t, losses


# ------------------------------------------------ texture-filter emulation
TEX_DC, TEX_HYBRID, TEX_SEILER = 0, 1, 2
TEX_MODES = {"decasteljau": TEX_DC, "hybrid": TEX_HYBRID, "seiler": TEX_SEILER}
ROUNDINGS = {"nearest": 0, "truncate": 1}


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def tex_texels(deg, mode):
    return lib().bzo_tex_texels(ctypes.c_int(deg), ctypes.c_int(TEX_MODES[mode]))


def tex_axis_weights(p, frac_bits=8, rounding="nearest"):
    """Filter weights of a 2-texel axis sampled at FP32 parameters p."""
    p = _f(p).ravel()
    w = np.empty(p.shape[0])
    lib().bzo_tex_axis_weights(_ptr(p), _I64(p.shape[0]), ctypes.c_int(frac_bits),
                               ctypes.c_int(ROUNDINGS[rounding]), _ptr(w))
    return w


def tex_build(ctrl, mode):
    """Curve textures tex[n][dim][texels] (float64) of ctrl[n][dim][d+1]."""
    ctrl = _d(ctrl)
    n, dim, dp1 = ctrl.shape
    ntx = tex_texels(dp1 - 1, mode)
    tex = np.empty((n, dim, ntx))
    lib().bzo_tex_build(_ptr(ctrl), _I64(n), ctypes.c_int(dp1 - 1), ctypes.c_int(dim),
                        ctypes.c_int(TEX_MODES[mode]), _ptr(tex))
    return tex


def tex_eval(tex, deg, mode, t, per_object=False, frac_bits=8, rounding="nearest"):
    """Emulated texture sampling of float32 textures tex[n][dim][texels] at
    FP32 parameters t -> out[dim][n*n_t] (float64)."""
    tex = _f(tex)
    n, dim, _ = tex.shape
    t = _f(t)
    nt = t.shape[-1]
    out = np.empty((dim, n * nt))
    lib().bzo_tex_eval(_ptr(tex), _I64(n), ctypes.c_int(deg), ctypes.c_int(dim), ctypes.c_int(TEX_MODES[mode]),
                       _ptr(t), _I64(nt), ctypes.c_int(int(per_object)), ctypes.c_int(frac_bits),
                       ctypes.c_int(ROUNDINGS[rounding]), _ptr(out))
    return out


def chain_texemu_eval(grid, T, frac_bits=8, rounding="nearest"):
    """Zig-zag grid[N+1][2][dim] (float32) read by the emulated bilinear
    filter at FP32 global parameters T -> out[dim][n_q]."""
    grid = _f(grid)
    nseg, dim = grid.shape[0] - 1, grid.shape[2]
    T = _f(T)
    out = np.empty((dim, T.shape[0]))
    lib().bzo_chain_texemu_eval(_ptr(grid), _I64(nseg), ctypes.c_int(dim), _ptr(T), _I64(T.shape[0]),
                                ctypes.c_int(frac_bits), ctypes.c_int(ROUNDINGS[rounding]), _ptr(out))
    return out


# ------------------------------------------------ Seiler surfaces and volumes
def tensor_to_seiler(ctrl, du, dv, dw=0):
    """Per-axis Seiler terms sc[n][dim][ncp] of tensor control points."""
    ctrl = _d(ctrl)
    n, dim, ncp = ctrl.shape
    assert ncp == (du + 1) * (dv + 1) * (dw + 1)
    sc = np.empty_like(ctrl)
    lib().bzo_tensor_to_seiler(_ptr(ctrl), _I64(n), ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(dw),
                               ctypes.c_int(dim), _ptr(sc))
    return sc


def tensor_seiler_points(sc, du, dv, dw, uvw):
    """Nested per-axis Seiler evaluation at uvw[n][n_per][2|3] -> out[dim][n*n_per]."""
    sc = _d(sc)
    n, dim, _ = sc.shape
    uvw = _d(uvw)
    n_per = uvw.shape[1]
    out = np.empty((dim, n * n_per))
    lib().bzo_tensor_seiler_points(_ptr(sc), _I64(n), ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(dw),
                                   ctypes.c_int(dim), _ptr(uvw), _I64(n_per), _ptr(out))
    return out


def tensor_seiler_grid(sc, du, dv, nu, nv):
    """Nested per-axis Seiler evaluation of surfaces on the inclusive nu x nv
    grid (u_a = a/(nu-1), v_b = b/(nv-1)) -> out[dim][n*nu*nv]."""
    n = np.asarray(sc).shape[0]
    u = np.arange(nu) / max(nu - 1, 1)
    v = np.arange(nv) / max(nv - 1, 1)
    uv = np.stack(np.meshgrid(u, v, indexing="ij"), axis=-1).reshape(1, nu * nv, 2)
    return tensor_seiler_points(sc, du, dv, 0, np.repeat(uv, n, axis=0))


def tex_patch_texels(du, dv, mode):
    return lib().bzo_tex_patch_texels(ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(TEX_MODES[mode]))


def tex_patch_build(ctrl, du, dv, mode):
    """Surface textures tex[n][dim][(dv+1)*texels] (float64) of patches ctrl[n][dim][(du+1)(dv+1)]."""
    ctrl = _d(ctrl)
    n, dim, _ = ctrl.shape
    tex = np.empty((n, dim, tex_patch_texels(du, dv, mode)))
    lib().bzo_tex_patch_build(_ptr(ctrl), _I64(n), ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(dim),
                              ctypes.c_int(TEX_MODES[mode]), _ptr(tex))
    return tex


def tex_patch_eval(tex, du, dv, mode, uv, frac_bits=8, rounding="nearest"):
    """Emulated reads of float32 surface textures at uv[n][n_per][2] -> out[dim][n*n_per]."""
    tex = _f(tex)
    n, dim, _ = tex.shape
    uv = _f(uv)
    n_per = uv.shape[1]
    out = np.empty((dim, n * n_per))
    lib().bzo_tex_patch_eval(_ptr(tex), _I64(n), ctypes.c_int(du), ctypes.c_int(dv), ctypes.c_int(dim),
                             ctypes.c_int(TEX_MODES[mode]), _ptr(uv), _I64(n_per), ctypes.c_int(frac_bits),
                             ctypes.c_int(ROUNDINGS[rounding]), _ptr(out))
    return out


# ------------------------------------------------ particle ring
PARTICLE_METHODS = {"polynomial": 0, "seiler": 1, "seiler_texture": 2, "table": 3}


def particles_step(seg, T, speed, dt, method, iters, samples=64):
    """One frame of the particle ring: returns (T_new float32, pos[3][P], shade[P])."""
    seg = _d(seg)
    T = _f(T).copy()
    speed = _f(speed)
    P = T.shape[0]
    pos = np.empty((3, P))
    shade = np.empty(P)
    lib().bzo_particles_step(_ptr(seg), _I64(seg.shape[0]), ctypes.c_int(PARTICLE_METHODS[method]),
                             ctypes.c_int(samples), _ptr(T), _ptr(speed), ctypes.c_float(dt), _I64(P),
                             ctypes.c_int(iters), _ptr(pos), _ptr(shade))
    return T, pos, shade
