"""Python binding of libbz, the gfx950 Bezier-family evaluation library.

Argument marshalling only: every function passes tensor data pointers and
torch's current HIP stream to the C ABI declared in ``include/bz.h``; all
arithmetic runs in the library's HIP kernels.  PyTorch provides device memory
and streams.  There is no fallback: if ``libbz.so`` is missing or fails to
load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbz.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bz.h")

OK, ERR_NULL, ERR_SHAPE, ERR_DTYPE, ERR_UNSUPPORTED, ERR_ALIGN, ERR_HIP, ERR_NOMEM, ERR_INTERNAL = range(9)
F32, F16, BF16 = 0, 1, 2
DECASTELJAU, BERNSTEIN, SEILER, AUTO = 0, 1, 2, 3
T_SHARED, T_PER_OBJECT = 0, 1
TP_VALU, TP_MFMA_F32, TP_MFMA_BF16, TP_MFMA_F16, TP_MFMA_F16X3 = 0, 1, 2, 3, 4

METHODS = {"decasteljau": DECASTELJAU, "bernstein": BERNSTEIN, "seiler": SEILER, "auto": AUTO}
ENGINES = {"valu": TP_VALU, "mfma_f32": TP_MFMA_F32, "mfma_bf16": TP_MFMA_BF16, "mfma_f16": TP_MFMA_F16,
           "mfma_f16x3": TP_MFMA_F16X3}
TEX_MODES = {"decasteljau": 0, "hybrid": 1, "seiler": 2}
TEX_ROUNDING = {"nearest": 0, "truncate": 1}
_DT = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}

_lib = None


class BzError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


_P, _I64, _I, _F = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float

_SIGS = {
    "bz_version": (_I, []),
    "bz_status_string": (ctypes.c_char_p, [_I]),
    "bz_last_error": (ctypes.c_char_p, []),
    "bz_device_cu_count": (_I, []),
    "bz_eval_bezier": (_I, [_P, _I, _I64, _I, _I, _P, _I64, _I, _I, _P, _P]),
    "bz_bezier_to_seiler": (_I, [_P, _I, _I64, _I, _I, _P, _P]),
    "bz_eval_seiler": (_I, [_P, _I64, _I, _I, _P, _I64, _I, _P, _P]),
    "bz_eval_rational": (_I, [_P, _P, _I, _I64, _I, _I, _P, _I64, _I, _I, _F, _P, _P, _P]),
    "bz_encode_piecewise": (_I, [_P, _I64, _I, _P, _P]),
    "bz_encode_piecewise_noalloc": (_I, [_P, _I64, _I, _P, _P]),
    "bz_eval_piecewise": (_I, [_P, _I64, _I, _P, _I64, _P, _P]),
    "bz_encode_piecewise_cubic": (_I, [_P, _I64, _I, _P, _P]),
    "bz_eval_piecewise_cubic": (_I, [_P, _I64, _I, _P, _I64, _P, _P]),
    "bz_texture_texels": (_I, [_I, _I]),
    "bz_build_texture": (_I, [_P, _I64, _I, _I, _I, _P, _P]),
    "bz_eval_texture": (_I, [_P, _I64, _I, _I, _I, _P, _I64, _I, _I, _I, _P, _P]),
    "bz_eval_piecewise_texemu": (_I, [_P, _I64, _I, _P, _I64, _I, _I, _P, _P]),
    "bz_eval_piecewise_texemu_tiled": (_I, [_P, _I64, _I, _P, _I64, _I, _I, _P, _P]),
    "bz_tensor_to_seiler": (_I, [_P, _I64, _I, _I, _I, _I, _P, _P]),
    "bz_eval_tensor_seiler": (_I, [_P, _I64, _I, _I, _I, _I, _P, _I64, _I, _I, _P, _P]),
    "bz_hbm_probe": (_I, [_I, _P, _P, _I64, _I, _P]),
    "bz_gather_probe": (_I, [_P, _I64, _I64, _I, _P, _P]),
    "bz_piecewise_cubic_tiled_floats": (_I64, [_I64, _I]),
    "bz_tile_piecewise_cubic": (_I, [_P, _I64, _I, _P, _P]),
    "bz_eval_piecewise_cubic_tiled": (_I, [_P, _I64, _I, _P, _I64, _P, _P]),
    "bz_texture_patch_texels": (_I, [_I, _I, _I]),
    "bz_build_texture_patch": (_I, [_P, _I64, _I, _I, _I, _I, _P, _P]),
    "bz_eval_texture_patch": (_I, [_P, _I64, _I, _I, _I, _I, _P, _I64, _I, _I, _P, _P]),
    "bz_particles_step": (_I, [_I, _P, _I64, _I, _P, _P, _F, _I64, _I, _P, _P, _P]),
    "bz_particle_ring_table": (_I, [_P, _I64, _I, _P, _P]),
    "bz_piecewise_tiled_floats": (_I64, [_I64, _I]),
    "bz_tile_piecewise": (_I, [_P, _I64, _I, _P, _P]),
    "bz_eval_piecewise_tiled": (_I, [_P, _I64, _I, _P, _I64, _P, _P]),
    "bz_piecewise_tiled16_halfs": (_I64, [_I64, _I]),
    "bz_tile_piecewise16": (_I, [_P, _I64, _I, _I, _P, _P]),
    "bz_eval_piecewise_tiled16": (_I, [_P, _I, _I64, _I, _P, _I64, _P, _P]),
    "bz_eval_tensor_patch": (_I, [_P, _I, _I64, _I, _I, _I, _I, _P, _I64, _I, _I, _I, _P, _P]),
    "bz_batch_plan_create": (_I, [_I64, _P, _P, _P, _P, _I, _I, _P, _P, _I64, _I, _P, ctypes.POINTER(_P)]),
    "bz_batch_eval": (_I, [_P, _P, _P, _P]),
    "bz_batch_eval_uv": (_I, [_P, _P, _P, _P, _P]),
    "bz_batch_plan_autotune": (_I, [_P, _P, _P, _P, _P]),
    "bz_batch_plan_info": (_I, [_P, _P]),
    "bz_batch_plan_configure": (_I, [_P, _I64, _I, _I, _I, _I64, _P]),
    "bz_plan_destroy": (_I, [_P]),
    "bz_adjoint_bezier": (_I, [_P, _P, _I64, _I, _I, _P, _I64, _I, _P, _P, _P, _P, _P]),
    "bz_l2_fit_adjoint": (_I, [_P, _I64, _I, _I, _P, _I64, _P, _P, _P, _P, _P]),
    "bz_fit_adam_step": (_I, [_P, _P, _P, _I64, _I, _I, _I64, _P, _P, _P, _P, _I, _F, _F, _F, _F, _P, _P]),
    "bz_fit_adam_run": (_I, [_P, _P, _P, _I64, _I, _I, _I64, _P, _P, _P, _P, _I, _I, _F, _F, _F, _F, _P, _P]),
}


def header_symbols():
    """Every function name the C header declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bz_[a-z_0-9]+)\s*\(", text, re.M)))


def lib():
    """Load libbz.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbz.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().bz_last_error().decode()


def status_string(code):
    return lib().bz_status_string(code).decode()


def check(rc):
    if rc != OK:
        raise BzError(rc, "%s: %s" % (status_string(rc), last_error()))


def _ptr(x):
    if x is None:
        return None
    assert x.is_cuda and x.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return x.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dtype(x):
    try:
        return _DT[x.dtype]
    except KeyError:
        raise BzError(ERR_DTYPE, "unsupported storage dtype %s" % x.dtype)


def _f32_only(what, *xs):
    """FP32 is the only type of parameters, gradients and adjoint inputs."""
    for x in xs:
        if x is not None and x.dtype != torch.float32:
            raise BzError(ERR_DTYPE, "%s must be float32 (got %s)" % (what, x.dtype))


def _tmode(t, n):
    _f32_only("t", t)
    if t.dim() == 1:
        return T_SHARED, t.shape[0]
    assert t.dim() == 2 and t.shape[0] == n, "t must be [n_t] or [n_curves, n_t]"
    return T_PER_OBJECT, t.shape[1]


def _f32_out(shape, device, out):
    if out is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    assert out.dtype == torch.float32 and tuple(out.shape) == tuple(shape) and out.is_contiguous()
    return out


# ---------------------------------------------------------------- curves
def eval_bezier(ctrl, t, method="decasteljau", out=None):
    """ctrl[n, dim, d+1] (f32/f16/bf16), t[n_t] or [n, n_t] f32 -> out[dim, n*n_t]."""
    n, dim, dp1 = ctrl.shape
    mode, nt = _tmode(t, n)
    out = _f32_out((dim, n * nt), ctrl.device, out)
    check(lib().bz_eval_bezier(_ptr(ctrl), _dtype(ctrl), n, dp1 - 1, dim, _ptr(t), nt, mode, METHODS[method],
                               _ptr(out), _stream()))
    return out


def bezier_to_seiler(ctrl, out=None):
    n, dim, dp1 = ctrl.shape
    out = _f32_out((n, dim, dp1), ctrl.device, out)
    check(lib().bz_bezier_to_seiler(_ptr(ctrl), _dtype(ctrl), n, dp1 - 1, dim, _ptr(out), _stream()))
    return out


def eval_seiler(seiler, t, out=None):
    n, dim, dp1 = seiler.shape
    mode, nt = _tmode(t, n)
    out = _f32_out((dim, n * nt), seiler.device, out)
    check(lib().bz_eval_seiler(_ptr(seiler), n, dp1 - 1, dim, _ptr(t), nt, mode, _ptr(out), _stream()))
    return out


def eval_rational(ctrl, w, t, method="decasteljau", kappa=64.0, out=None, n_fixed=None):
    """Rational curves; n_fixed (optional int32 device tensor of one element)
    is incremented by the number of points recomputed in FP64."""
    n, dim, dp1 = ctrl.shape
    assert w.shape == (n, dp1) and w.dtype == ctrl.dtype
    mode, nt = _tmode(t, n)
    out = _f32_out((dim, n * nt), ctrl.device, out)
    check(lib().bz_eval_rational(_ptr(ctrl), _ptr(w), _dtype(ctrl), n, dp1 - 1, dim, _ptr(t), nt, mode,
                                 METHODS[method], float(kappa), _ptr(out), _ptr(n_fixed), _stream()))
    return out


# ---------------------------------------------------------------- chains
def encode_piecewise(chain, out=None):
    """chain[2N+1, dim] -> zig-zag grid[N+1, 2, dim]."""
    m, dim = chain.shape
    nseg = (m - 1) // 2
    assert m == 2 * nseg + 1
    out = _f32_out((nseg + 1, 2, dim), chain.device, out)
    check(lib().bz_encode_piecewise(_ptr(chain), nseg, dim, _ptr(out), _stream()))
    return out


def encode_piecewise_noalloc(chain, out):
    """As encode_piecewise, through the allocation-free entry point (its
    workspace is the library's fixed per-device array); out is required, so
    nothing is allocated on this path either."""
    m, dim = chain.shape
    nseg = (m - 1) // 2
    assert m == 2 * nseg + 1
    _f32_only("chain and grid", chain, out)
    assert tuple(out.shape) == (nseg + 1, 2, dim) and out.is_contiguous()
    check(lib().bz_encode_piecewise_noalloc(_ptr(chain), nseg, dim, _ptr(out), _stream()))
    return out


def eval_piecewise(grid, T, out=None):
    """grid[N+1, 2, dim], T[n_q] -> out[dim, n_q]."""
    _f32_only("grid and T", grid, T)
    nseg = grid.shape[0] - 1
    dim = grid.shape[2]
    nq = T.shape[0]
    out = _f32_out((dim, nq), grid.device, out)
    check(lib().bz_eval_piecewise(_ptr(grid), nseg, dim, _ptr(T), nq, _ptr(out), _stream()))
    return out


def encode_piecewise_cubic(chain, out=None):
    """Cubic chain[3N+1, dim] -> two stacked zig-zag layers grid[N+1, 2, 2, dim]."""
    m, dim = chain.shape
    nseg = (m - 1) // 3
    assert m == 3 * nseg + 1
    out = _f32_out((nseg + 1, 2, 2, dim), chain.device, out)
    check(lib().bz_encode_piecewise_cubic(_ptr(chain), nseg, dim, _ptr(out), _stream()))
    return out


def eval_piecewise_cubic(grid, T, out=None):
    """grid[N+1, 2, 2, dim], T[n_q] -> out[dim, n_q]."""
    _f32_only("grid and T", grid, T)
    nseg, dim = grid.shape[0] - 1, grid.shape[3]
    nq = T.shape[0]
    out = _f32_out((dim, nq), grid.device, out)
    check(lib().bz_eval_piecewise_cubic(_ptr(grid), nseg, dim, _ptr(T), nq, _ptr(out), _stream()))
    return out


def hbm_probe(mode, src, dst, blocks_per_cu=4):
    """One streaming pass (mode "read", "write" or "copy") over float32 buffers."""
    m = {"read": 0, "write": 1, "copy": 2}[mode]
    check(lib().bz_hbm_probe(m, _ptr(src), _ptr(dst), dst.numel() if m else src.numel(), blocks_per_cu, _stream()))


def gather_probe(src, n_reads, vec16, sink):
    """n_reads random 128-byte-line reads of vec16 16-byte vectors from the
    float32 buffer src (the chain query's access pattern)."""
    check(lib().bz_gather_probe(_ptr(src), src.numel(), n_reads, vec16, _ptr(sink), _stream()))


def texture_texels(degree, mode):
    return lib().bz_texture_texels(degree, TEX_MODES[mode])


def build_texture(ctrl, mode, out=None):
    """FP32 ctrl[n, dim, d+1] -> emulated curve textures tex[n, dim, texels]."""
    n, dim, dp1 = ctrl.shape
    ntx = texture_texels(dp1 - 1, mode)
    out = _f32_out((n, dim, max(ntx, 1)), ctrl.device, out)
    check(lib().bz_build_texture(_ptr(ctrl), n, dp1 - 1, dim, TEX_MODES[mode], _ptr(out), _stream()))
    return out


def eval_texture(tex, degree, mode, t, frac_bits=8, rounding="nearest", out=None):
    """Sample emulated curve textures tex[n, dim, texels] at t ([n_t] shared
    or [n, n_t]) through the emulated linear filter -> out[dim, n*n_t]."""
    _f32_only("t", t)
    n, dim, _ = tex.shape
    per_object = t.dim() == 2
    nt = t.shape[-1]
    out = _f32_out((dim, n * nt), tex.device, out)
    check(lib().bz_eval_texture(_ptr(tex), n, degree, dim, TEX_MODES[mode], _ptr(t), nt,
                                T_PER_OBJECT if per_object else T_SHARED, frac_bits, TEX_ROUNDING[rounding],
                                _ptr(out), _stream()))
    return out


def build_texture_patch(ctrl, du, dv, mode, out=None):
    """FP32 patches [n, dim, (du+1)(dv+1)] -> emulated surface textures [n, dim, texels]."""
    n, dim, _ = ctrl.shape
    ntx = lib().bz_texture_patch_texels(du, dv, TEX_MODES[mode])
    out = _f32_out((n, dim, max(ntx, 1)), ctrl.device, out)
    check(lib().bz_build_texture_patch(_ptr(ctrl), n, du, dv, dim, TEX_MODES[mode], _ptr(out), _stream()))
    return out


def eval_texture_patch(tex, du, dv, mode, uv, frac_bits=8, rounding="nearest", out=None):
    """Surface textures read through the emulated filter at uv[n, n_per, 2] -> out[dim, n*n_per]."""
    n, dim, _ = tex.shape
    n_per = uv.shape[1]
    out = _f32_out((dim, n * n_per), tex.device, out)
    check(lib().bz_eval_texture_patch(_ptr(tex), n, du, dv, dim, TEX_MODES[mode], _ptr(uv), n_per, frac_bits,
                                      TEX_ROUNDING[rounding], _ptr(out), _stream()))
    return out


def eval_piecewise_texemu(grid, T, frac_bits=8, rounding="nearest", out=None):
    """Zig-zag grid[N+1, 2, dim] read by the emulated bilinear filter at T -> out[dim, n_q]."""
    nseg, dim = grid.shape[0] - 1, grid.shape[2]
    nq = T.shape[0]
    out = _f32_out((dim, nq), grid.device, out)
    check(lib().bz_eval_piecewise_texemu(_ptr(grid), nseg, dim, _ptr(T), nq, frac_bits, TEX_ROUNDING[rounding],
                                         _ptr(out), _stream()))
    return out


def eval_piecewise_texemu_tiled(tiles, n_seg, dim, T, frac_bits=8, rounding="nearest", out=None):
    """The chain's cache-line tiles (tile_piecewise) read by the emulated bilinear filter at T -> out[dim, n_q]."""
    nq = T.shape[0]
    out = _f32_out((dim, nq), tiles.device, out)
    check(lib().bz_eval_piecewise_texemu_tiled(_ptr(tiles), n_seg, dim, _ptr(T), nq, frac_bits,
                                               TEX_ROUNDING[rounding], _ptr(out), _stream()))
    return out


def tile_piecewise_cubic(grid, out=None):
    """Two-layer cubic grid[N+1, 2, 2, dim] -> cache-line tiles (flat float32)."""
    nseg, dim = grid.shape[0] - 1, grid.shape[3]
    n = lib().bz_piecewise_cubic_tiled_floats(nseg, dim)
    out = _f32_out((n,), grid.device, out)
    check(lib().bz_tile_piecewise_cubic(_ptr(grid), nseg, dim, _ptr(out), _stream()))
    return out


def eval_piecewise_cubic_tiled(tiles, n_seg, dim, T, out=None):
    _f32_only("tiles and T", tiles, T)
    nq = T.shape[0]
    out = _f32_out((dim, nq), tiles.device, out)
    check(lib().bz_eval_piecewise_cubic_tiled(_ptr(tiles), n_seg, dim, _ptr(T), nq, _ptr(out), _stream()))
    return out


PARTICLE_METHODS = {"polynomial": 0, "seiler": 1, "seiler_texture": 2, "table": 3}


def particle_ring_data(seg, method, samples=64):
    """Device ring representation for a particle method from seg[N, 3, 4]."""
    if method == "polynomial":
        return seg.contiguous()
    if method == "seiler":
        return bezier_to_seiler(seg)
    if method == "seiler_texture":
        return build_texture(seg, "seiler")
    return particle_ring_table(seg, samples)


def particle_ring_table(seg, samples=64, out=None):
    """Sampled table [3, N*samples] of the ring seg[N, 3, 4] (FP32) at t = j/samples."""
    _f32_only("seg", seg)
    n = seg.shape[0]
    assert tuple(seg.shape) == (n, 3, 4)
    out = _f32_out((3, n * samples), seg.device, out)
    check(lib().bz_particle_ring_table(_ptr(seg), n, samples, _ptr(out), _stream()))
    return out


def particles_step(method, ring, n_seg, T, speed, dt, iters, samples=64, pos=None, shade=None):
    """One frame: updates T in place, returns (pos[3, P], shade[P])."""
    P = T.shape[0]
    pos = _f32_out((3, P), T.device, pos)
    shade = _f32_out((P,), T.device, shade)
    check(lib().bz_particles_step(PARTICLE_METHODS[method], _ptr(ring), n_seg, samples, _ptr(T), _ptr(speed), dt, P,
                                  iters, _ptr(pos), _ptr(shade), _stream()))
    return pos, shade


def tile_piecewise(grid, out=None):
    """Zig-zag grid[N+1, 2, dim] -> cache-line tiles (flat float32, 128-byte aligned)."""
    nseg = grid.shape[0] - 1
    dim = grid.shape[2]
    n = lib().bz_piecewise_tiled_floats(nseg, dim)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=grid.device)
    assert out.numel() == n and out.data_ptr() % 128 == 0
    check(lib().bz_tile_piecewise(_ptr(grid), nseg, dim, _ptr(out), _stream()))
    return out


def eval_piecewise_tiled(tiles, n_seg, dim, T, out=None):
    _f32_only("tiles and T", tiles, T)
    nq = T.shape[0]
    out = _f32_out((dim, nq), tiles.device, out)
    check(lib().bz_eval_piecewise_tiled(_ptr(tiles), n_seg, dim, _ptr(T), nq, _ptr(out), _stream()))
    return out


def tile_piecewise16(grid, dtype=torch.float16, out=None):
    """Zig-zag grid[N+1, 2, dim] (float32) -> cache-line tiles with 16-bit
    texels (dtype float16 or bfloat16; flat, 128-byte aligned)."""
    _f32_only("grid", grid)
    nseg = grid.shape[0] - 1
    dim = grid.shape[2]
    n = lib().bz_piecewise_tiled16_halfs(nseg, dim)
    if out is None:
        out = torch.empty(n, dtype=dtype, device=grid.device)
    assert out.numel() == n and out.data_ptr() % 128 == 0
    check(lib().bz_tile_piecewise16(_ptr(grid), nseg, dim, _dtype(out), _ptr(out), _stream()))
    return out


def eval_piecewise_tiled16(tiles, n_seg, dim, T, out=None):
    _f32_only("T", T)
    nq = T.shape[0]
    out = _f32_out((dim, nq), tiles.device, out)
    check(lib().bz_eval_piecewise_tiled16(_ptr(tiles), _dtype(tiles), n_seg, dim, _ptr(T), nq, _ptr(out), _stream()))
    return out


# ---------------------------------------------------------------- tensor
def eval_tensor_patch(ctrl, du, dv, dw=0, uvw=None, nu=0, nv=0, engine="valu", out=None):
    _f32_only("uvw", uvw)
    n, dim, _ = ctrl.shape
    if uvw is None:
        nq, n_per = n * nu * nv, 0
    else:
        n_per = uvw.shape[1]
        nq = n * n_per
    out = _f32_out((dim, nq), ctrl.device, out)
    check(lib().bz_eval_tensor_patch(_ptr(ctrl), _dtype(ctrl), n, du, dv, dw, dim, _ptr(uvw), n_per, nu, nv,
                                     ENGINES[engine], _ptr(out), _stream()))
    return out


def tensor_to_seiler(ctrl, du, dv, dw=0, out=None):
    """FP32 tensor control points [n, dim, ncp] -> per-axis Seiler terms (same shape)."""
    n, dim, ncp = ctrl.shape
    out = _f32_out((n, dim, ncp), ctrl.device, out)
    check(lib().bz_tensor_to_seiler(_ptr(ctrl), n, du, dv, dw, dim, _ptr(out), _stream()))
    return out


def eval_tensor_seiler(sc, du, dv, dw=0, uvw=None, nu=0, nv=0, out=None):
    """Per-axis Seiler terms [n, dim, ncp] -> points (grid or uvw mode, as eval_tensor_patch)."""
    n, dim, _ = sc.shape
    if uvw is None:
        nq, n_per = n * nu * nv, 0
    else:
        n_per = uvw.shape[1]
        nq = n * n_per
    out = _f32_out((dim, nq), sc.device, out)
    check(lib().bz_eval_tensor_seiler(_ptr(sc), n, du, dv, dw, dim, _ptr(uvw), n_per, nu, nv, _ptr(out), _stream()))
    return out


# ---------------------------------------------------------------- batched
SCHEDULES = {"static": 0, "dynamic": 1}
SCHEDULES_BY_CODE = {v: k for k, v in SCHEDULES.items()}


class BatchPlan:
    """Plan for a mixed batch (see bz_batch_plan_create)."""

    def __init__(self, kind_degree, cp_offset, ctrl, w, dim, knot_offset, knots, n_t, method="bernstein"):
        self.n_obj = kind_degree.shape[0]
        self.dim, self.n_t = dim, n_t
        self.device = ctrl.device
        h = _P()
        check(lib().bz_batch_plan_create(self.n_obj, _ptr(kind_degree), _ptr(cp_offset), _ptr(ctrl), _ptr(w),
                                         _dtype(ctrl), dim, _ptr(knot_offset), _ptr(knots), n_t, METHODS[method],
                                         _stream(), ctypes.byref(h)))
        self._h = h

    def info(self):
        buf = (ctypes.c_int64 * 4)()
        check(lib().bz_batch_plan_info(self._h, ctypes.cast(buf, _P)))
        return {"n_classes": buf[0], "n_tiles": buf[1], "n_segments": buf[2], "workgroups": buf[3]}

    def autotune(self, t, out):
        buf = (ctypes.c_int64 * 6)()
        check(lib().bz_batch_plan_autotune(self._h, _ptr(t), _ptr(out), _stream(), ctypes.cast(buf, _P)))
        return {"workgroups": buf[0], "tile_multiple": buf[1], "us_per_launch": buf[2],
                "schedule": SCHEDULES_BY_CODE[buf[3]], "queries_per_lane": buf[4], "window": buf[5]}

    def configure(self, workgroups, sub_tiles=1, schedule="dynamic", queries_per_lane=1, window=0):
        """schedule: "dynamic" (atomic tile counter) or "static" (round robin)."""
        check(lib().bz_batch_plan_configure(self._h, workgroups, sub_tiles, SCHEDULES[schedule], queries_per_lane,
                                            window, _stream()))

    def __call__(self, t, out=None, v=None):
        """t[n_obj, n_t] (a patch's u) and, for plans with surface patches,
        v[n_obj, n_t] (a patch's v) -> out[dim, n_obj*n_t]."""
        _f32_only("t and v", t, v)
        assert t.shape == (self.n_obj, self.n_t) and (v is None or v.shape == t.shape)
        out = _f32_out((self.dim, self.n_obj * self.n_t), self.device, out)
        if v is None:
            check(lib().bz_batch_eval(self._h, _ptr(t), _ptr(out), _stream()))
        else:
            check(lib().bz_batch_eval_uv(self._h, _ptr(t), _ptr(v), _ptr(out), _stream()))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().bz_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- adjoint
def adjoint_bezier(ctrl, t, grad_out, w=None, need_ctrl=True, need_w=None, need_t=True):
    """Returns (grad_ctrl, grad_w, grad_t), FP32; entries not requested are
    None.  ctrl, w, t and grad_out must be FP32 (the adjoint's storage type)."""
    _f32_only("adjoint inputs (ctrl, w, t, grad_out)", ctrl, w, t, grad_out)
    n, dim, dp1 = ctrl.shape
    mode, nt = _tmode(t, n)
    need_w = (w is not None) if need_w is None else need_w
    dev = ctrl.device
    gc = torch.empty((n, dim, dp1), dtype=torch.float32, device=dev) if need_ctrl else None
    gw = torch.empty((n, dp1), dtype=torch.float32, device=dev) if need_w else None
    gt = torch.empty((n, nt), dtype=torch.float32, device=dev) if need_t else None
    check(lib().bz_adjoint_bezier(_ptr(ctrl), _ptr(w), n, dp1 - 1, dim, _ptr(t), nt, mode, _ptr(grad_out), _ptr(gc),
                                  _ptr(gw), _ptr(gt), _stream()))
    return gc, gw, gt


def l2_fit_adjoint(ctrl, t, y, need_loss=True, need_ctrl=True, need_t=True):
    """Least-squares loss L = sum |C(t) - y|^2 / (n*n_t) of integral curves
    ctrl[n, dim, d+1] at per-curve t[n, n_t] against y[dim, n*n_t] (all FP32):
    returns (loss_part[n], grad_ctrl, grad_t), each None when not requested.
    No optimiser step; inputs are not modified."""
    _f32_only("l2_fit_adjoint inputs", ctrl, t, y)
    n, dim, dp1 = ctrl.shape
    assert t.dim() == 2 and t.shape[0] == n, "t must be [n_curves, n_t]"
    nt = t.shape[1]
    assert tuple(y.shape) == (dim, n * nt)
    dev = ctrl.device
    lp = torch.empty(n, dtype=torch.float32, device=dev) if need_loss else None
    gc = torch.empty((n, dim, dp1), dtype=torch.float32, device=dev) if need_ctrl else None
    gt = torch.empty((n, nt), dtype=torch.float32, device=dev) if need_t else None
    check(lib().bz_l2_fit_adjoint(_ptr(ctrl), n, dp1 - 1, dim, _ptr(t), nt, _ptr(y), _ptr(lp), _ptr(gc), _ptr(gt),
                                  _stream()))
    return lp, gc, gt


def fit_adam_step(ctrl, t, y, m_ctrl, v_ctrl, m_t, v_t, step, lr=1e-2, betas=(0.9, 0.999), eps=1e-8,
                  loss_part=None):
    n, dim, dp1 = ctrl.shape
    nt = t.shape[1]
    check(lib().bz_fit_adam_step(_ptr(ctrl), _ptr(t), _ptr(y), n, dp1 - 1, dim, nt, _ptr(m_ctrl), _ptr(v_ctrl),
                                 _ptr(m_t), _ptr(v_t), step, lr, betas[0], betas[1], eps, _ptr(loss_part),
                                 _stream()))


def fit_adam_run(ctrl, t, y, m_ctrl, v_ctrl, m_t, v_t, first_step, n_steps, lr=1e-2, betas=(0.9, 0.999),
                 eps=1e-8, loss_part=None):
    n, dim, dp1 = ctrl.shape
    nt = t.shape[1]
    check(lib().bz_fit_adam_run(_ptr(ctrl), _ptr(t), _ptr(y), n, dp1 - 1, dim, nt, _ptr(m_ctrl), _ptr(v_ctrl),
                                _ptr(m_t), _ptr(v_t), first_step, n_steps, lr, betas[0], betas[1], eps,
                                _ptr(loss_part), _stream()))


class BezierCurve(torch.autograd.Function):
    """Differentiable curve evaluation: forward by eval_bezier (rational when
    w is given), backward by the hand-written adjoint kernel.  t must be per
    curve ([n, n_t]) to receive a gradient."""

    @staticmethod
    def forward(ctx, ctrl, t, w=None, method="decasteljau"):
        ctx.save_for_backward(ctrl, t, w)
        if w is None:
            return eval_bezier(ctrl, t, method)
        return eval_rational(ctrl, w, t, method)

    @staticmethod
    def backward(ctx, grad_out):
        ctrl, t, w = ctx.saved_tensors
        need_t = ctx.needs_input_grad[1]
        if need_t and t.dim() != 2:
            raise BzError(ERR_UNSUPPORTED, "gradient w.r.t. a shared t is not provided; pass t as [n, n_t]")
        # the adjoint runs in FP32: FP16/BF16 control points and weights are
        # widened (exactly) for it, and their gradients rounded back to the
        # storage type torch expects
        c32 = ctrl.float().contiguous()
        w32 = w.float().contiguous() if w is not None else None
        gc, gw, gt = adjoint_bezier(c32, t, grad_out.float().contiguous(), w=w32,
                                    need_ctrl=ctx.needs_input_grad[0],
                                    need_w=w is not None and ctx.needs_input_grad[2], need_t=need_t)
        if gc is not None:
            gc = gc.to(ctrl.dtype)
        if gw is not None:
            gw = gw.to(w.dtype)
        return gc, gt, gw, None


def bezier_curve(ctrl, t, w=None, method="decasteljau"):
    return BezierCurve.apply(ctrl, t, w, method)
