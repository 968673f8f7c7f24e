"""CPU-only checks of the C ABI: the library loads without a GPU, exports
every symbol the header declares, and rejects bad arguments with the
documented status codes before anything is launched."""
import ctypes

import pytest

import paper_2603_15447_amd as bz

FAKE = 0x10000  # a non-NULL, 256-byte aligned address; never dereferenced
ODD = 0x10002


@pytest.fixture(scope="module")
def L():
    return bz.lib()


def test_exports_every_header_symbol(L):
    syms = bz.header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(bz._SIGS)


def test_status_strings(L):
    assert L.bz_version() >= 10000
    for code in range(9):
        assert bz.status_string(code)
    assert bz.status_string(99) == "unknown status"


@pytest.mark.parametrize("degree,dim,code", [(0, 3, bz.ERR_SHAPE), (16, 3, bz.ERR_SHAPE), (3, 0, bz.ERR_SHAPE),
                                             (3, 5, bz.ERR_SHAPE)])
def test_bezier_shape_errors(L, degree, dim, code):
    rc = L.bz_eval_bezier(FAKE, bz.F32, 4, degree, dim, FAKE, 8, bz.T_SHARED, bz.BERNSTEIN, FAKE, None)
    assert rc == code
    assert "bz_eval_bezier" in bz.last_error()


def test_bezier_other_errors(L):
    assert L.bz_eval_bezier(FAKE, 7, 4, 3, 3, FAKE, 8, 0, 0, FAKE, None) == bz.ERR_DTYPE
    assert L.bz_eval_bezier(FAKE, 0, 4, 3, 3, FAKE, 8, 0, 9, FAKE, None) == bz.ERR_UNSUPPORTED
    assert L.bz_eval_bezier(FAKE, 0, 4, 3, 3, FAKE, 8, 5, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_bezier(None, 0, 4, 3, 3, FAKE, 8, 0, 0, FAKE, None) == bz.ERR_NULL
    assert L.bz_eval_bezier(FAKE, 0, 4, 3, 3, FAKE, 8, 0, 0, None, None) == bz.ERR_NULL
    assert L.bz_eval_bezier(ODD, 0, 4, 3, 3, FAKE, 8, 0, 0, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_eval_bezier(FAKE, 0, -1, 3, 3, FAKE, 8, 0, 0, FAKE, None) == bz.ERR_SHAPE
    # F16 storage needs only 2-byte alignment
    assert L.bz_eval_bezier(ODD, 1, 0, 3, 3, FAKE, 8, 0, 0, FAKE, None) == bz.OK
    # BZ_AUTO passes the method check (and then fails on the NULL ctrl); 4 is no method
    assert L.bz_eval_bezier(None, 0, 4, 3, 3, FAKE, 8, 0, bz.AUTO, FAKE, None) == bz.ERR_NULL
    assert L.bz_eval_bezier(None, 0, 4, 3, 3, FAKE, 8, 0, 4, FAKE, None) == bz.ERR_UNSUPPORTED
    assert L.bz_eval_rational(None, FAKE, 0, 4, 3, 3, FAKE, 8, 0, bz.AUTO, 64.0, FAKE, None, None) == bz.ERR_NULL
    assert L.bz_eval_rational(None, FAKE, 0, 4, 3, 3, FAKE, 8, 0, 4, 64.0, FAKE, None, None) == bz.ERR_UNSUPPORTED


def test_zero_size_calls_launch_nothing(L):
    # NULL pointers are fine when there is nothing to do
    assert L.bz_eval_bezier(None, 0, 0, 3, 3, None, 8, 0, 0, None, None) == bz.OK
    assert L.bz_eval_bezier(None, 0, 5, 3, 3, None, 0, 0, 0, None, None) == bz.OK
    assert L.bz_eval_seiler(None, 0, 3, 3, None, 4, 0, None, None) == bz.OK
    assert L.bz_eval_rational(None, None, 0, 0, 3, 3, None, 4, 0, 0, 64.0, None, None, None) == bz.OK
    assert L.bz_bezier_to_seiler(None, 0, 0, 3, 3, None, None) == bz.OK
    assert L.bz_encode_piecewise(None, 0, 3, None, None) == bz.OK
    assert L.bz_eval_piecewise(None, 4, 3, None, 0, None, None) == bz.OK


def test_rational_and_seiler_errors(L):
    assert L.bz_eval_rational(FAKE, None, 0, 4, 3, 3, FAKE, 8, 0, 0, 64.0, FAKE, None, None) == bz.ERR_NULL
    assert L.bz_eval_rational(FAKE, FAKE, 3, 4, 3, 3, FAKE, 8, 0, 0, 64.0, FAKE, None, None) == bz.ERR_DTYPE
    assert L.bz_eval_rational(FAKE, FAKE, 0, 4, 3, 3, FAKE, 8, 0, 0, 64.0, FAKE, ODD, None) == bz.ERR_ALIGN
    assert L.bz_eval_seiler(FAKE, 4, 16, 3, FAKE, 8, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_bezier_to_seiler(FAKE, 0, 4, 3, 9, FAKE, None) == bz.ERR_SHAPE


def test_piecewise_errors(L):
    assert L.bz_eval_piecewise(FAKE, 0, 3, FAKE, 10, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise(FAKE, 4, 5, FAKE, 10, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise(FAKE + 4, 4, 3, FAKE, 10, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise(None, 4, 3, FAKE, 10, FAKE, None) == bz.ERR_NULL
    assert L.bz_encode_piecewise(FAKE, -2, 3, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_encode_piecewise(FAKE, 4, 3, None, None) == bz.ERR_NULL


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    """The binding raises when the library is missing; it never computes on the CPU."""
    monkeypatch.setattr(bz, "_lib", None)
    monkeypatch.setattr(bz, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        bz.lib()


def test_cubic_chain_errors(L):
    assert L.bz_encode_piecewise_cubic(None, 0, 3, None, None) == bz.OK
    assert L.bz_encode_piecewise_cubic(FAKE, 4, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_encode_piecewise_cubic(None, 4, 3, FAKE, None) == bz.ERR_NULL
    assert L.bz_eval_piecewise_cubic(FAKE, 0, 3, FAKE, 10, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_cubic(FAKE + 8, 4, 3, FAKE, 10, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise_cubic(FAKE, 4, 3, FAKE, 0, FAKE, None) == bz.OK
    assert L.bz_piecewise_cubic_tiled_floats(1000, 3) == 500 * 32  # 2 segments per 128-byte tile in 3D
    assert L.bz_piecewise_cubic_tiled_floats(9, 1) == 32 and L.bz_piecewise_cubic_tiled_floats(0, 3) == 0
    assert L.bz_tile_piecewise_cubic(FAKE, 4, 3, FAKE + 4, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise_cubic_tiled(FAKE, 4, 7, FAKE, 10, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_piecewise_tiled_floats(1 << 20, 3) == (1 << 18) * 32  # 4 segments per tile


def test_tiled16_chain_errors(L):
    S3 = 32 // 3 - 1  # 9 segments per 128-byte tile of 16-bit texels in 3D
    assert L.bz_piecewise_tiled16_halfs(1 << 20, 3) == -(-(1 << 20) // S3) * 64
    assert L.bz_piecewise_tiled16_halfs(9, 3) == 64 and L.bz_piecewise_tiled16_halfs(10, 3) == 128
    assert L.bz_piecewise_tiled16_halfs(31, 1) == 64 and L.bz_piecewise_tiled16_halfs(7, 4) == 64
    assert L.bz_piecewise_tiled16_halfs(0, 3) == 0 and L.bz_piecewise_tiled16_halfs(10, 5) == 0
    assert L.bz_tile_piecewise16(FAKE, 4, 3, bz.F32, FAKE, None) == bz.ERR_DTYPE
    assert L.bz_tile_piecewise16(FAKE, 4, 3, 7, FAKE, None) == bz.ERR_DTYPE
    assert L.bz_tile_piecewise16(FAKE, 4, 5, bz.F16, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_tile_piecewise16(FAKE, 4, 3, bz.F16, FAKE + 64, None) == bz.ERR_ALIGN
    assert L.bz_tile_piecewise16(None, 4, 3, bz.BF16, FAKE, None) == bz.ERR_NULL
    assert L.bz_tile_piecewise16(None, 0, 3, bz.F16, None, None) == bz.OK
    assert L.bz_eval_piecewise_tiled16(FAKE, bz.F32, 4, 3, FAKE, 10, FAKE, None) == bz.ERR_DTYPE
    assert L.bz_eval_piecewise_tiled16(FAKE, bz.F16, 4, 0, FAKE, 10, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_tiled16(FAKE, bz.F16, 0, 3, FAKE, 10, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_tiled16(FAKE + 64, bz.BF16, 4, 3, FAKE, 10, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise_tiled16(FAKE, bz.F16, 4, 3, FAKE + 2, 10, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise_tiled16(None, bz.F16, 4, 3, FAKE, 10, FAKE, None) == bz.ERR_NULL
    assert L.bz_eval_piecewise_tiled16(FAKE, bz.F16, 4, 3, FAKE, 0, FAKE, None) == bz.OK


def test_texture_errors(L):
    assert [L.bz_texture_texels(d, 0) for d in (1, 2, 3, 8, 9)] == [0, 4, 8, 28, 0]
    assert [L.bz_texture_texels(d, 2) for d in (1, 2, 3, 4, 7, 8)] == [0, 4, 4, 8, 8, 0]
    assert L.bz_texture_texels(3, 5) == 0
    assert L.bz_build_texture(FAKE, 4, 8, 3, 2, FAKE, None) == bz.ERR_UNSUPPORTED
    assert L.bz_build_texture(FAKE, 4, 3, 3, 0, FAKE + 4, None) == bz.ERR_ALIGN
    assert L.bz_eval_texture(FAKE, 4, 3, 3, 0, FAKE, 8, 0, 21, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_texture(FAKE, 4, 3, 3, 0, FAKE, 8, 0, 8, 2, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_texture(FAKE, 4, 3, 3, 1, FAKE, 8, 3, 8, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_texture(None, 4, 3, 3, 1, FAKE, 8, 0, 8, 0, FAKE, None) == bz.ERR_NULL
    assert L.bz_eval_piecewise_texemu(FAKE, 1 << 25, 3, FAKE, 8, 8, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_texemu(FAKE + 4, 4, 3, FAKE, 8, 8, 0, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_texture_patch_texels(3, 3, 0) == 32 and L.bz_texture_patch_texels(2, 4, 2) == 20
    assert L.bz_texture_patch_texels(4, 3, 0) == 0 and L.bz_texture_patch_texels(3, 3, 1) == 0
    assert L.bz_build_texture_patch(FAKE, 4, 3, 5, 3, 2, FAKE, None) == bz.ERR_UNSUPPORTED
    assert L.bz_eval_texture_patch(FAKE, 4, 3, 3, 3, 2, FAKE + 4, 8, 8, 0, FAKE, None) == bz.ERR_ALIGN


def test_tensor_seiler_and_patch_errors(L):
    assert L.bz_tensor_to_seiler(FAKE, 4, 5, 3, 0, 3, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_tensor_to_seiler(None, 0, 3, 3, 0, 3, None, None) == bz.OK
    assert L.bz_eval_tensor_seiler(FAKE, 4, 3, 3, 1, 3, None, 0, 32, 32, FAKE, None) == bz.ERR_UNSUPPORTED
    assert L.bz_eval_tensor_seiler(FAKE, 4, 3, 3, 0, 3, None, 0, 0, 32, FAKE, None) == bz.ERR_SHAPE
    # MFMA engines: bicubic FP32 on 32x32 only; FP16x3 is engine 4, 5 is unknown
    assert L.bz_eval_tensor_patch(FAKE, 0, 4, 3, 3, 0, 3, None, 0, 16, 16, 4, FAKE, None) == bz.ERR_UNSUPPORTED
    assert L.bz_eval_tensor_patch(FAKE, 0, 4, 3, 3, 0, 3, None, 0, 32, 32, 5, FAKE, None) == bz.ERR_UNSUPPORTED


def test_particles_probe_and_plan_errors(L):
    assert L.bz_particles_step(4, FAKE, 16, 64, FAKE, FAKE, ctypes.c_float(0.01), 8, 0, FAKE, FAKE, None) \
        == bz.ERR_UNSUPPORTED
    assert L.bz_particles_step(3, FAKE, 16, 0, FAKE, FAKE, ctypes.c_float(0.01), 8, 0, FAKE, FAKE, None) \
        == bz.ERR_SHAPE
    assert L.bz_particles_step(0, FAKE + 4, 16, 64, FAKE, FAKE, ctypes.c_float(0.01), 8, 0, FAKE, FAKE, None) \
        == bz.ERR_ALIGN
    assert L.bz_particles_step(0, FAKE, 16, 64, FAKE, FAKE, ctypes.c_float(0.01), 0, 0, None, None, None) == bz.OK
    assert L.bz_hbm_probe(3, FAKE, FAKE, 16, 4, None) == bz.ERR_SHAPE
    assert L.bz_hbm_probe(2, FAKE, FAKE, 6, 4, None) == bz.ERR_SHAPE
    assert L.bz_hbm_probe(2, FAKE, FAKE, 16, -1, None) == bz.ERR_SHAPE
    assert L.bz_hbm_probe(2, FAKE, FAKE, 16, 65, None) == bz.ERR_SHAPE
    assert L.bz_hbm_probe(1, None, FAKE + 4, 16, 4, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise_texemu_tiled(FAKE + 64, 16, 3, FAKE, 8, 8, 0, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_eval_piecewise_texemu_tiled(FAKE, 16, 5, FAKE, 8, 8, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_texemu_tiled(FAKE, 0, 3, FAKE, 8, 8, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_texemu_tiled(FAKE, 16, 3, FAKE, 8, 21, 0, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_eval_piecewise_texemu_tiled(None, 16, 3, FAKE, 8, 8, 0, FAKE, None) == bz.ERR_NULL
    assert L.bz_eval_piecewise_texemu_tiled(None, 16, 3, None, 0, 8, 0, None, None) == bz.OK
    assert L.bz_gather_probe(FAKE, 64, 8, 5, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_gather_probe(FAKE, 48, 8, 3, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_gather_probe(FAKE, 0, 8, 3, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_gather_probe(FAKE, 64, -1, 3, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_gather_probe(FAKE, 64, 1 << 31, 3, FAKE, None) == bz.ERR_SHAPE
    assert L.bz_gather_probe(None, 64, 8, 3, FAKE, None) == bz.ERR_NULL
    assert L.bz_gather_probe(FAKE + 64, 64, 8, 3, FAKE, None) == bz.ERR_ALIGN
    assert L.bz_gather_probe(FAKE, 64, 0, 3, None, None) == bz.OK
    assert L.bz_batch_plan_configure(None, 64, 1, 1, 1, 0, None) == bz.ERR_NULL
    assert L.bz_batch_plan_autotune(None, FAKE, FAKE, None, None) == bz.ERR_NULL
    assert L.bz_batch_eval(None, FAKE, FAKE, None) == bz.ERR_NULL


def test_l2_fit_adjoint_errors(L):
    f = L.bz_l2_fit_adjoint
    assert f(FAKE, 4, 0, 3, FAKE, 8, FAKE, FAKE, FAKE, FAKE, None) == bz.ERR_SHAPE
    assert f(FAKE, 4, 16, 3, FAKE, 8, FAKE, FAKE, FAKE, FAKE, None) == bz.ERR_SHAPE
    assert f(FAKE, 4, 3, 5, FAKE, 8, FAKE, FAKE, FAKE, FAKE, None) == bz.ERR_SHAPE
    assert f(FAKE, -1, 3, 3, FAKE, 8, FAKE, FAKE, FAKE, FAKE, None) == bz.ERR_SHAPE
    assert f(None, 4, 3, 3, FAKE, 8, FAKE, FAKE, FAKE, FAKE, None) == bz.ERR_NULL
    assert f(FAKE, 4, 3, 3, FAKE, 8, None, FAKE, FAKE, FAKE, None) == bz.ERR_NULL
    assert f(FAKE, 4, 3, 3, FAKE, 8, FAKE, FAKE, ODD, FAKE, None) == bz.ERR_ALIGN
    # nothing to do: no pointer is needed
    assert f(None, 0, 3, 3, None, 8, None, None, None, None, None) == bz.OK
    assert f(None, 4, 3, 3, None, 0, None, None, None, None, None) == bz.OK
    assert "bz_l2_fit_adjoint" in (bz.last_error() or "bz_l2_fit_adjoint")


def test_half_precision_inputs_are_refused_where_only_fp32_is_read():
    # the adjoint reads FP32 only: half-precision control points, weights,
    # parameters or incoming gradients are rejected before any pointer is
    # passed on (the autograd backward widens them to FP32 first)
    import torch
    c32 = torch.zeros(2, 3, 4)
    t32 = torch.zeros(2, 5)
    g32 = torch.zeros(3, 10)
    for bad in ({"ctrl": c32.half()}, {"t": t32.half()}, {"grad_out": g32.bfloat16()},
                {"w": torch.ones(2, 4, dtype=torch.float16)}):
        args = {"ctrl": c32, "t": t32, "grad_out": g32, **bad}
        with pytest.raises(bz.BzError) as e:
            bz.adjoint_bezier(args["ctrl"], args["t"], args["grad_out"], w=args.get("w"))
        assert e.value.code == bz.ERR_DTYPE
    with pytest.raises(bz.BzError) as e:
        bz.eval_bezier(c32, t32.half())
    assert e.value.code == bz.ERR_DTYPE
    with pytest.raises(bz.BzError) as e:
        bz.l2_fit_adjoint(c32, t32, g32.half())
    assert e.value.code == bz.ERR_DTYPE


def test_particle_ring_table_errors(L):
    f = L.bz_particle_ring_table
    assert f(FAKE, 0, 64, FAKE, None) == bz.ERR_SHAPE
    assert f(FAKE, 16, 0, FAKE, None) == bz.ERR_SHAPE
    assert f(FAKE, 1 << 20, 64, FAKE, None) == bz.ERR_SHAPE  # more than 2^24 samples
    assert f(None, 16, 64, FAKE, None) == bz.ERR_NULL
    assert f(FAKE, 16, 64, ODD, None) == bz.ERR_ALIGN


C_CONSUMER = r"""
#include <stdio.h>
#include <string.h>
#include "bz.h"

/* A plain C99 caller of the library: no HIP or C++ header involved. */
int main(void) {
    const float fake = 0.0f;
    int rc;
    if (bz_version() < 10000) return 1;
    if (strcmp(bz_status_string(BZ_OK), bz_status_string(BZ_ERR_SHAPE)) == 0) return 2;
    /* degree 16 is out of range: rejected before any device work */
    rc = bz_eval_bezier(&fake, BZ_F32, 4, 16, 3, &fake, 8, BZ_T_SHARED, BZ_BERNSTEIN, (float *)&fake, 0);
    if (rc != BZ_ERR_SHAPE) return 3;
    if (strstr(bz_last_error(), "bz_eval_bezier") == NULL) return 4;
    printf("ok %d\n", bz_version());
    return 0;
}
"""


def test_header_serves_a_plain_c_caller(tmp_path):
    """include/bz.h compiles as strict C99 (no C++ or HIP header needed),
    and a C program linked against libbz.so gets the documented status
    codes back (argument checks only: nothing reaches a device)."""
    import os
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "consumer.c"
    src.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(bz.LIB_PATH)
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I" + os.path.join(root, "include"),
           str(src), "-L" + libdir, "-lbz", "-Wl,-rpath," + libdir, "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok "), (r.returncode, r.stdout, r.stderr)
