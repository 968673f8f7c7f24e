"""GPU parity through the C ABI from plain C programs, with no PyTorch in
the process: each program allocates device memory with the HIP runtime API,
calls the library on a stream of its own and writes the points to a file,
which the test compares with the FP64 oracle: curves in each form (Sec. 2:
the curve is the same whichever form evaluates it), and a mixed batch plan
(curves, rational curves and NURBS; Sec. 2.2) created, evaluated, autotuned,
evaluated again and destroyed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import bz_synth
import paper_2603_15447_amd as bz
from tests._batch import _extents
from tests._gpu import TOL_F32, bbox_err, extents

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_PROGRAM = r"""
#include <stdio.h>
#include <stdlib.h>
#include <hip/hip_runtime_api.h>
#include "bz.h"

static int read_all(const char *path, void *dst, size_t bytes) {
    FILE *f = fopen(path, "rb");
    size_t got;
    if (!f) return 0;
    got = fread(dst, 1, bytes, f);
    fclose(f);
    return got == bytes;
}

/* argv: n_curves degree dim n_t method ctrl.bin t.bin out.bin */
int main(int argc, char **argv) {
    long n, nt;
    int degree, dim, method, rc;
    size_t nc, no;
    float *hc, *ht, *ho, *dc = NULL, *dt = NULL, *dout = NULL;
    hipStream_t s;
    FILE *f;
    if (argc != 9) return 10;
    n = atol(argv[1]);
    degree = atoi(argv[2]);
    dim = atoi(argv[3]);
    nt = atol(argv[4]);
    method = atoi(argv[5]);
    nc = (size_t)n * dim * (degree + 1);
    no = (size_t)n * nt * dim;
    hc = malloc(nc * sizeof(float));
    ht = malloc(nt * sizeof(float));
    ho = malloc(no * sizeof(float));
    if (!hc || !ht || !ho) return 11;
    if (!read_all(argv[6], hc, nc * sizeof(float)) || !read_all(argv[7], ht, nt * sizeof(float))) return 12;
    if (hipStreamCreate(&s) != hipSuccess) return 13;
    if (hipMalloc((void **)&dc, nc * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&dt, nt * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&dout, no * sizeof(float)) != hipSuccess) return 14;
    if (hipMemcpy(dc, hc, nc * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dt, ht, nt * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return 15;
    rc = bz_eval_bezier(dc, BZ_F32, n, degree, dim, dt, nt, BZ_T_SHARED, method, dout, (bz_stream)s);
    if (rc != BZ_OK) {
        fprintf(stderr, "bz_eval_bezier: %s\n", bz_last_error());
        return 16;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return 17;
    if (hipMemcpy(ho, dout, no * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return 18;
    f = fopen(argv[8], "wb");
    if (!f || fwrite(ho, sizeof(float), no, f) != no) return 19;
    fclose(f);
    hipFree(dc);
    hipFree(dt);
    hipFree(dout);
    hipStreamDestroy(s);
    free(hc);
    free(ht);
    free(ho);
    printf("ok\n");
    return 0;
}
"""


C_BATCH = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <hip/hip_runtime_api.h>
#include "bz.h"

/* a host file of `bytes` bytes copied into a new device buffer */
static void *upload(const char *path, size_t bytes) {
    void *h = malloc(bytes ? bytes : 4), *d = NULL;
    FILE *f = fopen(path, "rb");
    size_t got;
    if (!h || !f) return NULL;
    got = fread(h, 1, bytes, f);
    fclose(f);
    if (got != bytes || hipMalloc(&d, bytes ? bytes : 4) != hipSuccess) return NULL;
    if (bytes && hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return NULL;
    free(h);
    return d;
}

/* argv: n_obj n_t dim n_cp n_knots kd cpo ctrl w ko knots t out_first out_tuned */
int main(int argc, char **argv) {
    long n_obj, n_t, n_cp, n_k;
    int dim, i, rc;
    size_t no;
    void *kd, *cpo, *ctrl, *w, *ko, *knots, *t;
    float *out = NULL, *h;
    int64_t best[6];
    bz_plan plan = NULL;
    hipStream_t s;
    FILE *f;
    if (argc != 15) return 10;
    n_obj = atol(argv[1]);
    n_t = atol(argv[2]);
    dim = atoi(argv[3]);
    n_cp = atol(argv[4]);
    n_k = atol(argv[5]);
    kd = upload(argv[6], n_obj * sizeof(uint16_t));
    cpo = upload(argv[7], (n_obj + 1) * sizeof(int64_t));
    ctrl = upload(argv[8], n_cp * dim * sizeof(float));
    w = upload(argv[9], n_cp * sizeof(float));
    ko = upload(argv[10], (n_obj + 1) * sizeof(int64_t));
    knots = upload(argv[11], n_k * sizeof(float));
    t = upload(argv[12], n_obj * n_t * sizeof(float));
    if (!kd || !cpo || !ctrl || !w || !ko || !knots || !t) return 11;
    no = (size_t)n_obj * n_t * dim;
    h = malloc(no * sizeof(float));
    if (!h || hipMalloc((void **)&out, no * sizeof(float)) != hipSuccess) return 12;
    if (hipStreamCreate(&s) != hipSuccess) return 13;
    rc = bz_batch_plan_create(n_obj, kd, cpo, ctrl, w, BZ_F32, dim, ko, knots, n_t, BZ_BERNSTEIN, (bz_stream)s, &plan);
    if (rc != BZ_OK) {
        fprintf(stderr, "plan: %s\n", bz_last_error());
        return 14;
    }
    /* the descriptor arrays are no longer needed once the plan exists */
    hipFree(kd);
    hipFree(cpo);
    hipFree(ctrl);
    hipFree(w);
    hipFree(ko);
    hipFree(knots);
    for (i = 0; i < 2; ++i) {
        if (i == 1 && bz_batch_plan_autotune(plan, t, out, (bz_stream)s, best) != BZ_OK) return 15;
        if (hipMemsetAsync(out, 0xff, no * sizeof(float), s) != hipSuccess) return 16;
        if (bz_batch_eval(plan, t, out, (bz_stream)s) != BZ_OK) {
            fprintf(stderr, "eval: %s\n", bz_last_error());
            return 17;
        }
        if (hipStreamSynchronize(s) != hipSuccess) return 18;
        if (hipMemcpy(h, out, no * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return 19;
        f = fopen(argv[13 + i], "wb");
        if (!f || fwrite(h, sizeof(float), no, f) != no) return 20;
        fclose(f);
    }
    bz_plan_destroy(plan);
    hipFree(t);
    hipFree(out);
    hipStreamDestroy(s);
    free(h);
    printf("ok %lld\n", (long long)best[4]); /* queries per lane of the tuned launch */
    return 0;
}
"""


def _compile(tmp_path_factory, name, program):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp(name)
    src = d / (name + ".c")
    src.write_text(program)
    exe = d / name
    libdir = os.path.dirname(bz.LIB_PATH)
    cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-isystem", "/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), str(src), "-L" + libdir, "-lbz", "-Wl,-rpath," + libdir,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
    return exe, d


@pytest.fixture(scope="module")
def c_caller(tmp_path_factory):
    return _compile(tmp_path_factory, "caller", C_PROGRAM)


@pytest.fixture(scope="module")
def c_batch(tmp_path_factory):
    return _compile(tmp_path_factory, "batch", C_BATCH)


@pytest.mark.parametrize("method", [bz.DECASTELJAU, bz.BERNSTEIN, bz.SEILER])
@pytest.mark.parametrize("n_curves,degree,dim,n_t", [(4096, 3, 3, 256), (37, 7, 2, 67)])
def test_c_program_matches_oracle(orc, c_caller, method, n_curves, degree, dim, n_t):
    """The 4096-curve cubic 3D workload with 256 shared t, and a ragged
    degree-7 2D case, each form, within 1e-5 of the control-point box."""
    exe, d = c_caller
    if (n_curves, degree) == (4096, 3):
        ctrl, t = bz_synth.plain_curves(n_curves=n_curves, n_t=n_t)
    else:
        ctrl, t = bz_synth.random_curves(n_curves, degree, dim, n_t, seed=7 * degree + dim, per_object=False)
    tag = "%d_%d_%d_%d_%d" % (method, n_curves, degree, dim, n_t)
    cpath, tpath, opath = d / ("c%s.bin" % tag), d / ("t%s.bin" % tag), d / ("o%s.bin" % tag)
    np.ascontiguousarray(ctrl, np.float32).tofile(cpath)
    np.ascontiguousarray(t, np.float32).tofile(tpath)
    r = subprocess.run([str(exe), str(n_curves), str(degree), str(dim), str(n_t), str(method), str(cpath),
                        str(tpath), str(opath)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr)
    got = np.fromfile(opath, dtype=np.float32).reshape(dim, n_curves * n_t)
    ref = orc.bezier_decasteljau(ctrl, t)
    err = bbox_err(got, ref, extents(ctrl), n_t)
    assert err <= TOL_F32, (method, n_curves, degree, dim, err)


def test_c_program_runs_a_batch_plan(orc, c_batch):
    """A mixed batch (curves of degree 1..15, half rational, and cubic NURBS,
    16 random t each) through bz_batch_plan_create / bz_batch_eval /
    bz_batch_plan_autotune / bz_plan_destroy from C: both evaluations within
    1e-5 of each object's box of the oracle, and bit-identical to each other
    when the tuned launch keeps four parameters per lane (the default; the
    one-parameter mapping contracts its FMAs differently, 1 ulp apart)."""
    exe, d = c_batch
    b = bz_synth.mixed_batch(n_bezier=3000, n_nurbs=300, n_t=16, deg_lo=1, seed=77)
    arrays = {"kd": b.kind_degree.astype(np.uint16), "cpo": b.cp_offset.astype(np.int64),
              "ctrl": b.ctrl.astype(np.float32), "w": b.w.astype(np.float32), "ko": b.knot_offset.astype(np.int64),
              "knots": b.knots.astype(np.float32), "t": b.t.astype(np.float32)}
    paths = {}
    for k, a in arrays.items():
        paths[k] = d / (k + ".bin")
        np.ascontiguousarray(a).tofile(paths[k])
    n_cp = int(b.cp_offset[-1])
    assert b.ctrl.size == n_cp * b.dim and b.w.size == n_cp and b.t.size == b.n_obj * b.n_t
    o1, o2 = d / "out1.bin", d / "out2.bin"
    r = subprocess.run([str(exe), str(b.n_obj), str(b.n_t), str(b.dim), str(n_cp), str(b.knots.size)] +
                       [str(paths[k]) for k in ("kd", "cpo", "ctrl", "w", "ko", "knots", "t")] + [str(o1), str(o2)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok "), (r.returncode, r.stdout, r.stderr)
    first = np.fromfile(o1, dtype=np.float32).reshape(b.dim, b.n_obj * b.n_t)
    tuned = np.fromfile(o2, dtype=np.float32).reshape(b.dim, b.n_obj * b.n_t)
    if int(r.stdout.split()[1]) == 4:
        assert np.array_equal(first.view(np.uint32), tuned.view(np.uint32))
    ref = orc.batch_eval(b)
    for got in (first, tuned):
        d_ = np.abs(got.astype(np.float64) - ref)
        assert not np.isnan(d_).any()
        err = float((d_.max(axis=0).reshape(-1, b.n_t).max(axis=1) / _extents(b)).max())
        assert err <= TOL_F32, err
