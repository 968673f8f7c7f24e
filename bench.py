"""Benchmark of the Bezier-family evaluators on one MI355X.

Headline workload (the JSON line's `value`): plain FP32 evaluation of 4096
independent cubic 3D Bezier curves (control points U[-1,1]^3) at 256 uniform
t_j = j/255, by each of the three forms (de Casteljau lerps, the Bernstein
polynomial, Seiler interpolation).  One step is one replay of a HIP graph that
holds the three launches (3 x 2^20 evaluations); the inputs are resident in
HBM.  The final JSON line also carries, for the metric's comparison, the mixed
batch in one persistent launch (2^20 Bezier curves of degree 2..15, half
rational, plus 2^16 cubic NURBS, 16 random t each) with FP32 and with FP16
storage, each with its max error against the FP64 oracle, and the C0 quadratic
chain (2^20 segments, 2^24 random T) as a secondary record.

`--suite` runs the other workloads as well (each with its own kernel time,
roofline and CPU-baseline leg) and writes them to a JSON file (`--suite-out`);
the final stdout line stays compact.

Prints one JSON line on stdout (progress goes to stderr).
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak for code built without packed-FP32 instructions:
# 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# the published FP32 vector peak, which counts packed FP32 FMAs (two per lane)
FP32_PUBLISHED_TFLOPS = 157.3
METRIC = "G curve-point evals/s and % HBM roofline, plain FP32 vs batched/FP16 at max err"
CHAIN_COUNTERS = "chain_eval_counters.json"  # keys: grid, tiled, tiled16


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def chain_bytes(n_seg, dim, n_q, es=4):
    """Algorithmic HBM bytes of one evaluation launch: the texels once (es
    bytes each), T in, points out (FP32)."""
    return (n_seg + 1) * 2 * dim * es + n_q * 4 + n_q * dim * 4


def particle_frame_bytes(n):
    """Algorithmic HBM bytes of one particle frame: the phase T read and
    written, the speed read, three coordinates and the shade written (the
    16-segment ring itself stays in cache)."""
    return n * (4 + 4 + 4 + 3 * 4 + 4)


def recorded_traffic(name, workload, key=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when a kernel source it names has changed since the counters were
    taken, or the workload differs from the one they were taken on.  `key`
    picks one kernel of a summary that holds several."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
        srcs = d.get("kernel_sources") or {d["kernel_source"]: d["kernel_source_sha256"]}
        for path, want in srcs.items():
            with open(os.path.join(ROOT, path), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != want:
                    return None
        wl = d.get("workload") or {"n_seg": d["n_seg"], "n_q": d["n_q"]}
        if any(wl.get(k) != v for k, v in workload.items()):
            return None
        t = d["traffic_bytes_per_dispatch"]
        return t.get(key) if key is not None else t
    except (OSError, KeyError, ValueError, AttributeError):
        return None


def alu_roof(tflops):
    """FP32 VALU roofline of a rate: against the non-packed peak that the
    library, compiled without packed-FP32 instructions, can reach, and against
    the published (packed) peak beside it."""
    return {"bound": "alu", "achieved": tflops, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tflops / FP32_VALU_PEAK_TFLOPS, "published_peak": FP32_PUBLISHED_TFLOPS,
            "frac_of_published": tflops / FP32_PUBLISHED_TFLOPS}


def event_time_ms(fn, iters, torch):
    """Average device time of fn() over `iters` back-to-back launches, with
    HIP events recorded on the stream the kernels are launched on."""
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(iters):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / iters


def timed(fn, torch, iters=20, warmup=3):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    return event_time_ms(fn, iters, torch)


def graph_time_ms(fn, torch, launches=50, replays=5, trials=1):
    """Device time per launch of fn() with launch overhead removed: `launches`
    back-to-back calls captured once into a HIP graph (the library launches
    on torch's current stream, which is the capture stream here), the graph
    replayed `replays` times between HIP events; with trials > 1, the median
    over that many such timings of the same graph.  For kernels of a few
    microseconds, where issuing each launch from Python costs more than the
    kernel itself."""
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(launches):
            fn()
    g.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(trials):
        a.record(s)
        for _ in range(replays):
            g.replay()
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b) / (replays * launches))
    del g
    times.sort()
    return times[len(times) // 2]


def hbm_roof(nbytes, ms):
    a = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS}


def oracle_timed(fn, budget_s=10.0, max_reps=8):
    """Run an oracle call repeatedly for up to budget_s; returns (result, seconds per call, calls)."""
    t0 = time.perf_counter()
    reps, res = 0, None
    while True:
        res = fn()
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= max_reps:
            return res, el / reps, reps


def max_err_bbox(got, ref, ext, per_obj):
    d = np.abs(np.asarray(got, np.float64) - ref)
    if np.isnan(d).any():
        return float("inf")
    return float((d.max(axis=0).reshape(-1, per_obj).max(axis=1) / ext).max())


# a box side below this fraction of the object's largest |coordinate| cannot
# be resolved to 1e-5 by FP32 results (two roundings, 2 * 2^-24, exceed it)
FP32_RESOLVABLE = 2.0 ** -23 / 1e-5


def extents(ctrl):
    """Per-object error normaliser: the largest side of the control-point box,
    floored at FP32_RESOLVABLE of the largest |coordinate|."""
    c = np.asarray(ctrl, np.float64)
    side = (c.max(axis=2) - c.min(axis=2)).max(axis=1)
    return np.maximum(np.maximum(side, FP32_RESOLVABLE * np.abs(c).max(axis=(1, 2))), 1e-30)


def hbm_probe(torch, bz, mib=1024, iters=10):
    """Measured HBM ceiling: streaming read, write and copy of `mib` MiB with
    the library's probe kernels (best over persistent-grid sizes), timed with
    HIP events; copy counts read + write bytes."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    res = {"bytes": 4 * n}
    for mode in ("read", "write", "copy"):
        best = None
        for bpc in (0, 2, 4, 8, 16):  # 0: one 16-byte vector per thread
            ms = timed(lambda: bz.hbm_probe(mode, src, dst, bpc), torch, iters=iters)
            gbs = (2 if mode == "copy" else 1) * 4 * n / (ms * 1e-3) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, bpc)
        res[mode + "_GB/s"], res[mode + "_blocks_per_cu"] = best
    del src, dst
    return res


def gather_ceiling(torch, bz, buf, n_reads, kern_ms, vec16=3, iters=20):
    """The measured ceiling of the chain query's access pattern: as many
    reads of 16*vec16 contiguous bytes at the start of uniformly random
    128-byte lines of `buf` (the tiled grid itself, so the footprint is the
    grid's) as the chain has queries, and the evaluator's query rate as a
    fraction of that line rate."""
    sink = torch.zeros(1, dtype=torch.float32, device=buf.device)
    fn = lambda: bz.gather_probe(buf, n_reads, vec16, sink)
    for _ in range(3):
        fn()
    ms = event_time_ms(fn, iters, torch)
    rate = n_reads / (ms * 1e-3) / 1e9
    return {"G_lines/s": rate, "footprint_MB": buf.numel() * 4 / 1e6, "bytes_per_read": 16 * vec16, "probe_ms": ms,
            "evaluator_frac": (n_reads / (kern_ms * 1e-3) / 1e9) / rate}


def suite_chain_footprint(torch, bz, bz_synth, cpu):
    """The tiled chain evaluator and the random-line gather probe over chains
    of 2^15 .. 2^23 segments (tiled grid 1 MB .. 268 MB) at 2^24 queries: where
    the grid leaves an XCD's 4 MB L2 and the 256 MB Infinity Cache."""
    log("suite: chain footprint sweep")
    n_q, dim = 1 << 24, 3
    rows = []
    for lg in range(15, 24):
        n_seg = 1 << lg
        chain, T = bz_synth.chain_walk(n_seg=n_seg, dim=dim, n_q=n_q)
        chain_d, T_d = torch.from_numpy(chain).cuda(), torch.from_numpy(T).cuda()
        tiles = bz.tile_piecewise(bz.encode_piecewise(chain_d))
        out = torch.empty((dim, n_q), dtype=torch.float32, device="cuda")
        fn = lambda: bz.eval_piecewise_tiled(tiles, n_seg, dim, T_d, out=out)
        for _ in range(3):
            fn()
        ms = event_time_ms(fn, 20, torch)
        g = gather_ceiling(torch, bz, tiles, n_q, ms)
        rows.append({"n_seg": n_seg, "tiled_MB": g["footprint_MB"], "kernel_ms": ms,
                     "G evals/s": n_q / (ms * 1e-3) / 1e9, "gather_G_lines/s": g["G_lines/s"],
                     "frac_of_gather": g["evaluator_frac"],
                     "hbm_frac": hbm_roof(chain_bytes(n_seg, dim, n_q), ms)["frac"]})
        del chain_d, T_d, tiles, out
    return {"workload": "C0 quadratic chain (tiled), 2^15..2^23 segments, 2^24 uniform random global T, 3D, FP32",
            "unit": "G evals/s", "rows": rows}


# ---------------------------------------------------------------- headline
def cpu_baseline_chain(chain, T, out_dev, budget_s=10.0):
    """CPU-baseline leg: the oracle's chain definition on the first 4M queries,
    timed on the host cores; its outputs also give the GPU's error there."""
    import oracle
    m = min(T.shape[0], 1 << 22)
    ref, sec, reps = oracle_timed(lambda: oracle.chain_eval(chain, T[:m]), budget_s)
    got = out_dev[:, :m].cpu().numpy().astype(np.float64)
    ext = float((chain.max(axis=0) - chain.min(axis=0)).max())
    err = float(np.abs(got - ref).max() / ext)
    # one thread beside the OpenMP figure: median of 3 runs over the first 2^20 queries
    m1 = min(m, 1 << 20)
    prev = oracle.set_threads(1)
    try:
        secs = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.chain_eval(chain, T[:m1])
            secs.append(time.perf_counter() - t0)
    finally:
        oracle.set_threads(prev)
    single = {"value": m1 / sorted(secs)[1] / 1e9, "unit": "G evals/s", "cores": 1,
              "sample": "median of 3 x %d random T" % m1}
    return {"value": m / sec / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d x %d random T of the same 2^20-segment chain (FP64 chain definition, OpenMP)"
                      % (reps, m), "host": host_cpu(), "single_thread": single}, err


def host_cpu():
    """The host's CPU model name, as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------- suite
def suite_plain(torch, bz, bz_synth, cpu):
    log("suite: plain curves")
    ctrl, t = bz_synth.plain_curves()
    res = {}
    c_d, t_d = torch.from_numpy(ctrl).cuda(), torch.from_numpy(t).cuda()
    out = torch.empty((3, ctrl.shape[0] * t.shape[0]), device="cuda")
    ref = None
    if cpu:
        import oracle
        ref, sec, _ = oracle_timed(lambda: oracle.bezier_decasteljau(ctrl, t), 2.0)
        res["cpu_baseline"] = {"value": out.shape[1] / sec / 1e9, "unit": "G evals/s",
                               "cores": oracle.max_threads(), "kind": "oracle", "sample": "all 4096 x 256 points"}
    nbytes = out.numel() * 4 + ctrl.nbytes + t.nbytes
    for m in ("decasteljau", "bernstein", "seiler"):
        # a ~5 us kernel: eager launches from Python are launch-bound, so the
        # figure of merit is the graph-replayed launch (eager time kept beside it)
        eager = timed(lambda: bz.eval_bezier(c_d, t_d, m, out=out), torch, iters=50)
        ms = graph_time_ms(lambda: bz.eval_bezier(c_d, t_d, m, out=out), torch)
        e = {"kernel_ms": ms, "timing": "HIP graph of 50 launches", "eager_launch_ms": eager,
             "value": out.shape[1] / (ms * 1e-3) / 1e9, "roofline": hbm_roof(nbytes, ms)}
        if ref is not None:
            e["max_err_bbox"] = max_err_bbox(out.cpu().numpy(), ref, extents(ctrl), 256)
        res[m] = e
    # x16 curves: past the launch-bound regime
    c16 = torch.from_numpy(bz_synth.plain_curves(n_curves=1 << 16)[0]).cuda()
    o16 = torch.empty((3, (1 << 16) * 256), device="cuda")
    n16 = o16.numel() * 4 + c16.numel() * 4 + t.nbytes
    for m in ("decasteljau", "bernstein", "seiler"):
        ms = timed(lambda: bz.eval_bezier(c16, t_d, m, out=o16), torch)
        res[m + "_x16"] = {"kernel_ms": ms, "value": o16.shape[1] / (ms * 1e-3) / 1e9, "roofline": hbm_roof(n16, ms)}
    # x64 curves: 805 MB of points, more than the 256 MB Infinity Cache can hold
    # (the x16 outputs, 201 MB, may stay in it between launches)
    c64 = torch.from_numpy(bz_synth.plain_curves(n_curves=1 << 18)[0]).cuda()
    o64 = torch.empty((3, (1 << 18) * 256), device="cuda")
    n64 = o64.numel() * 4 + c64.numel() * 4 + t.nbytes
    for m in ("decasteljau", "bernstein", "seiler"):
        ms = timed(lambda: bz.eval_bezier(c64, t_d, m, out=o64), torch)
        res[m + "_x64"] = {"kernel_ms": ms, "value": o64.shape[1] / (ms * 1e-3) / 1e9, "roofline": hbm_roof(n64, ms)}
    del c64, o64
    # random t per curve (t[n][256] ~ U[0,1), seed 1001): 4 bytes in and 12 out per point
    c16h, tr = bz_synth.random_curves(1 << 16, 3, 3, 256, seed=1001 + 16)
    c16r, tr_d = torch.from_numpy(c16h).cuda(), torch.from_numpy(tr).cuda()
    nr = o16.numel() * 4 + c16r.numel() * 4 + tr.nbytes
    for m in ("decasteljau", "bernstein", "seiler"):
        ms = timed(lambda: bz.eval_bezier(c16r, tr_d, m, out=o16), torch)
        e = {"kernel_ms": ms, "value": o16.shape[1] / (ms * 1e-3) / 1e9, "roofline": hbm_roof(nr, ms)}
        if cpu and m == "decasteljau":
            import oracle
            k = 1024
            ref = oracle.bezier_decasteljau(c16h[:k], tr[:k], per_object=True)
            e["max_err_bbox"] = max_err_bbox(o16[:, :k * 256].cpu().numpy(), ref, extents(c16h[:k]), 256)
        res[m + "_x16_random_t"] = e
    return {"workload": "4096 cubic 3D Bezier curves x 256 shared t (1M points), FP32; *_x16: 65536 curves; "
                        "*_x64: 262144 curves; *_x16_random_t: 65536 curves x 256 random t each",
            "unit": "G evals/s", **res}


def batch_bytes(b, es):
    """Algorithmic bytes of one batched launch, as the caller's problem states
    them: every control point (dim values) and the weight of every rational or
    NURBS control point in the storage type (es bytes), every knot (FP32),
    8 bytes of offsets per object and 8 more per NURBS (its knot offset), and
    per query the parameter in (two for a surface patch) and the point out
    (FP32).  The plan's own
    derived data (class-sorted copies, extracted NURBS segments, tables) is
    not counted: it is the implementation's choice, not the problem's."""
    kind = b.kind_degree >> 8
    ncp = np.diff(b.cp_offset)
    nk = np.diff(b.knot_offset)
    rd = int(ncp.sum()) * b.dim * es + int(ncp[kind != 0].sum()) * es + int(nk.sum()) * 4
    rd += b.n_obj * 8 + int((kind == 2).sum()) * 8
    rd += int((kind == 3).sum()) * b.n_t * 4  # a surface patch's second parameter v
    return rd + b.n_obj * b.n_t * (4 + 4 * b.dim)


def suite_batched(torch, bz, bz_synth, cpu):
    log("suite: batched (generating 2^20 + 2^16 objects)")
    b = bz_synth.mixed_batch()
    n_q = b.n_obj * b.n_t
    kd = torch.from_numpy(b.kind_degree.astype(np.int16)).cuda()
    cpo = torch.from_numpy(b.cp_offset).cuda()
    ko = torch.from_numpy(b.knot_offset).cuda()
    kn = torch.from_numpy(b.knots).cuda()
    t = torch.from_numpy(b.t).cuda()
    out = torch.empty((3, n_q), device="cuda")
    res = {}
    sub_n = 16384
    ref = sub = ext = None
    if cpu:
        import oracle
        cp, kk = b.cp_offset[:sub_n + 1], b.knot_offset[:sub_n + 1]
        sub = bz_synth.Batch(dim=3, n_t=16, kind_degree=b.kind_degree[:sub_n], cp_offset=cp, ctrl=b.ctrl[:cp[-1] * 3],
                             w=b.w[:cp[-1]], knot_offset=kk, knots=b.knots[:kk[-1]], t=b.t[:sub_n])
        ref, sec, _ = oracle_timed(lambda: oracle.batch_eval(sub), 5.0)
        res["cpu_baseline"] = {"value": sub_n * 16 / sec / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "first %d objects x 16 t (de Casteljau / de Boor)" % sub_n}
        ext = np.empty(sub_n)
        for o in range(sub_n):
            P = sub.ctrl[cp[o] * 3:cp[o + 1] * 3].reshape(3, -1).astype(np.float64)
            ext[o] = max((P.max(1) - P.min(1)).max(), np.abs(P).max())
    for dt, name in ((torch.float32, "fp32"), (torch.float16, "fp16")):
        ctrl = torch.from_numpy(b.ctrl).cuda().to(dt)
        w = torch.from_numpy(b.w).cuda().to(dt)
        plan = bz.BatchPlan(kd, cpo, ctrl, w, 3, ko, kn, 16, "bernstein")
        tune = plan.autotune(t, out)
        ms = timed(lambda: plan(t, out=out), torch)
        info = plan.info()
        nbytes = batch_bytes(b, 4 if dt == torch.float32 else 2)
        e = {"kernel_ms": ms, "value": n_q / (ms * 1e-3) / 1e9, "roofline": hbm_roof(nbytes, ms),
             "algorithmic_bytes": nbytes, "autotune": tune, "plan": info}
        if ref is not None:
            got = out[:, :sub_n * 16].cpu().numpy()
            if name == "fp32":
                e["max_err_bbox"] = max_err_bbox(got, ref, ext, 16)
            else:
                import oracle
                rsub = bz_synth.Batch(**{**sub.__dict__})
                rsub.ctrl = ctrl[:len(sub.ctrl)].float().cpu().numpy()
                rsub.w = w[:len(sub.w)].float().cpu().numpy()
                e["max_err_bbox_vs_rounded_inputs"] = max_err_bbox(got, oracle.batch_eval(rsub), ext, 16)
                e["max_err_bbox_vs_fp32_inputs"] = max_err_bbox(got, ref, ext, 16)
        plan.close()
        res[name] = e
    return {"workload": "2^20 Bezier curves (degree U{2..15}, half rational) + 2^16 cubic NURBS (8-64 knots), "
                        "16 random t each, one persistent launch, Bernstein form", "unit": "G evals/s", **res}


def suite_patches(torch, bz, bz_synth, cpu):
    log("suite: patches")
    n = 1 << 18
    P = bz_synth.patches(n_obj=n)
    Pd = torch.from_numpy(P).cuda()
    out = torch.empty((3, n * 1024), device="cuda")
    nbytes = out.numel() * 4 + P.nbytes
    res = {}
    pick = np.arange(0, n, n // 1024)
    ref = None
    if cpu:
        import oracle
        ref, sec, _ = oracle_timed(lambda: oracle.tensor_grid(P[pick], 3, 3, 32, 32), 3.0)
        res["cpu_baseline"] = {"value": len(pick) * 1024 / sec / 1e9, "unit": "G points/s",
                               "cores": oracle.max_threads(), "kind": "oracle", "sample": "1024 patches x 32x32"}
    for eng in ("valu", "mfma_f32", "mfma_bf16", "mfma_f16", "mfma_f16x3"):
        ms = timed(lambda: bz.eval_tensor_patch(Pd, 3, 3, nu=32, nv=32, engine=eng, out=out), torch, iters=10)
        e = {"kernel_ms": ms, "value": n * 1024 / (ms * 1e-3) / 1e9, "roofline": hbm_roof(nbytes, ms)}
        if ref is not None:
            got = out.view(3, n, 1024)[:, torch.from_numpy(pick).cuda()].cpu().numpy().reshape(3, -1)
            e["max_err_bbox"] = max_err_bbox(got, ref, extents(P[pick]), 1024)
        res[eng] = e
    del out
    return {"workload": "2^18 bicubic 3D patches tessellated on a 32x32 grid (2^28 points)", "unit": "G points/s",
            **res}


def suite_volumes(torch, bz, bz_synth, cpu):
    log("suite: volumes")
    ctrl, uvw = bz_synth.volumes()
    n, per = ctrl.shape[0], uvw.shape[1]
    c_d, u_d = torch.from_numpy(ctrl).cuda(), torch.from_numpy(uvw).cuda()
    out = torch.empty((3, n * per), device="cuda")
    ms = timed(lambda: bz.eval_tensor_patch(c_d, 3, 3, 3, uvw=u_d, out=out), torch)
    nbytes = ctrl.nbytes + uvw.nbytes + out.numel() * 4
    # per query: three cubic bases (~15 ops each) and, per coordinate, 64 + 16 + 4 multiply-adds
    flop = n * per * (3 * 15 + 3 * 84 * 2)
    tf = flop / (ms * 1e-3) / 1e12
    res = {"kernel_ms": ms, "value": n * per / (ms * 1e-3) / 1e9, "hbm": hbm_roof(nbytes, ms),
           "roofline": alu_roof(tf)}
    # the same volumes in per-axis Seiler form (terms converted once)
    sc = bz.tensor_to_seiler(c_d, 3, 3, 3)
    torch.cuda.synchronize()
    conv_ms = event_time_ms(lambda: bz.tensor_to_seiler(c_d, 3, 3, 3, out=sc), 3, torch)
    out_s = torch.empty_like(out)
    ms_s = timed(lambda: bz.eval_tensor_seiler(sc, 3, 3, 3, uvw=u_d, out=out_s), torch)
    tf_s = flop / (ms_s * 1e-3) / 1e12
    res["seiler"] = {"kernel_ms": ms_s, "value": n * per / (ms_s * 1e-3) / 1e9, "convert_ms": conv_ms,
                     "roofline": alu_roof(tf_s)}
    if cpu:
        import oracle
        k = 512
        ref, sec, _ = oracle_timed(lambda: oracle.tensor_points(ctrl[:k], 3, 3, 3, uvw[:k]), 3.0)
        gs = out_s.view(3, n, per)[:, :k].cpu().numpy().reshape(3, -1)
        res["seiler"]["max_err_bbox"] = max_err_bbox(gs, ref, extents(ctrl[:k]), per)
        res["cpu_baseline"] = {"value": k * per / sec / 1e9, "unit": "G points/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "first 512 volumes x 256 points"}
        got = out.view(3, n, per)[:, :k].cpu().numpy().reshape(3, -1)
        res["max_err_bbox"] = max_err_bbox(got, ref, extents(ctrl[:k]), per)
    return {"workload": "2^16 tricubic 3D volumes at 2^24 random (u,v,w); Bernstein and per-axis Seiler forms",
            "unit": "G points/s", **res}


def suite_cubic_chain(torch, bz, bz_synth, cpu):
    log("suite: cubic chain (generating 2^20 segments)")
    chain, T = bz_synth.cubic_chain_walk()
    n_seg, n_q, dim = (chain.shape[0] - 1) // 3, T.shape[0], chain.shape[1]
    c_d, T_d = torch.from_numpy(chain).cuda(), torch.from_numpy(T).cuda()
    grid = bz.encode_piecewise_cubic(c_d)
    torch.cuda.synchronize()
    enc_ms = event_time_ms(lambda: bz.encode_piecewise_cubic(c_d, out=grid), 5, torch)
    tiles = bz.tile_piecewise_cubic(grid)
    out = torch.empty((dim, n_q), device="cuda")
    nbytes = grid.numel() * 4 + n_q * 4 + n_q * dim * 4
    ms_grid = timed(lambda: bz.eval_piecewise_cubic(grid, T_d, out=out), torch)
    ms = timed(lambda: bz.eval_piecewise_cubic_tiled(tiles, n_seg, dim, T_d, out=out), torch)
    res = {"kernel_ms": ms, "value": n_q / (ms * 1e-3) / 1e9, "roofline": hbm_roof(nbytes, ms), "layout": "tiled",
           "algorithmic_bytes": nbytes, "encode_ms": enc_ms,
           "grid_layout": {"kernel_ms": ms_grid, "value": n_q / (ms_grid * 1e-3) / 1e9,
                           "roofline": hbm_roof(nbytes, ms_grid)},
           # a query's 72-byte window lies in one line; the probe reads 64 of them
           "gather_ceiling": gather_ceiling(torch, bz, tiles, n_q, ms, vec16=4)}
    if cpu:
        import oracle
        m = 1 << 22
        ref, sec, reps = oracle_timed(lambda: oracle.cubic_chain_eval(chain, T[:m]), 5.0)
        res["cpu_baseline"] = {"value": m / sec / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "%d x %d random T (FP64 chain definition)" % (reps, m)}
        ext = float((chain.max(axis=0) - chain.min(axis=0)).max())
        res["max_err_bbox"] = float(np.abs(out[:, :m].cpu().numpy().astype(np.float64) - ref).max() / ext)
    return {"workload": "C0 piecewise cubic chain as two stacked zig-zag layers (cache-line tiles; the two-layer "
                        "grid as comparison), 2^20 segments, 2^24 uniform random global T, 3D, FP32",
            "unit": "G evals/s", **res}


def suite_texemu(torch, bz, bz_synth, cpu):
    """Texture-filter emulation: Fig. 3's three read modes of a cubic and the
    zig-zag chain through the emulated bilinear filter, 8-bit weights.  The
    quantisation errors come from the CPU-baseline leg (the oracle's exact
    curves and emulated filter on a sample)."""
    log("suite: texture-filter emulation")
    ctrl, t = bz_synth.plain_curves(n_curves=1 << 16)
    n, nt = ctrl.shape[0], t.shape[0]
    c_d, t_d = torch.from_numpy(ctrl).cuda(), torch.from_numpy(t).cuda()
    out = torch.empty((3, n * nt), device="cuda")
    sub = 1024  # error sample: the first 1024 curves, every t
    res = {}
    exact = ext = None
    if cpu:
        import oracle
        exact = oracle.bezier_decasteljau(ctrl[:sub], t)
        ext = extents(ctrl[:sub])
    for mode in ("decasteljau", "hybrid", "seiler"):
        tex = bz.build_texture(c_d, mode)
        torch.cuda.synchronize()
        build_ms = event_time_ms(lambda: bz.build_texture(c_d, mode, out=tex), 5, torch)
        e = {"texels_per_coord": tex.shape[2], "build_ms": build_ms}
        for rounding in ("nearest", "truncate"):
            ms = timed(lambda: bz.eval_texture(tex, 3, mode, t_d, 8, rounding, out=out), torch)
            nbytes = tex.numel() * 4 + t.nbytes + out.numel() * 4
            r = {"kernel_ms": ms, "value": n * nt / (ms * 1e-3) / 1e9, "roofline": hbm_roof(nbytes, ms)}
            if cpu:
                got = out[:, :sub * nt].cpu().numpy()
                ref = oracle.tex_eval(tex[:sub].cpu().numpy(), 3, mode, t, False, 8, rounding)
                r["quantisation_err_bbox"] = max_err_bbox(got, exact, ext, nt)
                r["max_err_bbox_vs_oracle_emulation"] = max_err_bbox(got, ref, ext, nt)
            e[rounding] = r
        res[mode] = e
    # degree 7 in one 2x2x2 Seiler texture read at (t, st, (st)^2)
    c7, _ = bz_synth.random_curves(1 << 14, 7, 3, nt, seed=1001 + 700, per_object=False)
    c7_d = torch.from_numpy(c7).cuda()
    tex7 = bz.build_texture(c7_d, "seiler")
    o7 = torch.empty((3, c7.shape[0] * nt), device="cuda")
    ms = timed(lambda: bz.eval_texture(tex7, 7, "seiler", t_d, 8, "nearest", out=o7), torch)
    r = {"kernel_ms": ms, "value": c7.shape[0] * nt / (ms * 1e-3) / 1e9,
         "roofline": hbm_roof(tex7.numel() * 4 + t.nbytes + o7.numel() * 4, ms)}
    if cpu:
        got = o7[:, :sub * nt].cpu().numpy()
        e7 = extents(c7[:sub])
        r["quantisation_err_bbox"] = max_err_bbox(got, oracle.bezier_decasteljau(c7[:sub], t), e7, nt)
        ref = oracle.tex_eval(tex7[:sub].cpu().numpy(), 7, "seiler", t, False, 8, "nearest")
        r["max_err_bbox_vs_oracle_emulation"] = max_err_bbox(got, ref, e7, nt)
    res["seiler_degree7"] = r
    # bicubic patches through the emulated filter: 2^16 patches x 256 random (u, v)
    P = bz_synth.patches(n_obj=1 << 16)
    uvp = np.random.default_rng(1004 + 1).random((1 << 16, 256, 2)).astype(np.float32)
    P_d, uv_d = torch.from_numpy(P).cuda(), torch.from_numpy(uvp).cuda()
    op = torch.empty((3, (1 << 16) * 256), device="cuda")
    kp = 512
    exact_p = oracle.tensor_points(P[:kp], 3, 3, 0, uvp[:kp]) if cpu else None
    for mode in ("decasteljau", "seiler"):
        texp = bz.build_texture_patch(P_d, 3, 3, mode)
        ms = timed(lambda: bz.eval_texture_patch(texp, 3, 3, mode, uv_d, 8, "nearest", out=op), torch)
        r = {"kernel_ms": ms, "value": op.shape[1] / (ms * 1e-3) / 1e9,
             "roofline": hbm_roof(texp.numel() * 4 + uvp.nbytes + op.numel() * 4, ms)}
        if cpu:
            got = op[:, :kp * 256].cpu().numpy()
            ref = oracle.tex_patch_eval(texp[:kp].cpu().numpy(), 3, 3, mode, uvp[:kp])
            r["quantisation_err_bbox"] = max_err_bbox(got, exact_p, extents(P[:kp]), 256)
            r["max_err_bbox_vs_oracle_emulation"] = max_err_bbox(got, ref, extents(P[:kp]), 256)
        res["patch_" + mode] = r
    del op
    del out
    chain, T = bz_synth.chain_walk()
    nseg, nq = (chain.shape[0] - 1) // 2, T.shape[0]
    grid = bz.encode_piecewise(torch.from_numpy(chain).cuda())
    T_d = torch.from_numpy(T).cuda()
    out = torch.empty((3, nq), device="cuda")
    m = 1 << 22
    cext = float((chain.max(axis=0) - chain.min(axis=0)).max())
    chain_exact = oracle.chain_eval(chain, T[:m]) if cpu else None
    tiles = bz.tile_piecewise(grid)
    ch = {"layout": "tiled"}
    for rounding in ("nearest", "truncate"):
        ms = timed(lambda: bz.eval_piecewise_texemu_tiled(tiles, nseg, 3, T_d, 8, rounding, out=out), torch)
        r = {"kernel_ms": ms, "value": nq / (ms * 1e-3) / 1e9, "roofline": hbm_roof(chain_bytes(nseg, 3, nq), ms)}
        if rounding == "nearest":
            ms_g = timed(lambda: bz.eval_piecewise_texemu(grid, T_d, 8, rounding, out=out), torch)
            r["grid_layout"] = {"kernel_ms": ms_g, "value": nq / (ms_g * 1e-3) / 1e9,
                                "roofline": hbm_roof(chain_bytes(nseg, 3, nq), ms_g)}
            r["gather_ceiling"] = gather_ceiling(torch, bz, tiles, nq, ms)
            bz.eval_piecewise_texemu_tiled(tiles, nseg, 3, T_d, 8, rounding, out=out)  # out: the tiled result again
        if cpu:
            got = out[:, :m].cpu().numpy().astype(np.float64)
            ref = oracle.chain_texemu_eval(grid.cpu().numpy(), T[:m], 8, rounding)
            r["quantisation_err_bbox"] = float(np.abs(got - chain_exact).max() / cext)
            r["max_err_bbox_vs_oracle_emulation"] = float(np.abs(got - ref).max() / cext)
        ch[rounding] = r
    res["chain"] = ch
    if cpu:
        tex = oracle.tex_build(ctrl[:sub], "decasteljau").astype(np.float32)
        _, sec, _ = oracle_timed(lambda: oracle.tex_eval(tex, 3, "decasteljau", t), 2.0)
        res["cpu_baseline"] = {"value": sub * nt / sec / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "1024 curves x 256 t, trilinear mode"}
    return {"workload": "texture-filter emulation, 8 fractional weight bits: 65536 cubic 3D curves x 256 shared t "
                        "in the trilinear / hybrid / Seiler modes (quantisation error on the first 1024 curves), 16384 "
                        "degree-7 curves in one 2x2x2 Seiler texture, 2^16 bicubic patches at 256 random (u, v) "
                        "(de Casteljau isoline reads / Seiler surface reads), "
                        "and the 2^20-segment chain at 2^24 random T", "unit": "G evals/s", **res}


def suite_particles(torch, bz, bz_synth, cpu):
    """Sec. 5's particle test on MI355X: particles on a ring of 16 chained
    cubics, one frame = phase update + position + a K-step consumer, for
    1M / 5M / 10M particles and K = 0 / 64 / 256, each position method."""
    log("suite: particle ring")
    methods = ("polynomial", "seiler", "seiler_texture", "table")
    res = {}
    for n in (1_000_000, 5_000_000, 10_000_000):
        seg, T, speed = bz_synth.particle_ring(n_particles=n)
        seg_d, s_d = torch.from_numpy(seg).cuda(), torch.from_numpy(speed).cuda()
        T_d = torch.from_numpy(T).cuda()
        pos = torch.empty((3, n), device="cuda")
        shade = torch.empty(n, device="cuda")
        rings = {m: bz.particle_ring_data(seg_d, m, 64) for m in methods}
        for K in (0, 64, 256):
            row = {}
            for m in methods:
                # frames replayed from a HIP graph: the 1M-particle frames last ~5 us
                ms = graph_time_ms(lambda: bz.particles_step(m, rings[m], 16, T_d, s_d, 1 / 60, K, 64, pos, shade),
                                   torch)
                row[m] = {"ms_per_frame": ms, "G particles/s": n / (ms * 1e-3) / 1e9}
            row["hbm_frac_polynomial"] = (particle_frame_bytes(n) / (row["polynomial"]["ms_per_frame"] * 1e-3) / 1e9
                                          / HBM_PEAK_GBS)
            # consumer: K FMAs = 2K flop per particle
            row["consumer_alu_frac_polynomial"] = (2 * K * n / (row["polynomial"]["ms_per_frame"] * 1e-3) / 1e12
                                                   / FP32_VALU_PEAK_TFLOPS)
            res["%dM_K%d" % (n // 1_000_000, K)] = row
    if cpu:
        import oracle
        seg, T, speed = bz_synth.particle_ring(n_particles=1 << 20)
        _, sec, _ = oracle_timed(lambda: oracle.particles_step(seg, T, speed, 1 / 60, "polynomial", 64), 3.0)
        res["cpu_baseline"] = {"value": (1 << 20) / sec / 1e9, "unit": "G particles/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "2^20 particles, one frame, polynomial, K = 64"}
    return {"timing": "HIP graph of 50 frames, replayed",
            "workload": "particle ring (16 chained cubic segments), one frame per launch: phase update, position "
                        "by polynomial / Seiler terms / 8-bit Seiler texture emulation / 64-sample table, K-step "
                        "consumer", "unit": "G particles/s", **res}


def suite_fit(torch, bz, bz_synth, cpu):
    log("suite: fit")
    gt_ctrl, tau, eps = bz_synth.fit_problem()
    n, nt = tau.shape
    res = {}
    # targets y = G(tau) + noise, evaluated by the curve kernel
    y = bz.eval_bezier(torch.from_numpy(gt_ctrl).cuda(), torch.from_numpy(tau).cuda())
    y += torch.from_numpy(eps).cuda()
    y3 = y.view(3, n, nt)
    frac = torch.arange(4, device="cuda", dtype=torch.float32) / 3.0
    ctrl = (y3[:, :, 0].T[:, :, None] * (1 - frac) + y3[:, :, -1].T[:, :, None] * frac).contiguous()
    t = torch.arange(nt, device="cuda", dtype=torch.float32).div(nt - 1).repeat(n, 1).contiguous()
    mc, vc, mt, vt = (torch.zeros_like(ctrl), torch.zeros_like(ctrl), torch.zeros_like(t), torch.zeros_like(t))
    loss = torch.zeros(n, device="cuda")
    bz.fit_adam_step(ctrl, t, y, mc, vc, mt, vt, 1, loss_part=loss)
    loss0 = float(loss.sum())
    s = torch.cuda.current_stream()
    a, bb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    bz.fit_adam_run(ctrl, t, y, mc, vc, mt, vt, 2, 199, loss_part=loss)
    bb.record(s)
    bb.synchronize()
    ms_199 = a.elapsed_time(bb)
    ms_step = ms_199 / 199
    # Per sample and step (counted from the kernel): cubic and quadratic
    # Bernstein bases ~14 flop; per coordinate value 7, hodograph 10, residual,
    # loss, gradient scale and dL/dt 7, dL/dP 8 -> 32; Adam on t and clamp ~16.
    flop = n * nt * (14 + 3 * 32 + 16)
    tf = flop / (ms_step * 1e-3) / 1e12
    run_bytes = n * nt * (4 * 2 + 12 + 16) + n * 12 * 4 * 6 + n * 4  # state read and written once per run
    res.update({"ms_per_step": ms_step, "run_ms_199_steps": ms_199,
                "value": n * nt / (ms_step * 1e-3) / 1e9,
                "roofline": alu_roof(tf),
                "hbm": hbm_roof(run_bytes, ms_199),
                "loss_step1": loss0, "loss_step200": float(loss.sum())})
    if cpu:
        import oracle
        yh = y.cpu().numpy().astype(np.float64)
        c0 = np.zeros((n, 3, 4))
        t0 = np.tile(np.arange(nt) / (nt - 1), (n, 1))
        _, sec, _ = oracle_timed(lambda: oracle.fit_loss_grad(c0, t0, yh), 1.0, 1)
        res["cpu_baseline"] = {"value": n * nt / sec / 1e9, "unit": "G sample-steps/s", "cores": oracle.max_threads(),
                               "kind": "oracle", "sample": "one full loss+gradient evaluation (65536 x 128), "
                                                           "i.e. one of the 200 steps; the 200-step run "
                                                           "extrapolates to 200 times its time",
                               "run_200_steps_s": 200 * sec}
    return {"workload": "fit 65536 cubic 3D curves to 128 noisy samples each: fused L2 loss + adjoint + Adam, "
                        "200 steps in one register-resident launch", "unit": "G sample-steps/s", **res}


FORMS = ("decasteljau", "bernstein", "seiler")
PLAIN_COUNTERS = "plain_curves_counters.json"
# The final stdout line is kept below this size (the full suite goes to a file).
RECORD_MAX_BYTES = 2048


def plain_bytes(n_curves, degree, dim, n_t):
    """Algorithmic bytes of one plain-curve launch with shared t: the points
    out, the control points and the parameter vector once."""
    return n_curves * n_t * dim * 4 + n_curves * dim * (degree + 1) * 4 + n_t * 4


def headline_plain(torch, bz, bz_synth, steps, warmup, cpu, n_curves=4096, n_t=256):
    """The plain FP32 workload: n_curves cubic 3D curves x n_t shared t by the
    three forms.  One step = the three launches (3 x n_curves*n_t points).
    The warm-up steps replay a HIP graph of one step; the `steps` timed steps
    are captured in one HIP graph and replayed once, since a graph replay
    issued from Python costs more host time (about 17 us) than a step takes
    on the GPU (about 12 us).  One replay per step is timed afterwards for
    context.  Returns the headline fields."""
    log("headline: plain cubic curves, %d x %d t, three forms" % (n_curves, n_t))
    ctrl, t = bz_synth.plain_curves(n_curves=n_curves, n_t=n_t)
    c_d, t_d = torch.from_numpy(ctrl).cuda(), torch.from_numpy(t).cuda()
    n_q = n_curves * n_t
    outs = {m: torch.empty((3, n_q), device="cuda") for m in FORMS}

    def step_eager():
        for m in FORMS:
            bz.eval_bezier(c_d, t_d, m, out=outs[m])

    for _ in range(3):
        step_eager()
    torch.cuda.synchronize()
    # eager steps (one Python call and one launch per form) for context
    eager_ms = event_time_ms(step_eager, max(steps, 20), torch)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step_eager()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    g_all = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_all):
        for _ in range(steps):
            step_eager()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ea.record(s)
    g_all.replay()
    eb.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / steps
    gpu_ms_per_step = ea.elapsed_time(eb) / steps
    del g_all
    # context: one replay of the one-step graph per step (host-bound)
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    replay_ms = (time.perf_counter() - t0) * 1e3 / steps
    del g
    # each form's kernel on its own: a HIP graph of 50 launches replayed 10
    # times between HIP events on the launch stream (the kernels last a few
    # us), the median of five such timings
    nbytes = plain_bytes(n_curves, 3, 3, n_t)
    forms = {}
    for m in FORMS:
        ms = graph_time_ms(lambda: bz.eval_bezier(c_d, t_d, m, out=outs[m]), torch, launches=50, replays=10, trials=5)
        forms[m] = {"us": ms * 1e3, "G/s": n_q / (ms * 1e-3) / 1e9, "frac": hbm_roof(nbytes, ms)["frac"]}
    dom = max(FORMS, key=lambda m: forms[m]["us"])
    roof = hbm_roof(nbytes, forms[dom]["us"] * 1e-3)
    roof["kernel"] = "k_curves<%s>" % dom
    roof["bytes_per_launch"] = nbytes
    roof["traffic"] = recorded_traffic(PLAIN_COUNTERS, {"n_curves": n_curves, "n_t": n_t}, dom)
    # what a launch of this size costs at best: a write-only kernel storing the
    # same output bytes (one 16-byte vector per thread), timed the same way
    wbuf = torch.empty(3 * n_q, device="cuda")
    floor_ms = graph_time_ms(lambda: bz.hbm_probe("write", wbuf, wbuf, blocks_per_cu=0), torch, launches=50, replays=10,
                             trials=5)
    del wbuf
    floor = {"us": floor_ms * 1e3, "bytes": 12 * n_q, "of_dominant": floor_ms * 1e3 / forms[dom]["us"]}
    rec = {"value": 3 * n_q / (ms_per_step * 1e-3) / 1e9, "ms_per_step": ms_per_step,
           "gpu_ms_per_step": gpu_ms_per_step, "replay_ms_per_step": replay_ms, "eager_ms_per_step": eager_ms,
           "forms": forms, "roofline": roof,
           "launch_floor": floor}
    # 16x the curves with random t per curve (65536 x 256 = 2^24 points per
    # form, 4 bytes in and 12 out per point): past the launch-bound regime
    c16h, t16h = bz_synth.random_curves(16 * n_curves, 3, 3, n_t, seed=1001 + 16)
    c16, t16 = torch.from_numpy(c16h).cuda(), torch.from_numpy(t16h).cuda()
    o16 = torch.empty((3, 16 * n_q), device="cuda")
    n16 = o16.numel() * 4 + c16.numel() * 4 + t16.numel() * 4
    gs, fr = [], []
    for m in FORMS:
        ms = timed(lambda: bz.eval_bezier(c16, t16, m, out=o16), torch, iters=20)
        gs.append(16 * n_q / (ms * 1e-3) / 1e9)
        fr.append(hbm_roof(n16, ms)["frac"])
    rec["x16_random_t"] = {"G/s": gs, "frac": fr}  # in the order of FORMS
    del c16, t16, o16
    if cpu:
        import oracle
        log("headline: CPU baseline (oracle, three forms)")
        ref = oracle.bezier_decasteljau(ctrl, t)
        ext = extents(ctrl)
        rec["max_err_bbox"] = {m: max_err_bbox(outs[m].cpu().numpy(), ref, ext, n_t) for m in FORMS}

        def oracle_step():
            oracle.bezier_decasteljau(ctrl, t)
            oracle.bezier_bernstein(ctrl, t)
            oracle.seiler_eval(oracle.seiler_from_bezier(ctrl), t)

        _, sec, reps = oracle_timed(oracle_step, budget_s=10.0, max_reps=200)
        rec["cpu_baseline"] = {"value": 3 * n_q / sec / 1e9, "unit": "G evals/s", "cores": oracle.max_threads(),
                               "kind": "oracle",
                               "sample": "3 forms x %d x %d points, FP64, %d reps"
                                         % (n_curves, n_t, reps), "host": host_cpu()}
    return rec


def batched_record(torch, bz, bz_synth, cpu, n_sample=16384):
    """The mixed batch in one persistent launch, FP32 and FP16 storage.  Max
    errors on a seeded random sample of objects spread over the whole batch
    (with the first and last objects included); FP16 is measured against the
    oracle on the FP32 inputs (its rounding included) and on the rounded
    inputs."""
    log("batched: generating 2^20 Bezier + 2^16 NURBS objects")
    b = bz_synth.mixed_batch()
    n_q = b.n_obj * b.n_t
    kd = torch.from_numpy(b.kind_degree.astype(np.int16)).cuda()
    cpo = torch.from_numpy(b.cp_offset).cuda()
    ko = torch.from_numpy(b.knot_offset).cuda()
    kn = torch.from_numpy(b.knots).cuda()
    t = torch.from_numpy(b.t).cuda()
    out = torch.empty((3, n_q), device="cuda")
    idx = np.unique(np.concatenate([np.random.default_rng(7).choice(b.n_obj, n_sample - 2, replace=False),
                                    [0, b.n_obj - 1]]))
    sub = b.subset(idx)
    idx_d = torch.from_numpy(idx).cuda()
    ref = ext = None
    res = {}
    if cpu:
        import oracle
        ref, sec, reps = oracle_timed(lambda: oracle.batch_eval(sub), 5.0)
        res["cpu_baseline"] = {"value": len(idx) * b.n_t / sec / 1e9, "unit": "G evals/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": "%d random objects x 16 t, FP64" % len(idx)}
        ext = np.empty(len(idx))
        for i in range(len(idx)):
            ext[i] = _box(sub.ctrl[sub.cp_offset[i] * 3:sub.cp_offset[i + 1] * 3].astype(np.float64).reshape(3, -1))
    for dt, name in ((torch.float32, "fp32"), (torch.float16, "fp16")):
        log("batched: %s plan + autotune" % name)
        ctrl = torch.from_numpy(b.ctrl).cuda().to(dt)
        w = torch.from_numpy(b.w).cuda().to(dt)
        plan = bz.BatchPlan(kd, cpo, ctrl, w, 3, ko, kn, b.n_t, "bernstein")
        tune = plan.autotune(t, out)
        ms = timed(lambda: plan(t, out=out), torch, iters=20)
        nbytes = batch_bytes(b, 4 if dt == torch.float32 else 2)
        e = {"us": ms * 1e3, "G/s": n_q / (ms * 1e-3) / 1e9, "frac": hbm_roof(nbytes, ms)["frac"],
             "bytes": nbytes, "config": [tune["workgroups"], tune["tile_multiple"], tune["schedule"],
                                         tune["queries_per_lane"], tune["window"]]}
        if ref is not None:
            got = out.view(3, b.n_obj, b.n_t)[:, idx_d].reshape(3, -1).cpu().numpy()
            e["max_err_bbox"] = max_err_bbox(got, ref, ext, b.n_t)
            if name == "fp16":
                import oracle
                rsub = dataclasses.replace(sub)
                rsub.ctrl = torch.from_numpy(sub.ctrl).to(dt).float().numpy()
                rsub.w = torch.from_numpy(sub.w).to(dt).float().numpy()
                e["max_err_bbox_vs_rounded"] = max_err_bbox(got, oracle.batch_eval(rsub), ext, b.n_t)
        plan.close()
        del ctrl, w
        res[name] = e
    res["fp16_speedup"] = res["fp32"]["us"] / res["fp16"]["us"]
    del t, out, kd, cpo, ko, kn
    torch.cuda.empty_cache()
    res["fp32_with_patches"] = batched_patches_record(torch, bz, bz_synth, cpu)
    return res


def batched_patches_record(torch, bz, bz_synth, cpu, n_sample=8192):
    """The same mixed batch plus 2^16 bicubic surface patches at 16 random
    (u, v) each, FP32, in the one persistent launch (u from t, v from a second
    parameter array)."""
    log("batched: with 2^16 bicubic patches")
    b = bz_synth.mixed_batch(n_patches=1 << 16)
    n_q = b.n_obj * b.n_t
    ctrl = torch.from_numpy(b.ctrl).cuda()
    plan = bz.BatchPlan(torch.from_numpy(b.kind_degree.astype(np.int16)).cuda(), torch.from_numpy(b.cp_offset).cuda(),
                        ctrl, torch.from_numpy(b.w).cuda(), 3, torch.from_numpy(b.knot_offset).cuda(),
                        torch.from_numpy(b.knots).cuda(), b.n_t, "bernstein")
    t, v = torch.from_numpy(b.t).cuda(), torch.from_numpy(b.v).cuda()
    out = torch.empty((3, n_q), device="cuda")
    plan.autotune(t, out)
    ms = timed(lambda: plan(t, out=out, v=v), torch, iters=20)
    nbytes = batch_bytes(b, 4)
    rec = {"us": ms * 1e3, "G/s": n_q / (ms * 1e-3) / 1e9, "frac": hbm_roof(nbytes, ms)["frac"]}
    if cpu:
        import oracle
        kinds = b.kind_degree >> 8
        idx = np.unique(np.concatenate([np.random.default_rng(8).choice(b.n_obj, n_sample, replace=False),
                                        np.nonzero(kinds == 3)[0][:256]]))
        sub = b.subset(idx)
        got = out.view(3, b.n_obj, b.n_t)[:, torch.from_numpy(idx).cuda()].reshape(3, -1).cpu().numpy()
        ext = np.array([_box(sub.ctrl[sub.cp_offset[i] * 3:sub.cp_offset[i + 1] * 3].astype(np.float64).reshape(3, -1))
                        for i in range(len(idx))])
        rec["max_err_bbox"] = max_err_bbox(got, oracle.batch_eval(sub), ext, b.n_t)
    plan.close()
    return rec


def _box(P):
    """Error normaliser of one object's control points P[dim][m]: the largest
    side of their bounding box, floored at FP32_RESOLVABLE of the largest
    |coordinate|."""
    return max((P.max(axis=1) - P.min(axis=1)).max(), FP32_RESOLVABLE * np.abs(P).max(), 1e-30)


def chain_record(torch, bz, bz_synth, cpu, n_seg=1 << 20, n_q=1 << 24):
    """The C0 quadratic chain (zig-zag texels in cache-line tiles), secondary."""
    log("chain: generating %d segments, %d T" % (n_seg, n_q))
    chain, T = bz_synth.chain_walk(n_seg=n_seg, dim=3, n_q=n_q)
    chain_d, T_d = torch.from_numpy(chain).cuda(), torch.from_numpy(T).cuda()
    grid = bz.encode_piecewise(chain_d)
    tiles = bz.tile_piecewise(grid)
    out = torch.empty((3, n_q), device="cuda")
    ms = timed(lambda: bz.eval_piecewise_tiled(tiles, n_seg, 3, T_d, out=out), torch, iters=20)
    nbytes = chain_bytes(n_seg, 3, n_q)
    rec = {"us": ms * 1e3, "G/s": n_q / (ms * 1e-3) / 1e9, "frac": hbm_roof(nbytes, ms)["frac"]}
    traffic = recorded_traffic(CHAIN_COUNTERS, {"n_seg": n_seg, "n_q": n_q}, "tiled")
    if traffic:
        rec["traffic_over_algorithmic"] = traffic / nbytes
        rec["traffic_frac"] = traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    # the same tiles with FP16 texels (2.2x fewer bytes; error: the texel rounding)
    tiles16 = bz.tile_piecewise16(grid, torch.float16)
    out16 = torch.empty((3, n_q), device="cuda")
    ms16 = timed(lambda: bz.eval_piecewise_tiled16(tiles16, n_seg, 3, T_d, out=out16), torch, iters=20)
    nb16 = chain_bytes(n_seg, 3, n_q, es=2)
    ext = float((chain.max(axis=0) - chain.min(axis=0)).max())
    rec["fp16"] = {"us": ms16 * 1e3, "G/s": n_q / (ms16 * 1e-3) / 1e9, "frac": hbm_roof(nb16, ms16)["frac"],
                   "max_diff_vs_fp32_bbox": float((out16 - out).abs().max().item()) / ext}
    traffic16 = recorded_traffic(CHAIN_COUNTERS, {"n_seg": n_seg, "n_q": n_q}, "tiled16")
    if traffic16:
        rec["fp16"]["traffic_over_algorithmic"] = traffic16 / nb16
    if cpu:
        import oracle
        m = 1 << 20
        ref = oracle.chain_eval(chain, T[:m])
        rec["max_err_bbox"] = float(np.abs(out[:, :m].cpu().numpy().astype(np.float64) - ref).max() / ext)
        rec["fp16"]["max_err_bbox"] = float(np.abs(out16[:, :m].cpu().numpy().astype(np.float64) - ref).max() / ext)
    return rec


def _round(x, nd=4):
    """Floats to `nd` significant digits, recursively (keeps the line short)."""
    if isinstance(x, float):
        return float("%.*g" % (nd, x))
    if isinstance(x, dict):
        return {k: _round(v, nd) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_round(v, nd) for v in x]
    return x


def compact_record(head, batched, chain, steps, warmup, n_curves, n_t, suite_file=None, suite_summary=None):
    """The final JSON line: the bench contract's keys with the plain FP32
    headline, and the batched FP32 / FP16 and chain records beside it."""
    rec = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "G evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain FP32: %d cubic 3D Bezier curves x %d uniform t, 3 forms" % (n_curves, n_t),
                   "timing": "step = 3 launches (3 x %d evals); %d steps in 1 HIP graph, 1 replay, wall"
                             % (n_curves * n_t, steps),
                   "n_curves": n_curves, "n_t": n_t, "dim": 3, "degree": 3},
        "roofline": head["roofline"],
    }
    for k in ("cpu_baseline", "max_err_bbox", "forms", "launch_floor", "x16_random_t", "replay_ms_per_step"):
        if k in head:
            rec[k] = head[k]
    if batched:
        rec["batched"] = batched
    if chain:
        rec["chain"] = chain
    if suite_summary:
        rec["suite"] = suite_summary
    if suite_file:
        rec["suite_file"] = suite_file
    rec = _round(rec)
    for k in ("value", "ms_per_step"):
        rec[k] = float("%.6g" % head[k])
    return rec


def suite_summary(suite):
    """One [G/s, roofline fraction] pair per suite workload, for the final line."""
    out = {}

    def pick(name, e):
        if isinstance(e, dict) and "value" in e and "roofline" in e:
            out[name] = [e["value"], e["roofline"]["frac"]]

    for w, rec in suite.items():
        if not isinstance(rec, dict):
            continue
        pick(w, rec)
        for k, e in rec.items():
            if k in ("cpu_baseline",):
                continue
            pick(w + "." + k, e)
    return _round(out, 3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n-curves", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline legs")
    ap.add_argument("--headline-only", action="store_true", help="plain headline only (no batch, no chain)")
    ap.add_argument("--suite", action="store_true", help="also run every suite workload (written to --suite-out)")
    ap.add_argument("--suite-out", default="bench_suite.json", help="file for the full suite record")
    ap.add_argument("--suite-only", choices=["plain", "chain_footprint", "cubic_chain", "texemu", "batched", "patches",
                                             "volumes", "fit", "particles", "chain"], default=None,
                    help="run one suite workload only (no headline) and print its record")
    ap.add_argument("--n-seg", type=int, default=1 << 20, help="chain segments (--suite-only chain)")
    ap.add_argument("--n-q", type=int, default=1 << 24, help="chain queries (--suite-only chain)")
    ap.add_argument("--layout", choices=["grid", "tiled"], default="tiled",
                    help="placement of the zig-zag texels for --suite-only chain")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import bz_synth
    import paper_2603_15447_amd as bz

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}), flush=True)
        return
    suites = {"plain": suite_plain, "chain_footprint": suite_chain_footprint, "cubic_chain": suite_cubic_chain,
              "texemu": suite_texemu, "batched": suite_batched, "patches": suite_patches, "volumes": suite_volumes,
              "fit": suite_fit, "particles": suite_particles}
    if args.suite_only == "chain":
        print(json.dumps({"chain": suite_chain(torch, bz, bz_synth, args)}), flush=True)
        return
    if args.suite_only:
        print(json.dumps({args.suite_only: suites[args.suite_only](torch, bz, bz_synth, not args.no_cpu)}),
              flush=True)
        return
    cpu = not args.no_cpu
    head = headline_plain(torch, bz, bz_synth, args.steps, args.warmup, cpu, n_curves=args.n_curves)
    log("headline: %.2f G evals/s (%.4f ms per step)" % (head["value"], head["ms_per_step"]))
    torch.cuda.empty_cache()
    batched = chain = None
    if not args.headline_only:
        batched = batched_record(torch, bz, bz_synth, cpu)
        torch.cuda.empty_cache()
        chain = chain_record(torch, bz, bz_synth, cpu)
        torch.cuda.empty_cache()
    summary = suite_file = None
    if args.suite:
        suite = {"chain": suite_chain(torch, bz, bz_synth, args)}
        for name, fn in suites.items():
            suite[name] = fn(torch, bz, bz_synth, cpu)
            torch.cuda.empty_cache()
        with open(args.suite_out, "w") as f:
            json.dump(suite, f)
        summary, suite_file = suite_summary(suite), args.suite_out
    rec = compact_record(head, batched, chain, args.steps, args.warmup, args.n_curves, 256, suite_file, summary)
    line = json.dumps(rec, separators=(",", ":"))
    if len(line) > RECORD_MAX_BYTES:  # drop the least important parts rather than overflow
        for k in ("suite", "x16_random_t", "forms"):
            rec.pop(k, None)
            line = json.dumps(rec, separators=(",", ":"))
            if len(line) <= RECORD_MAX_BYTES:
                break
    print(line, flush=True)


def suite_chain(torch, bz, bz_synth, args):
    """The C0 quadratic chain in full (both texel layouts, encoder time, the
    HBM probes, the random-line gather ceiling, counters-based traffic and the
    CPU baseline)."""
    dim = 3
    log("suite: quadratic chain (generating the chain)")
    chain, T = bz_synth.chain_walk(n_seg=args.n_seg, dim=dim, n_q=args.n_q)
    chain_d = torch.from_numpy(chain).cuda()
    T_d = torch.from_numpy(T).cuda()
    grid = torch.empty((args.n_seg + 1, 2, dim), dtype=torch.float32, device="cuda")
    out = torch.empty((dim, args.n_q), dtype=torch.float32, device="cuda")
    bz.encode_piecewise(chain_d, out=grid)
    torch.cuda.synchronize()
    enc_ms = event_time_ms(lambda: bz.encode_piecewise(chain_d, out=grid), 5, torch)
    tiles = bz.tile_piecewise(grid)
    steps = {"grid": lambda: bz.eval_piecewise(grid, T_d, out=out),
             "tiled": lambda: bz.eval_piecewise_tiled(tiles, args.n_seg, dim, T_d, out=out)}
    other = "grid" if args.layout == "tiled" else "tiled"
    other_ms = timed(steps[other], torch, iters=50)
    kern_ms = timed(steps[args.layout], torch, iters=200, warmup=20)
    nbytes = chain_bytes(args.n_seg, dim, args.n_q)
    roof = hbm_roof(nbytes, kern_ms)
    roof["traffic"] = recorded_traffic(CHAIN_COUNTERS, {"n_seg": args.n_seg, "n_q": args.n_q}, args.layout)
    rec = {"workload": "C0 piecewise quadratic chain, zig-zag encoded (E=(B+C)/2), %d segments, %d uniform random "
                       "global T, 3D, FP32" % (args.n_seg, args.n_q),
           "layout": args.layout, "kernel_ms": kern_ms, "value": args.n_q / (kern_ms * 1e-3) / 1e9,
           "roofline": roof, "algorithmic_bytes": nbytes,
           "other_layout": {"layout": other, "kernel_ms": other_ms, "value": args.n_q / (other_ms * 1e-3) / 1e9},
           "encode_ms": enc_ms}
    probe = hbm_probe(torch, bz)
    probe["frac_of_read"] = roof["achieved"] / probe["read_GB/s"]
    rec["hbm_probe"] = probe
    if args.layout == "tiled":
        rec["gather_ceiling"] = gather_ceiling(torch, bz, tiles, args.n_q, kern_ms)
        # the same tiles with FP16 texels: 2.25x fewer bytes, one line per query
        tiles16 = bz.tile_piecewise16(grid, torch.float16)
        out16 = torch.empty_like(out)
        ms16 = timed(lambda: bz.eval_piecewise_tiled16(tiles16, args.n_seg, dim, T_d, out=out16), torch, iters=200,
                     warmup=20)
        nb16 = chain_bytes(args.n_seg, dim, args.n_q, es=2)
        bz.eval_piecewise_tiled(tiles, args.n_seg, dim, T_d, out=out)
        ext = float((chain.max(axis=0) - chain.min(axis=0)).max())
        ceiling16 = gather_ceiling(torch, bz, tiles16.view(torch.float32), args.n_q, ms16, vec16=2)
        rec["fp16_texels"] = {"kernel_ms": ms16, "value": args.n_q / (ms16 * 1e-3) / 1e9,
                              "roofline": hbm_roof(nb16, ms16), "algorithmic_bytes": nb16,
                              "tiles_MB": tiles16.numel() * 2 / 1e6, "gather_ceiling": ceiling16,
                              "max_diff_vs_fp32_bbox": float((out16 - out).abs().max().item()) / ext}
        del tiles16, out16
    if roof["traffic"]:
        rate = roof["traffic"] / (kern_ms * 1e-3) / 1e9
        rec["actual_traffic"] = {"bytes_per_launch": roof["traffic"], "over_algorithmic": roof["traffic"] / nbytes,
                                 "GB/s": rate, "frac_of_peak": rate / HBM_PEAK_GBS,
                                 "frac_of_read_probe": rate / probe["read_GB/s"]}
    if not args.no_cpu:
        rec["cpu_baseline"], rec["max_err_bbox"] = cpu_baseline_chain(chain, T, out)
    return rec


if __name__ == "__main__":
    main()
