"""Benchmark: random-access evaluation of a C0 quadratic chain in the
shared-diagonal (zig-zag) encoding on one MI355X.

Workload: a chain of 2^20 quadratic segments (control points a random walk
with U[-0.1,0.1]^3 steps), encoded once into the 2 x (N+1) zig-zag grid, then
evaluated at 2^24 uniform random global parameters T in [0, 2^20) per step.
One step is one bz_eval_piecewise call over all 2^24 queries (parameter
decode, grid gather, bilinear diagonal read, store), inputs resident in HBM.

Prints one JSON line: throughput in G curve-point evaluations/s, the HBM
roofline of the kernel (algorithmic bytes per launch over its event-timed
average duration), the max error against the FP64 oracle on a sample, and the
oracle's own throughput on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "G curve-point evals/s and % HBM roofline, plain FP32 vs batched/FP16 at max err"


def chain_bytes(n_seg, dim, n_q):
    """Algorithmic HBM bytes of one evaluation launch: the grid once, T in, points out."""
    return (n_seg + 1) * 2 * dim * 4 + n_q * 4 + n_q * dim * 4


def recorded_traffic(name="chain_eval_counters.json"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
        with open(os.path.join(ROOT, d["kernel_source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    return d["traffic_bytes_per_dispatch"] if sha == d["kernel_source_sha256"] else None


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


def cpu_baseline(chain, T, budget_s=10.0):
    import oracle
    n = T.shape[0]
    sample = T[: min(n, 1 << 22)]
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.chain_eval(chain, sample)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 8:
            break
    rate = reps * sample.shape[0] / el / 1e9
    return {"value": rate, "unit": "G evals/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%d x %d random T of the same 2^20-segment chain (FP64 chain definition, OpenMP)"
                      % (reps, sample.shape[0])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n-seg", type=int, default=1 << 20)
    ap.add_argument("--n-q", type=int, default=1 << 24)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
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
    dim = 3
    chain, T = bz_synth.chain_walk(n_seg=args.n_seg, dim=dim, n_q=args.n_q)
    chain_d = torch.from_numpy(chain).to(dev)
    T_d = torch.from_numpy(T).to(dev)
    grid = torch.empty((args.n_seg + 1, 2, dim), dtype=torch.float32, device=dev)
    out = torch.empty((dim, args.n_q), dtype=torch.float32, device=dev)
    bz.encode_piecewise(chain_d, out=grid)
    torch.cuda.synchronize()
    enc_ms = event_time_ms(lambda: bz.encode_piecewise(chain_d, out=grid), 5, torch)

    step = lambda: bz.eval_piecewise(grid, T_d, out=out)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    kern_ms = event_time_ms(step, args.steps, torch)

    # parity on a sample of outputs, every one recomputed by the FP64 oracle
    import oracle
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(args.n_q, size=min(args.n_q, 1 << 16), replace=False))
    got = out[:, torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    ref = oracle.chain_eval(chain, T[idx])
    ext = float((chain.max(axis=0) - chain.min(axis=0)).max())
    max_err = float(np.abs(got - ref).max() / ext)

    nbytes = chain_bytes(args.n_seg, dim, args.n_q)
    achieved = nbytes / (kern_ms * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": args.n_q / (ms_per_step * 1e-3) / 1e9,
        "unit": "G evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C0 piecewise quadratic chain, zig-zag encoded (E=(B+C)/2), %d segments, "
                               "%d uniform random global T, 3D, FP32" % (args.n_seg, args.n_q),
                   "n_seg": args.n_seg, "n_q": args.n_q, "dim": dim},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic()},
        "kernel": "k_piecewise_eval",
        "kernel_ms": kern_ms,
        "algorithmic_bytes": nbytes,
        "max_err_bbox": max_err,
        "encode_ms": enc_ms,
    }
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(chain, T)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
