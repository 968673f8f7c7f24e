"""The bench.py contract: argument handling and byte models on the CPU, and
(on a GPU) one small headline run whose JSON line carries every field."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import bz_synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_chain_bytes():
    # grid (n_seg+1) x 2 x dim floats, T in, dim floats out per query
    assert bench.chain_bytes(1 << 20, 3, 1 << 24) == ((1 << 20) + 1) * 24 + (1 << 24) * 16
    assert bench.chain_bytes(1, 1, 0) == 16


def test_particle_frame_bytes():
    # T in and out, speed in, x y z out, shade out: seven floats per particle
    assert bench.particle_frame_bytes(10_000_000) == 10_000_000 * 7 * 4


def test_batch_bytes_counts_each_part():
    b = bz_synth.mixed_batch(n_bezier=40, n_nurbs=6, n_t=5, seed=3)
    kind = b.kind_degree >> 8
    ncp = np.diff(b.cp_offset)
    n_segs = 17
    got = bench.batch_bytes(b, 4, n_segs, 3)
    want = (ncp[kind != 2].sum() * 3 * 4 + ncp[kind == 1].sum() * 4 + n_segs * 4 * 4 * 4 + (kind == 2).sum() * 12
            + n_segs * 4 + b.n_obj * 12 + b.n_obj * 5 * 16)
    assert got == want


def test_recorded_traffic_is_bound_to_its_workload():
    t = bench.recorded_traffic("chain_eval_tiled_counters.json", 1 << 20, 1 << 24)
    with open(os.path.join(ROOT, "profiles", "chain_eval_tiled_counters.json")) as f:
        d = json.load(f)
    assert t in (None, d["traffic_bytes_per_dispatch"])  # None once the kernel source has changed
    assert bench.recorded_traffic("chain_eval_tiled_counters.json", 1 << 12, 1 << 16) is None
    assert bench.recorded_traffic("no_such_file.json", 1 << 20, 1 << 24) is None


def test_cpu_baseline_leg_reports_both_thread_counts():
    import torch
    import oracle
    chain, T = bz_synth.chain_walk(n_seg=1 << 10, dim=3, n_q=1 << 14, seed=3)
    ref = oracle.chain_eval(chain, T)
    before = oracle.max_threads()
    cb, err = bench.cpu_baseline_chain(chain, T, torch.from_numpy(ref.astype(np.float32)), budget_s=0.2)
    assert oracle.max_threads() == before  # the single-thread leg puts the thread count back
    assert cb["kind"] == "oracle" and cb["cores"] == before and cb["value"] > 0
    assert cb["single_thread"]["cores"] == 1 and cb["single_thread"]["value"] > 0
    assert err < 1e-6  # FP32 rounding of the oracle's own values


def test_oracle_thread_count_does_not_change_results():
    import oracle
    chain, T = bz_synth.chain_walk(n_seg=1 << 9, dim=2, n_q=1 << 12, seed=4)
    a = oracle.chain_eval(chain, T)
    prev = oracle.set_threads(1)
    try:
        b = oracle.chain_eval(chain, T)
    finally:
        oracle.set_threads(prev)
    assert np.array_equal(a, b)


def test_roofline_fraction():
    r = bench.hbm_roof(8e9, 1000.0)  # 8 GB in one second
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and abs(r["frac"] - 1e-3) < 1e-12


@pytest.mark.gpu
def test_headline_json_line():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--no-suite", "--steps", "3", "--warmup", "1",
                        "--n-seg", "4096", "--n-q", "65536"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    rec = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == 3 and rec["warmup"] == 1 and rec["value"] > 0
    assert rec["config"]["n_seg"] == 4096 and "workload" in rec["config"]
    roof = rec["roofline"]
    assert set(roof) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert roof["traffic"] is None  # counters were taken on the full-size workload only
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-9
    cb = rec["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    assert rec["max_err_bbox"] < 1e-5
