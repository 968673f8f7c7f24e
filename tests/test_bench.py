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


def test_alu_roof_reports_both_peaks():
    r = bench.alu_roof(39.3216)
    assert r["bound"] == "alu" and abs(r["peak"] - 78.6432) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert r["published_peak"] == 157.3 and abs(r["frac_of_published"] - 39.3216 / 157.3) < 1e-12


def test_chain_bytes():
    # grid (n_seg+1) x 2 x dim floats, T in, dim floats out per query
    assert bench.chain_bytes(1 << 20, 3, 1 << 24) == ((1 << 20) + 1) * 24 + (1 << 24) * 16
    assert bench.chain_bytes(1, 1, 0) == 16
    assert bench.chain_bytes(1 << 20, 3, 1 << 24, es=2) == ((1 << 20) + 1) * 12 + (1 << 24) * 16


def test_particle_frame_bytes():
    # T in and out, speed in, x y z out, shade out: seven floats per particle
    assert bench.particle_frame_bytes(10_000_000) == 10_000_000 * 7 * 4


def test_batch_bytes_counts_each_part():
    b = bz_synth.mixed_batch(n_bezier=40, n_nurbs=6, n_t=5, seed=3)
    kind = b.kind_degree >> 8
    ncp = np.diff(b.cp_offset)
    nk = np.diff(b.knot_offset)
    for es in (4, 2):
        got = bench.batch_bytes(b, es)
        want = (ncp.sum() * 3 * es + ncp[kind != 0].sum() * es + nk.sum() * 4 + b.n_obj * 8 + (kind == 2).sum() * 8
                + b.n_obj * 5 * 16)
        assert got == want


def test_batch_bytes_of_the_mixed_workload():
    # 2^20 Bezier curves of degree 2..15 (half rational) + 2^16 cubic NURBS,
    # 16 t each: about 477 MB with FP32 storage and 391 MB with FP16
    b = bz_synth.mixed_batch()
    assert abs(bench.batch_bytes(b, 4) / 1e6 - 477) < 2
    assert abs(bench.batch_bytes(b, 2) / 1e6 - 391) < 2


def test_plain_bytes():
    # 4096 cubic 3D curves x 256 shared t: points out, control points and t once
    assert bench.plain_bytes(4096, 3, 3, 256) == 4096 * 256 * 12 + 4096 * 48 + 256 * 4 == 12_780_544


def test_recorded_traffic_is_bound_to_its_workload():
    wl = {"n_seg": 1 << 20, "n_q": 1 << 24}
    with open(os.path.join(ROOT, "profiles", bench.CHAIN_COUNTERS)) as f:
        d = json.load(f)
    for layout in ("grid", "tiled", "tiled16"):
        t = bench.recorded_traffic(bench.CHAIN_COUNTERS, wl, layout)
        assert t in (None, d["traffic_bytes_per_dispatch"][layout])  # None once a kernel source has changed
        assert bench.recorded_traffic(bench.CHAIN_COUNTERS, {"n_seg": 1 << 12, "n_q": 1 << 16}, layout) is None
    assert bench.recorded_traffic("no_such_file.json", wl) is None


def test_recorded_traffic_per_kernel_and_source(tmp_path, monkeypatch):
    # a summary naming several kernels is read per key, and any changed source voids it
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    import hashlib
    d = {"kernel_sources": {"k.hip": hashlib.sha256(b"kernel v1").hexdigest()}, "workload": {"n": 4},
         "traffic_bytes_per_dispatch": {"a": 100.0, "b": 200.0}}
    (prof / "x.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("x.json", {"n": 4}, "b") == 200.0
    assert bench.recorded_traffic("x.json", {"n": 5}, "b") is None
    src.write_bytes(b"kernel v2")
    assert bench.recorded_traffic("x.json", {"n": 4}, "b") is None


def _synthetic_records():
    rng = np.random.default_rng(0)
    r = lambda: float(rng.random() * 1e3 + 1e-7)  # noqa: E731
    forms = {m: {"us": r(), "G/s": r(), "frac": r()} for m in bench.FORMS}
    head = {"value": r(), "ms_per_step": r(), "gpu_ms_per_step": r(), "replay_ms_per_step": r(),
            "eager_ms_per_step": r(), "forms": forms,
            "x16_random_t": {"G/s": [r() for _ in bench.FORMS], "frac": [r() for _ in bench.FORMS]},
            "launch_floor": {"us": r(), "bytes": 12582912, "of_dominant": r()},
            "roofline": {"bound": "hbm", "achieved": r(), "peak": 8000.0, "unit": "GB/s", "frac": r(),
                         "traffic": r(), "kernel": "k_curves<seiler>", "bytes_per_launch": 12780544},
            "max_err_bbox": {m: r() for m in bench.FORMS},
            "cpu_baseline": {"value": r(), "unit": "G evals/s", "cores": 16, "kind": "oracle",
                             "sample": "3 forms x 4096 x 256 points, FP64, 200 reps",
                             "host": "AMD EPYC 9575F 64-Core Processor"}}
    batched = {n: {"us": r(), "G/s": r(), "frac": r(), "bytes": 477089864, "max_err_bbox": r(),
                   "max_err_bbox_vs_rounded": r(), "config": [3072, 4, "static", 4, 131072]}
               for n in ("fp32", "fp16")}
    batched["cpu_baseline"] = {"value": r(), "unit": "G evals/s", "cores": 16, "kind": "oracle",
                               "sample": "16384 random objects x 16 t, FP64"}
    batched["fp16_speedup"] = r()
    chain = {"us": r(), "G/s": r(), "frac": r(), "traffic_over_algorithmic": r(), "traffic_frac": r(),
             "max_err_bbox": r(), "fp16": {"us": r(), "G/s": r(), "frac": r(), "max_diff_vs_fp32_bbox": r(),
                                          "max_err_bbox": r()}}
    suite = {w: {"value": r(), "roofline": {"frac": r()}, **{k: {"value": r(), "roofline": {"frac": r()}}
                                                            for k in ("a", "bb", "ccc", "dddd")}}
             for w in ("plain", "cubic_chain", "texemu", "batched", "patches", "volumes", "fit", "particles")}
    return head, batched, chain, suite


def test_final_record_is_compact_and_complete():
    head, batched, chain, suite = _synthetic_records()
    for summary in (None, bench.suite_summary(suite)):
        rec = bench.compact_record(head, batched, chain, 20, 5, 4096, 256, "bench_suite.json" if summary else None,
                                   summary)
        line = json.dumps(rec, separators=(",", ":"))
        for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                  "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "batched"):
            assert k in rec, k
        assert rec["metric"] == bench.METRIC and rec["n_gpus"] == 1 and rec["steps"] == 20
        assert set(rec["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
        assert "plain" in rec["config"]["workload"] and "graph" in rec["config"]["timing"]
        assert {"fp32", "fp16"} <= set(rec["batched"])
        assert set(rec["launch_floor"]) == {"us", "bytes", "of_dominant"}
        if summary is None:  # the contract's part alone fits well inside the limit, x16 included
            assert len(line) <= bench.RECORD_MAX_BYTES, len(line)
            assert "x16_random_t" in rec


def test_main_trims_the_line_to_the_limit():
    head, batched, chain, suite = _synthetic_records()
    rec = bench.compact_record(head, batched, chain, 20, 5, 4096, 256, "f.json", bench.suite_summary(suite))
    for k in ("suite", "x16_random_t", "forms"):
        if len(json.dumps(rec, separators=(",", ":"))) <= bench.RECORD_MAX_BYTES:
            break
        rec.pop(k, None)
    assert len(json.dumps(rec, separators=(",", ":"))) <= bench.RECORD_MAX_BYTES


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
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--headline-only", "--steps", "3", "--warmup",
                        "1", "--n-curves", "256"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1 and len(lines[0]) <= bench.RECORD_MAX_BYTES
    rec = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in rec, k
    assert rec["n_gpus"] == 1 and rec["steps"] == 3 and rec["warmup"] == 1 and rec["value"] > 0
    assert rec["config"]["n_curves"] == 256 and "workload" in rec["config"]
    roof = rec["roofline"]
    assert set(roof) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert roof["traffic"] is None  # counters were taken on the full-size workload only
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3 * roof["frac"]
    cb = rec["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]
    assert max(rec["max_err_bbox"].values()) < 1e-5
