"""GPU: library calls captured into a HIP graph (torch.cuda.CUDAGraph) and
replayed several times, with eager work and synchronisations between the
replays and the inputs changed in place between them; every replay must
equal the eager call on the same inputs.  The batched plan's persistent
kernel resets its own tile counters at the end of a launch, so it needs no
memset inside a captured graph; its atomic-counter schedule is covered here."""
import numpy as np
import pytest
import torch

import bz_synth
import paper_2603_15447_amd as bz
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu


def _capture(fn):
    """Warm up on a side stream, then capture fn() once."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def _replays(g, out, refill, n=4):
    """Replay n times; before each, refill the inputs in place (refill(i)
    returns the eager result for them) and poison the output."""
    for i in range(n):
        want = refill(i)
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.clone()
        assert torch.equal(got, want), i
        _ = (got * 2.0).sum().item()  # unrelated eager work between replays


def test_graph_plain_curves():
    ctrl, t = bz_synth.plain_curves(n_curves=1024)
    c = to_dev(ctrl)
    td = to_dev(t)
    out = torch.empty((3, 1024 * t.shape[0]), device="cuda")
    g = _capture(lambda: bz.eval_bezier(c, td, "bernstein", out=out))
    rng = np.random.default_rng(5)

    def refill(i):
        c.copy_(to_dev(rng.uniform(-1, 1, size=ctrl.shape).astype(np.float32)))
        return bz.eval_bezier(c, td, "bernstein")

    _replays(g, out, refill)


def test_graph_chain_tiled():
    chain, T = bz_synth.chain_walk(n_seg=4096, dim=3, n_q=100003, seed=31)
    grid = bz.encode_piecewise(to_dev(chain))
    tiles = bz.tile_piecewise(grid)
    Td = to_dev(T)
    out = torch.empty((3, T.shape[0]), device="cuda")
    g = _capture(lambda: bz.eval_piecewise_tiled(tiles, 4096, 3, Td, out=out))
    rng = np.random.default_rng(6)

    def refill(i):
        Td.copy_(to_dev((rng.random(T.shape[0]) * 4096).astype(np.float32)))
        return bz.eval_piecewise_tiled(tiles, 4096, 3, Td)

    _replays(g, out, refill)


@pytest.mark.parametrize("schedule,window", [("static", 0), ("dynamic", 0), ("static", 500), ("dynamic", 500)])
def test_graph_batched(schedule, window):
    b = bz_synth.mixed_batch(n_bezier=3000, n_nurbs=300, n_t=16, seed=21)
    dev = {
        "kd": torch.from_numpy(b.kind_degree.astype(np.int16)).cuda(),
        "cpo": torch.from_numpy(b.cp_offset).cuda(),
        "ko": torch.from_numpy(b.knot_offset).cuda(),
        "kn": to_dev(b.knots),
    }
    plan = bz.BatchPlan(dev["kd"], dev["cpo"], to_dev(b.ctrl), to_dev(b.w), 3, dev["ko"], dev["kn"], 16)
    plan.configure(600, 2, schedule, 4, window)
    t = to_dev(b.t)
    out = torch.empty((3, b.n_obj * 16), device="cuda")
    g = _capture(lambda: plan(t, out=out))
    rng = np.random.default_rng(7)

    def refill(i):
        t.copy_(to_dev(rng.random(b.t.shape).astype(np.float32)))
        return plan(t)  # eager launch on the same plan: the counters must be back at zero

    _replays(g, out, refill, n=5)
    plan.close()


def test_graph_texture_reads():
    ctrl, t = bz_synth.plain_curves(n_curves=512)
    tex = bz.build_texture(to_dev(ctrl), "seiler")
    td = to_dev(t)
    out = torch.empty((3, 512 * t.shape[0]), device="cuda")
    g = _capture(lambda: bz.eval_texture(tex, 3, "seiler", td, 8, "nearest", out=out))
    rng = np.random.default_rng(8)

    def refill(i):
        td.copy_(to_dev(rng.random(t.shape[0]).astype(np.float32)))
        return bz.eval_texture(tex, 3, "seiler", td, 8, "nearest")

    _replays(g, out, refill)
