"""The schedule autotuner on the device: every candidate it times runs
through the C ABI, and the schedule it returns must give the oracle's
distances (timing decides the choice, so the choice itself is only checked
for validity)."""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og
from paper_1911_07260_amd.autotune import Autotuner

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_autotune_sssp_road(orc):
    g = gg.road(256, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    srcs = gg.pick_sources(g, 2, seed=41)
    say("autotune sssp road256 (eager, lazy, directions, bins)")
    res = Autotuner.for_sssp(dg, srcs).tune(weight_scale=float(np.median(g.w)), lazy=True)
    assert np.isfinite(res.best_ms) and res.best_ms == min(t.engine_ms for t in res.trials if t.ok)
    assert len(res.trials) > 20
    for s in srcs:
        d, p, st = og.sssp(dg, int(s), res.best)
        torch.cuda.synchronize()
        ref_d, ref_p = orc.sssp(g, int(s))
        assert np.array_equal(d.cpu().numpy(), ref_d) and np.array_equal(p.cpu().numpy(), ref_p)


def test_autotune_ppsp_batch(orc):
    g = gg.road(128, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    rng = np.random.default_rng(42)
    srcs = gg.pick_sources(g, 16, seed=43)
    tgts = rng.integers(0, g.n, size=16)
    h = gg.grid_heuristic_device(128, tgts, device=DEV)
    say("autotune astar batch road128 x16")
    res = Autotuner.for_ppsp_batch(dg, srcs, tgts, h).tune(weight_scale=float(np.median(g.w)))
    d, _, _ = og.astar_batch(dg, srcs, tgts, h, res.best)
    torch.cuda.synchronize()
    for q in range(16):
        want = orc.ppsp(g, int(srcs[q]), int(tgts[q]))
        assert int(d[q][int(tgts[q])]) == (og.INF if want < 0 else want)
