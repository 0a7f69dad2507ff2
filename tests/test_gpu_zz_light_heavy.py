"""GPU parity of the light/heavy edge split (OG_FLAG_LIGHT_HEAVY, Meyer and
Sanders' Delta-stepping) through the C ABI.  This file is collected last
among the GPU tests (its name sorts after the others).  The split changes only which
round relaxes an edge, never the result: distances and canonical
predecessors must equal the oracle's bit for bit for every Delta (all edges
light, all heavy, or mixed), update, engine and query shape, and rows long
enough for the wavefront split pass must be split correctly too.
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LH = og.OG_FLAG_LIGHT_HEAVY


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def graphs():
    out = {"grid": gg.grid(64, 64, 1, 100, seed=0), "road": gg.road(256, seed=0), "rmat": gg.rmat(14, 16, seed=0)}
    return {k: (g, og.DeviceGraph.from_host(g, DEV)) for k, g in out.items()}


def check(orc, g, src, d, p, tag):
    ref_d, ref_p = orc.sssp(g, src)
    d = d.cpu().numpy()
    assert np.array_equal(d, ref_d), f"{tag}: {int(np.count_nonzero(d != ref_d))} distances differ"
    if p is not None:
        assert np.array_equal(p.cpu().numpy(), ref_p), f"{tag}: predecessors differ"


@pytest.mark.parametrize("engine", [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS])
@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
@pytest.mark.parametrize("kind,delta", [("grid", 1), ("grid", 16), ("grid", 100), ("road", 16), ("road", 512),
                                        ("rmat", 4), ("rmat", 32), ("rmat", 2000)])
def test_split_parity(orc, graphs, kind, delta, update, engine):
    g, dg = graphs[kind]
    for src in gg.pick_sources(g, 2, seed=31):
        tag = f"split {kind} src={src} delta={delta} update={update} engine={engine}"
        say(tag)
        d, p, st = og.sssp(dg, int(src), og.Schedule(delta=delta, update=update, engine=engine, flags=LH))
        torch.cuda.synchronize()
        check(orc, g, int(src), d, p, tag)


@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
def test_split_hub_heavy_slices(orc, update):
    """Heavy parts longer than 4,096 edges are filed as one heavy-list entry
    per 4,096-edge slice: a path of light edges with two hubs joined to every
    path vertex by heavy edges (heavy parts of 9,000 edges, three slices each,
    many of them shortening paths) gives the oracle's distances and canonical
    predecessors."""
    N, delta = 9000, 64
    rng = np.random.default_rng(41)
    src, dst, w = [], [], []
    pw = rng.integers(1, 8, N - 1)
    for i in range(N - 1):
        src += [i, i + 1]
        dst += [i + 1, i]
        w += [int(pw[i])] * 2
    for h in (N, N + 1):
        hw = rng.integers(delta, 3 * delta, N)
        for i in range(N):
            src += [h, i]
            dst += [i, h]
            w += [int(hw[i])] * 2
    g = gg.from_edges(N + 2, src, dst, w)
    dg = og.DeviceGraph.from_host(g, DEV)
    for s0 in (0, N // 2, N + 1):
        tag = f"split hubs src={s0} update={update}"
        say(tag)
        d, p, st = og.sssp(dg, s0, og.Schedule(delta=delta, update=update, flags=LH))
        torch.cuda.synchronize()
        assert st["status"] == 0
        check(orc, g, s0, d, p, tag)
    # the same three queries in one launch: every copy files its hubs' slices
    say(f"split hubs batch x3 update={update}")
    d, p, st = og.sssp_batch(dg, [0, N // 2, N + 1], og.Schedule(delta=delta, update=update, flags=LH))
    torch.cuda.synchronize()
    assert st["status"] == 0
    for q, s0 in enumerate((0, N // 2, N + 1)):
        check(orc, g, s0, d[q], p[q], f"split hubs batch q={q}")


def test_split_reduces_relaxations(orc, graphs):
    g, dg = graphs["rmat"]
    src = int(gg.pick_sources(g, 1, seed=32)[0])
    say("split vs plain relaxation counts, rmat delta=32")
    _, _, plain = og.sssp(dg, src, og.Schedule(delta=32, update=og.OG_EAGER_NO_FUSION))
    d, p, st = og.sssp(dg, src, og.Schedule(delta=32, update=og.OG_EAGER_NO_FUSION, flags=LH))
    torch.cuda.synchronize()
    check(orc, g, src, d, p, "split counts")
    assert st["relaxations"] <= plain["relaxations"]


def test_split_long_rows_and_ties(orc):
    """A star with 5,000 leaves (rows longer than the per-thread split) and
    mixed light/heavy weights with many ties and zeros."""
    rng = np.random.default_rng(33)
    n = 5001
    leaves = np.arange(1, n)
    src = np.concatenate([np.zeros(n - 1, dtype=np.int64), leaves])
    dst = np.concatenate([leaves, np.zeros(n - 1, dtype=np.int64)])
    extra = rng.integers(1, n, size=(20000, 2))
    src = np.concatenate([src, extra[:, 0]])
    dst = np.concatenate([dst, extra[:, 1]])
    w = rng.integers(0, 40, size=len(src))
    g = gg.from_edges(n, src, dst, w)
    dg = og.DeviceGraph.from_host(g, DEV)
    for delta in (1, 8, 20, 64):
        for s in (0, 17, 4999):
            say(f"split star delta={delta} src={s}")
            d, p, st = og.sssp(dg, s, og.Schedule(delta=delta, flags=LH))
            torch.cuda.synchronize()
            ref_d, _ = orc.sssp(g, s)
            assert np.array_equal(d.cpu().numpy(), ref_d)
            assert orc.check(g, s, d.cpu().numpy(), None) == 0


def test_split_batch_ppsp_astar_wbfs_f32(orc, graphs):
    g, dg = graphs["road"]
    srcs = gg.pick_sources(g, 6, seed=34)
    say("split sssp_batch x6")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=64, flags=LH))
    torch.cuda.synchronize()
    for q, s in enumerate(srcs):
        check(orc, g, int(s), d[q], p[q], f"split batch q={q}")
    rng = np.random.default_rng(35)
    for i in range(3):
        s, t = int(srcs[i]), int(rng.integers(0, g.n))
        want = orc.ppsp(g, s, t)
        exp = og.INF if want < 0 else want
        say(f"split ppsp/astar s={s} t={t}")
        dist, _, _ = og.ppsp(dg, s, t, og.Schedule(delta=32, flags=LH))
        h = torch.from_numpy(gg.grid_heuristic(256, t)).to(DEV)
        dista, _, _ = og.astar(dg, s, t, h, og.Schedule(delta=16, flags=LH))
        torch.cuda.synchronize()
        assert int(dist[t]) == exp and int(dista[t]) == exp
    rg, _ = graphs["rmat"]
    wg = gg.with_weights(rg, rg.w % 13 + 1)
    s = int(gg.pick_sources(wg, 1, seed=36)[0])
    say("split wbfs (every edge heavy at Delta 1)")
    d, p, st = og.wbfs(og.DeviceGraph.from_host(wg, DEV), s, og.Schedule(flags=LH))
    torch.cuda.synchronize()
    check(orc, wg, s, d, p, "split wbfs")
    say("split is int32-only: float32 weights are rejected")
    w = torch.from_numpy(gg.float_weights(g, 1.0, 1000.0, seed=9)).to(DEV)
    _, _, _, st = og.sssp_f32(dg, w, int(srcs[0]), og.Schedule(delta=300, flags=LH), check=False)
    assert st["status"] == og.OG_ERR_INVALID_ARG


@pytest.mark.slow
def test_split_rmat20(orc):
    g = gg.rmat(20, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    say("split rmat20 delta=32 unfused")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=32, update=og.OG_EAGER_NO_FUSION, flags=LH))
    torch.cuda.synchronize()
    check(orc, g, src, d, p, "split rmat20")


@pytest.mark.slow
def test_split_rmat24_kept_full_size(orc):
    """The R-MAT benchmark line's schedule at its full size: R-MAT scale 24,
    the benchmark's first two sources, Delta 64, unfused, light/heavy split
    with the copy kept (the first call builds it, the second reuses it):
    distances and predecessors bit-exact."""
    say("rmat24: generating")
    g = gg.rmat(24, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    ws = og.Workspace(DEV)
    srcs = [int(x) for x in gg.pick_sources(g, 4, seed=2)][:2]
    for i, src in enumerate(srcs):
        say(f"split rmat24 src={src} delta=64 unfused kept ({'build' if i == 0 else 'reuse'})")
        d, p, st = og.sssp(dg, src, og.Schedule(delta=64, update=og.OG_EAGER_NO_FUSION,
                                                flags=LH | og.OG_FLAG_KEEP_SPLIT), ws=ws)
        torch.cuda.synchronize()
        assert st["status"] == 0
        say(f"split rmat24 src={src}: oracle")
        check(orc, g, src, d, p, f"split rmat24 src={src}")


def test_split_copy_kept_across_calls(orc, graphs):
    """OG_FLAG_KEEP_SPLIT reuses the split copy of the previous split call on
    the same workspace, graph and Delta, and rebuilds it whenever one of them
    changed or another call used the workspace in between; every result must
    still be the oracle's."""
    g, dg = graphs["rmat"]
    rg, rdg = graphs["road"]
    ws = og.Workspace(DEV)
    keep = LH | og.OG_FLAG_KEEP_SPLIT
    srcs = [int(x) for x in gg.pick_sources(g, 3, seed=35)]
    rsrc = int(gg.pick_sources(rg, 1, seed=36)[0])
    w2 = gg.with_weights(g, g.w % 50 + 1)
    dg2 = og.DeviceGraph.from_host(w2, DEV)
    steps = [
        ("build", dg, g, srcs[0], 64, keep),
        ("reuse", dg, g, srcs[1], 64, keep),
        ("reuse again", dg, g, srcs[2], 64, keep),
        ("other delta: rebuild", dg, g, srcs[0], 16, keep),
        ("back to 64: rebuild", dg, g, srcs[1], 64, keep),
        ("plain call on the workspace", dg, g, srcs[2], 64, 0),
        ("after it: rebuild", dg, g, srcs[0], 64, keep),
        ("other graph of the same shape: rebuild", dg2, w2, srcs[1], 64, keep),
        ("road graph: rebuild", rdg, rg, rsrc, 512, keep),
        ("road reuse", rdg, rg, rsrc, 512, keep),
        ("split without keep: rebuild", dg, g, srcs[2], 64, LH),
        ("reuse after it", dg, g, srcs[0], 64, keep),
    ]
    for tag, dgx, gx, src, delta, flags in steps:
        say(f"keep split: {tag}")
        d, p, st = og.sssp(dgx, src, og.Schedule(delta=delta, update=og.OG_EAGER_NO_FUSION, flags=flags), ws=ws)
        torch.cuda.synchronize()
        assert st["status"] == 0
        check(orc, gx, src, d, p, f"keep split: {tag}")
