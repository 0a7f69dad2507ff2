"""GPU parity of the lazy bucket update (section 3.1) and of k-core
decomposition (section 6.1) through the C ABI, against the CPU oracle.

Lazy SSSP reaches the same unique distances (and canonical predecessors)
as the eager engine, so it is compared bit for bit with the oracle's
Dijkstra over Delta, engines and query shapes.  Coreness is unique too:
every update mode (lazy with the constant-sum count, eager, eager with
fusion), window size, engine and queue capacity must give the oracle's
peeling result exactly.
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAZY = og.OG_LAZY_UPDATE


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def undirected(n, pairs):
    src = [a for a, b in pairs] + [b for a, b in pairs]
    dst = [b for a, b in pairs] + [a for a, b in pairs]
    return gg.from_edges(n, src, dst, np.ones(len(src), dtype=np.int64))


@pytest.fixture(scope="module")
def graphs():
    out = {
        "grid": gg.grid(64, 64, 1, 100, seed=0),
        "road": gg.road(256, seed=0),
        "rmat": gg.rmat(14, 16, seed=0),
    }
    return {k: (g, og.DeviceGraph.from_host(g, DEV)) for k, g in out.items()}


def check_sssp(orc, g, src, d, p, tag):
    ref_d, ref_p = orc.sssp(g, src)
    d = d.cpu().numpy()
    assert np.array_equal(d, ref_d), f"{tag}: {int(np.count_nonzero(d != ref_d))} distances differ"
    if p is not None:
        assert np.array_equal(p.cpu().numpy(), ref_p), f"{tag}: predecessors differ"


@pytest.mark.parametrize("engine", [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS])
@pytest.mark.parametrize("kind,delta", [("grid", 1), ("grid", 16), ("grid", 1 << 20), ("road", 256), ("road", 4096),
                                        ("rmat", 8), ("rmat", 64)])
def test_lazy_sssp(orc, graphs, kind, delta, engine):
    g, dg = graphs[kind]
    for src in gg.pick_sources(g, 2, seed=11):
        tag = f"lazy sssp {kind} src={src} delta={delta} engine={engine}"
        say(tag)
        d, p, st = og.sssp(dg, int(src), og.Schedule(delta=delta, update=LAZY, engine=engine))
        torch.cuda.synchronize()
        check_sssp(orc, g, int(src), d, p, tag)
        assert st["pushes_local"] == 0
        assert st["barriers"] == 2 * st["rounds"]


def test_lazy_small_window_and_far(orc, graphs):
    g, dg = graphs["road"]
    src = int(gg.pick_sources(g, 1, seed=12)[0])
    say("lazy K=2 delta=16")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=16, update=LAZY, window_buckets=2))
    torch.cuda.synchronize()
    assert st["far_pushes"] > 0
    check_sssp(orc, g, src, d, p, "lazy far")


def test_lazy_batch_wbfs_ppsp_astar(orc, graphs):
    g, dg = graphs["road"]
    srcs = gg.pick_sources(g, 8, seed=13)
    say("lazy sssp_batch x8")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=512, update=LAZY))
    torch.cuda.synchronize()
    for q, s in enumerate(srcs):
        check_sssp(orc, g, int(s), d[q], p[q], f"lazy batch q={q}")
    rg, _ = graphs["rmat"]
    wg = gg.with_weights(rg, rg.w % 13 + 1)
    dwg = og.DeviceGraph.from_host(wg, DEV)
    s = int(gg.pick_sources(wg, 1, seed=14)[0])
    say("lazy wbfs")
    d, p, st = og.wbfs(dwg, s, og.Schedule(update=LAZY))
    torch.cuda.synchronize()
    check_sssp(orc, wg, s, d, p, "lazy wbfs")
    rng = np.random.default_rng(15)
    for i in range(4):
        s, t = int(srcs[i]), int(rng.integers(0, g.n))
        want = orc.ppsp(g, s, t)
        say(f"lazy ppsp/astar s={s} t={t}")
        dist, _, _ = og.ppsp(dg, s, t, og.Schedule(delta=256, update=LAZY))
        h = torch.from_numpy(gg.grid_heuristic(256, t)).to(DEV)
        dista, _, _ = og.astar(dg, s, t, h, og.Schedule(delta=128, update=LAZY))
        torch.cuda.synchronize()
        exp = og.INF if want < 0 else want
        assert int(dist[t]) == exp and int(dista[t]) == exp


MODES = [LAZY, og.OG_EAGER_NO_FUSION, og.OG_EAGER_WITH_FUSION]


def run_kcore(dg, **kw):
    core, st = og.kcore(dg, og.Schedule(**kw))
    torch.cuda.synchronize()
    return core.cpu().numpy(), st


@pytest.mark.parametrize("engine", [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS])
@pytest.mark.parametrize("update", MODES)
@pytest.mark.parametrize("kind", ["grid", "road", "rmat"])
def test_kcore_parity(orc, graphs, kind, update, engine):
    g, _ = graphs[kind]
    dg = og.DeviceGraph.from_host(g, DEV, weights=False)
    tag = f"kcore {kind} update={update} engine={engine}"
    say(tag)
    core, st = run_kcore(dg, update=update, engine=engine)
    assert st["status"] == 0
    want = orc.kcore(g)
    assert np.array_equal(core, want), f"{tag}: {int(np.count_nonzero(core != want))} differ"
    assert st["reached_vertices"] == g.n and st["reached_edges"] == g.m
    if update == LAZY:
        assert st["barriers"] == 2 * st["rounds"]


@pytest.mark.parametrize("window", [2, 64])
@pytest.mark.parametrize("update", MODES)
def test_kcore_windows(orc, graphs, window, update):
    g, _ = graphs["rmat"]
    dg = og.DeviceGraph.from_host(g, DEV, weights=False)
    say(f"kcore rmat window={window} update={update}")
    core, st = run_kcore(dg, update=update, window_buckets=window)
    assert np.array_equal(core, orc.kcore(g))
    if window == 2:
        assert st["far_pushes"] > 0


def test_kcore_small_graphs(orc):
    rng = np.random.default_rng(16)
    cases = [
        undirected(1, []),
        undirected(5, []),
        undirected(2, [(0, 1)]),
        undirected(40, [(a, b) for a in range(40) for b in range(a + 1, 40)]),
        undirected(12, [(i, (i + 1) % 12) for i in range(12)]),
        undirected(9, [(0, i) for i in range(1, 9)]),
    ]
    clique_path = [(a, b) for a in range(6) for b in range(a + 1, 6)] + [(5 + i, 6 + i) for i in range(20)]
    cases.append(undirected(26, clique_path))
    for _ in range(20):
        n = int(rng.integers(2, 200))
        p = float(rng.uniform(0.01, 0.3))
        cases.append(undirected(n, [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]))
    for i, g in enumerate(cases):
        dg = og.DeviceGraph.from_host(g, DEV, weights=False)
        want = orc.kcore(g)
        for update in MODES:
            say(f"kcore small case {i} n={g.n} m={g.m} update={update}")
            core, st = run_kcore(dg, update=update, fusion_threshold=int(rng.choice([1, 64, 1024])))
            assert np.array_equal(core, want), (i, update)


def test_kcore_round_limit_and_queue_errors(graphs):
    g, _ = graphs["rmat"]
    dg = og.DeviceGraph.from_host(g, DEV, weights=False)
    say("kcore max_rounds=1")
    core, st = og.kcore(dg, og.Schedule(update=LAZY, max_rounds=1), check=False)
    torch.cuda.synchronize()
    assert st["status"] == og.OG_ERR_ROUND_LIMIT
    say("kcore queue_capacity below n")
    core, st = og.kcore(dg, og.Schedule(update=og.OG_EAGER_NO_FUSION, queue_capacity=64), check=False)
    torch.cuda.synchronize()
    assert st["status"] in (0, og.OG_ERR_WORKSPACE)


@pytest.mark.slow
@pytest.mark.parametrize("update", MODES)
def test_kcore_rmat20(orc, update):
    g = gg.rmat(20, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV, weights=False)
    say(f"kcore rmat20 update={update}")
    core, st = run_kcore(dg, update=update, window_buckets=64)
    assert st["status"] == 0
    assert np.array_equal(core, orc.kcore(g))


@pytest.mark.slow
def test_lazy_road_full_size(orc):
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=1)[0])
    say(f"lazy road4096 src={src} delta=1024")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=1024, update=LAZY))
    torch.cuda.synchronize()
    check_sssp(orc, g, src, d, p, "lazy road4096")
