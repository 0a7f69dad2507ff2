"""GPU parity of the pull traversal direction (section 4.2, DensePull and the
SparsePush-DensePull hybrid, combined with lazy bucket updates as in section
5.1) through the C ABI, against the CPU oracle.

A pull round changes how a round's relaxations are carried out (each vertex
gathers from the frontier marked in a dense array, with no atomic on the
destination) but not the fixed point: distances (and canonical
predecessors) must equal the oracle's Dijkstra bit for bit, and coreness the
oracle's peeling result, for every engine, Delta and query shape.  With
OG_FLAG_DENSE_PULL every round pulls, which the barrier count shows (three
device-wide barriers per round).
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
PULL = og.OG_FLAG_DENSE_PULL
HYBRID = og.OG_FLAG_HYBRID_DIRECTION
ENGINES = [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def undirected(n, pairs, w=None):
    src = [a for a, b in pairs] + [b for a, b in pairs]
    dst = [b for a, b in pairs] + [a for a, b in pairs]
    ww = list(w) + list(w) if w is not None else [1] * len(src)
    return gg.from_edges(n, src, dst, np.asarray(ww, dtype=np.int64))


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


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("flag", [PULL, HYBRID])
@pytest.mark.parametrize("kind,delta", [("grid", 1), ("grid", 16), ("grid", 1 << 20), ("road", 256), ("road", 4096),
                                        ("rmat", 8), ("rmat", 64), ("rmat", 1 << 20)])
def test_pull_sssp(orc, graphs, kind, delta, flag, engine):
    g, dg = graphs[kind]
    for src in gg.pick_sources(g, 2, seed=21):
        tag = f"pull sssp {kind} src={src} delta={delta} flag={flag} engine={engine}"
        say(tag)
        d, p, st = og.sssp(dg, int(src), og.Schedule(delta=delta, update=LAZY, engine=engine, flags=flag))
        torch.cuda.synchronize()
        assert st["status"] == 0
        check_sssp(orc, g, int(src), d, p, tag)
        assert st["pushes_local"] == 0
        if flag == PULL:
            assert st["barriers"] == 3 * st["rounds"], tag
        else:
            assert 2 * st["rounds"] <= st["barriers"] <= 3 * st["rounds"], tag


def test_hybrid_switches_direction(orc, graphs):
    """One bucket holding the whole graph: the frontier passes n/20 entries
    after a few rounds, so the hybrid pulls some rounds and pushes others."""
    g, dg = graphs["rmat"]
    src = int(gg.pick_sources(g, 1, seed=22)[0])
    say(f"hybrid rmat single bucket src={src}")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=1 << 24, update=LAZY, flags=HYBRID))
    torch.cuda.synchronize()
    check_sssp(orc, g, src, d, p, "hybrid single bucket")
    pulls = st["barriers"] - 2 * st["rounds"]
    assert 0 < pulls < st["rounds"], st


def test_pull_small_window_far_and_thresholds(orc, graphs):
    g, dg = graphs["road"]
    src = int(gg.pick_sources(g, 1, seed=23)[0])
    for flag in (PULL, HYBRID):
        say(f"pull K=2 delta=16 flag={flag}")
        d, p, st = og.sssp(dg, src, og.Schedule(delta=16, update=LAZY, window_buckets=2, flags=flag))
        torch.cuda.synchronize()
        assert st["far_pushes"] > 0
        check_sssp(orc, g, src, d, p, f"pull far flag={flag}")
        say(f"pull workgroups=3 flag={flag}")
        d, p, st = og.sssp(dg, src, og.Schedule(delta=512, update=LAZY, workgroups=3, flags=flag))
        torch.cuda.synchronize()
        check_sssp(orc, g, src, d, p, f"pull 3 workgroups flag={flag}")


@pytest.mark.parametrize("flag", [PULL, HYBRID])
def test_pull_batch_multi_wbfs_ppsp_astar(orc, graphs, flag):
    g, dg = graphs["road"]
    srcs = gg.pick_sources(g, 8, seed=24)
    say(f"pull sssp_batch x8 flag={flag}")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=512, update=LAZY, flags=flag))
    torch.cuda.synchronize()
    for q, s in enumerate(srcs):
        check_sssp(orc, g, int(s), d[q], p[q], f"pull batch q={q}")
    say(f"pull sssp_multi x4 flag={flag}")
    dm, pm, st = og.sssp_multi(dg, srcs[:4], og.Schedule(delta=512, update=LAZY, flags=flag))
    torch.cuda.synchronize()
    ref = np.min(np.stack([orc.sssp(g, int(s))[0] for s in srcs[:4]]), axis=0)
    assert np.array_equal(dm.cpu().numpy(), ref)
    rg, _ = graphs["rmat"]
    wg = gg.with_weights(rg, rg.w % 13 + 1)
    dwg = og.DeviceGraph.from_host(wg, DEV)
    s = int(gg.pick_sources(wg, 1, seed=25)[0])
    say(f"pull wbfs flag={flag}")
    d, p, st = og.wbfs(dwg, s, og.Schedule(update=LAZY, flags=flag))
    torch.cuda.synchronize()
    check_sssp(orc, wg, s, d, p, "pull wbfs")
    rng = np.random.default_rng(26)
    for i in range(4):
        s, t = int(srcs[i]), int(rng.integers(0, g.n))
        want = orc.ppsp(g, s, t)
        say(f"pull ppsp/astar s={s} t={t} flag={flag}")
        dist, _, _ = og.ppsp(dg, s, t, og.Schedule(delta=256, update=LAZY, flags=flag))
        h = torch.from_numpy(gg.grid_heuristic(256, t)).to(DEV)
        dista, _, _ = og.astar(dg, s, t, h, og.Schedule(delta=128, update=LAZY, flags=flag))
        torch.cuda.synchronize()
        exp = og.INF if want < 0 else want
        assert int(dist[t]) == exp and int(dista[t]) == exp
    ts = rng.integers(0, g.n, size=8)
    say(f"pull ppsp_batch x8 flag={flag}")
    db, _, _ = og.ppsp_batch(dg, srcs, ts, og.Schedule(delta=256, update=LAZY, flags=flag))
    torch.cuda.synchronize()
    for q in range(8):
        want = orc.ppsp(g, int(srcs[q]), int(ts[q]))
        assert int(db[q][int(ts[q])]) == (og.INF if want < 0 else want)


def test_pull_small_graphs(orc):
    """Edge cases: one vertex, no edges, zero weights, a disconnected pair,
    a star (one long row), a path (one vertex per round)."""
    rng = np.random.default_rng(27)
    cases = [
        undirected(1, []),
        undirected(5, []),
        undirected(2, [(0, 1)], [0]),
        undirected(4, [(0, 1), (2, 3)], [5, 7]),
        undirected(300, [(0, i) for i in range(1, 300)], list(rng.integers(0, 50, 299))),
        undirected(200, [(i, i + 1) for i in range(199)], list(rng.integers(1, 9, 199))),
    ]
    for _ in range(12):
        n = int(rng.integers(2, 150))
        pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < 0.05]
        cases.append(undirected(n, pairs, list(rng.integers(0, 30, len(pairs)))))
    for i, g in enumerate(cases):
        dg = og.DeviceGraph.from_host(g, DEV)
        for flag in (PULL, HYBRID):
            for delta in (1, 7, 1 << 20):
                say(f"pull small case {i} n={g.n} m={g.m} flag={flag} delta={delta}")
                d, p, st = og.sssp(dg, 0, og.Schedule(delta=delta, update=LAZY, flags=flag))
                torch.cuda.synchronize()
                ref_d, ref_p = orc.sssp(g, 0)
                assert np.array_equal(d.cpu().numpy(), ref_d), (i, flag, delta)
                # zero weights: only the distances are unique
                if (g.w > 0).all():
                    assert np.array_equal(p.cpu().numpy(), ref_p), (i, flag, delta)


def test_pull_validation_rejects_asymmetric_graph(graphs):
    g, dg = graphs["grid"]
    sched = og.Schedule(delta=16, update=LAZY, flags=PULL | og.OG_FLAG_VALIDATE)
    say("pull validate symmetric grid")
    d, p, st = og.sssp(dg, 0, sched)
    torch.cuda.synchronize()
    assert st["status"] == 0
    # one weight changed on one direction only
    w = g.w.copy()
    w[5] += 1
    bad = gg.with_weights(g, w)
    dbad = og.DeviceGraph.from_host(bad, DEV)
    say("pull validate asymmetric weights")
    d, p, st = og.sssp(dbad, 0, sched, check=False)
    torch.cuda.synchronize()
    assert st["status"] == og.OG_ERR_INVALID_ARG
    # one edge without its reverse
    one_way = gg.from_edges(3, [0, 1, 1], [1, 0, 2], [1, 1, 1])
    say("pull validate one-way edge")
    for flag in (PULL, HYBRID):
        d, p, st = og.sssp(og.DeviceGraph.from_host(one_way, DEV), 0,
                           og.Schedule(update=LAZY, flags=flag | og.OG_FLAG_VALIDATE), check=False)
        torch.cuda.synchronize()
        assert st["status"] == og.OG_ERR_INVALID_ARG
        core, st = og.kcore(og.DeviceGraph.from_host(one_way, DEV, weights=False),
                            og.Schedule(update=LAZY, flags=flag | og.OG_FLAG_VALIDATE), check=False)
        torch.cuda.synchronize()
        assert st["status"] == og.OG_ERR_INVALID_ARG


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("flag", [PULL, HYBRID])
@pytest.mark.parametrize("kind", ["grid", "road", "rmat"])
def test_pull_kcore(orc, graphs, kind, flag, engine):
    g, _ = graphs[kind]
    dg = og.DeviceGraph.from_host(g, DEV, weights=False)
    tag = f"pull kcore {kind} flag={flag} engine={engine}"
    say(tag)
    core, st = og.kcore(dg, og.Schedule(update=LAZY, engine=engine, flags=flag))
    torch.cuda.synchronize()
    assert st["status"] == 0
    want = orc.kcore(g)
    core = core.cpu().numpy()
    assert np.array_equal(core, want), f"{tag}: {int(np.count_nonzero(core != want))} differ"
    if flag == PULL:
        assert st["barriers"] == 3 * st["rounds"]


def test_pull_kcore_small_graphs_and_windows(orc, graphs):
    rng = np.random.default_rng(28)
    cases = [
        undirected(1, []),
        undirected(5, []),
        undirected(2, [(0, 1)]),
        undirected(40, [(a, b) for a in range(40) for b in range(a + 1, 40)]),
        undirected(12, [(i, (i + 1) % 12) for i in range(12)]),
        undirected(9, [(0, i) for i in range(1, 9)]),
    ]
    for _ in range(12):
        n = int(rng.integers(2, 200))
        p = float(rng.uniform(0.01, 0.3))
        cases.append(undirected(n, [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]))
    for i, g in enumerate(cases):
        dg = og.DeviceGraph.from_host(g, DEV, weights=False)
        want = orc.kcore(g)
        for flag in (PULL, HYBRID):
            say(f"pull kcore small case {i} n={g.n} m={g.m} flag={flag}")
            core, st = og.kcore(dg, og.Schedule(update=LAZY, flags=flag))
            torch.cuda.synchronize()
            assert np.array_equal(core.cpu().numpy(), want), (i, flag)
    g, _ = graphs["rmat"]
    dg = og.DeviceGraph.from_host(g, DEV, weights=False)
    for window in (2, 64):
        say(f"pull kcore rmat window={window}")
        core, st = og.kcore(dg, og.Schedule(update=LAZY, window_buckets=window, flags=PULL))
        torch.cuda.synchronize()
        assert np.array_equal(core.cpu().numpy(), orc.kcore(g))


@pytest.mark.slow
@pytest.mark.parametrize("flag", [PULL, HYBRID])
def test_pull_rmat20(orc, flag):
    g = gg.rmat(20, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=29)[0])
    say(f"pull rmat20 sssp flag={flag}")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=32, update=LAZY, flags=flag))
    torch.cuda.synchronize()
    check_sssp(orc, g, src, d, p, "pull rmat20")
    dk = og.DeviceGraph.from_host(g, DEV, weights=False)
    say(f"pull rmat20 kcore flag={flag}")
    core, st = og.kcore(dk, og.Schedule(update=LAZY, window_buckets=64, flags=flag))
    torch.cuda.synchronize()
    assert np.array_equal(core.cpu().numpy(), orc.kcore(g))
