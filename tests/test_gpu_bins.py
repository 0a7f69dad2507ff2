"""GPU parity of degree-binned load balancing (OG_FLAG_DEGREE_BINS) through
the C ABI, against the CPU oracle.

The bins only change which lanes relax which edges (one lane per small
vertex, one wavefront per medium vertex, the whole workgroup for the rest),
so distances and canonical predecessors must equal the oracle's Dijkstra bit
for bit for every cut-off, update strategy, engine and query shape.
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
BINS = og.OG_FLAG_DEGREE_BINS
UPDATES = [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION, og.OG_LAZY_UPDATE]
ENGINES = [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


@pytest.mark.parametrize("update", UPDATES)
@pytest.mark.parametrize("kind,delta", [("grid", 1), ("grid", 16), ("grid", 1 << 20), ("road", 256), ("road", 4096),
                                        ("rmat", 8), ("rmat", 64)])
def test_bins_sssp(orc, graphs, kind, delta, update):
    g, dg = graphs[kind]
    for src in gg.pick_sources(g, 2, seed=31):
        tag = f"bins sssp {kind} src={src} delta={delta} update={update}"
        say(tag)
        d, p, st = og.sssp(dg, int(src), og.Schedule(delta=delta, update=update, flags=BINS))
        torch.cuda.synchronize()
        assert st["status"] == 0
        check_sssp(orc, g, int(src), d, p, tag)


@pytest.mark.parametrize("cuts", [(1, 0), (1, 1), (2, 8), (3, 64), (4, 4), (4, 1000), (4, 1 << 30), (9, 64)])
@pytest.mark.parametrize("kind", ["road", "rmat"])
def test_bins_cutoffs(orc, graphs, kind, cuts):
    """Every split of the degrees between the bins (the lane bin alone, the
    wavefront bin taking everything, lane cut-off above its cap of 4)."""
    g, dg = graphs[kind]
    bt, bw = cuts
    for update in (og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION):
        src = int(gg.pick_sources(g, 1, seed=32)[0])
        tag = f"bins cut-offs {kind} thread={bt} wave={bw} update={update}"
        say(tag)
        d, p, st = og.sssp(dg, src, og.Schedule(delta=64 if kind == "rmat" else 512, update=update, flags=BINS,
                                                bin_thread=bt, bin_wave=bw))
        torch.cuda.synchronize()
        check_sssp(orc, g, src, d, p, tag)


@pytest.mark.parametrize("engine", ENGINES)
def test_bins_engines_and_thresholds(orc, graphs, engine):
    g, dg = graphs["road"]
    src = int(gg.pick_sources(g, 1, seed=33)[0])
    for thr in (1, 64, 1024):
        tag = f"bins engine={engine} threshold={thr}"
        say(tag)
        d, p, st = og.sssp(dg, src, og.Schedule(delta=512, engine=engine, fusion_threshold=thr, flags=BINS))
        torch.cuda.synchronize()
        check_sssp(orc, g, src, d, p, tag)
    say(f"bins engine={engine} K=2 far")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=16, engine=engine, window_buckets=2, flags=BINS))
    torch.cuda.synchronize()
    assert st["far_pushes"] > 0
    check_sssp(orc, g, src, d, p, "bins far")


def test_bins_batch_multi_wbfs_ppsp_astar(orc, graphs):
    g, dg = graphs["road"]
    srcs = gg.pick_sources(g, 8, seed=34)
    say("bins sssp_batch x8")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=512, flags=BINS))
    torch.cuda.synchronize()
    for q, s in enumerate(srcs):
        check_sssp(orc, g, int(s), d[q], p[q], f"bins batch q={q}")
    say("bins sssp_multi x4")
    dm, pm, st = og.sssp_multi(dg, srcs[:4], og.Schedule(delta=512, flags=BINS))
    torch.cuda.synchronize()
    ref = np.min(np.stack([orc.sssp(g, int(s))[0] for s in srcs[:4]]), axis=0)
    assert np.array_equal(dm.cpu().numpy(), ref)
    rg, _ = graphs["rmat"]
    wg = gg.with_weights(rg, rg.w % 13 + 1)
    dwg = og.DeviceGraph.from_host(wg, DEV)
    s = int(gg.pick_sources(wg, 1, seed=35)[0])
    for update in UPDATES:
        say(f"bins wbfs update={update}")
        d, p, st = og.wbfs(dwg, s, og.Schedule(update=update, flags=BINS))
        torch.cuda.synchronize()
        check_sssp(orc, wg, s, d, p, "bins wbfs")
    rng = np.random.default_rng(36)
    ts = rng.integers(0, g.n, size=8)
    for i in range(4):
        s, t = int(srcs[i]), int(ts[i])
        want = orc.ppsp(g, s, t)
        say(f"bins ppsp/astar s={s} t={t}")
        dist, _, _ = og.ppsp(dg, s, t, og.Schedule(delta=256, flags=BINS))
        h = torch.from_numpy(gg.grid_heuristic(256, t)).to(DEV)
        dista, _, _ = og.astar(dg, s, t, h, og.Schedule(delta=128, flags=BINS))
        torch.cuda.synchronize()
        exp = og.INF if want < 0 else want
        assert int(dist[t]) == exp and int(dista[t]) == exp
    say("bins astar_batch x8")
    hb = gg.grid_heuristic_device(256, ts, device=DEV)
    db, _, _ = og.astar_batch(dg, srcs, ts, hb, og.Schedule(delta=128, flags=BINS))
    torch.cuda.synchronize()
    for q in range(8):
        want = orc.ppsp(g, int(srcs[q]), int(ts[q]))
        assert int(db[q][int(ts[q])]) == (og.INF if want < 0 else want)


def test_bins_small_graphs(orc):
    """One vertex, no edges, zero weights, a star (a row in the workgroup
    bin), a path, rows of 5..70 edges (the wavefront bin)."""
    rng = np.random.default_rng(37)

    def undirected(n, pairs, w):
        src = [a for a, b in pairs] + [b for a, b in pairs]
        dst = [b for a, b in pairs] + [a for a, b in pairs]
        return gg.from_edges(n, src, dst, np.asarray(list(w) + list(w), dtype=np.int64))

    cases = [
        undirected(1, [], []),
        undirected(5, [], []),
        undirected(2, [(0, 1)], [0]),
        undirected(300, [(0, i) for i in range(1, 300)], rng.integers(1, 50, 299)),
        undirected(200, [(i, i + 1) for i in range(199)], rng.integers(1, 9, 199)),
    ]
    for _ in range(10):
        n = int(rng.integers(2, 160))
        pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < float(rng.uniform(0.02, 0.5))]
        cases.append(undirected(n, pairs, rng.integers(0, 30, len(pairs))))
    for i, g in enumerate(cases):
        dg = og.DeviceGraph.from_host(g, DEV)
        ref_d, ref_p = orc.sssp(g, 0)
        for update in UPDATES:
            for delta in (1, 7, 1 << 20):
                say(f"bins small case {i} n={g.n} m={g.m} update={update} delta={delta}")
                d, p, st = og.sssp(dg, 0, og.Schedule(delta=delta, update=update, flags=BINS, bin_wave=16))
                torch.cuda.synchronize()
                assert np.array_equal(d.cpu().numpy(), ref_d), (i, update, delta)
                if (g.w > 0).all():
                    assert np.array_equal(p.cpu().numpy(), ref_p), (i, update, delta)


@pytest.mark.slow
def test_bins_full_size(orc):
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=1)[0])
    say(f"bins road4096 src={src} delta=512")
    d, p, st = og.sssp(dg, src, og.Schedule(delta=512, flags=BINS))
    torch.cuda.synchronize()
    check_sssp(orc, g, src, d, p, "bins road4096")
    del dg
    g = gg.rmat(20, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    for update in (og.OG_EAGER_NO_FUSION, og.OG_EAGER_WITH_FUSION):
        say(f"bins rmat20 src={src} delta=32 update={update}")
        d, p, st = og.sssp(dg, src, og.Schedule(delta=32, update=update, flags=BINS))
        torch.cuda.synchronize()
        check_sssp(orc, g, src, d, p, "bins rmat20")
