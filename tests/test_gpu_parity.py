"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Distances and canonical predecessors are integers and must match bit for
bit.  Every Delta, fused / unfused update, engine, fusion threshold, window
size and queue capacity must give the same (unique) answer: any
schedule-dependent output is a bug.
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu

INF = og.INF
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cfg0():
    g = gg.grid(64, 64, 1, 100, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.fixture(scope="module")
def road256():
    g = gg.road(256, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.fixture(scope="module")
def rmat14():
    g = gg.rmat(14, 16, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


def run_sssp(dg, src, sched, fn="sssp", **kw):
    f = getattr(og, fn)
    d, p, st = f(dg, src, sched, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), (p.cpu().numpy() if p is not None else None), st


def assert_exact(orc, g, src, d, p, tag=""):
    ref_d, ref_p = orc.sssp(g, src)
    nd = int(np.count_nonzero(d != ref_d))
    assert nd == 0, f"{tag}: {nd} distances differ (first at {np.nonzero(d != ref_d)[0][:5]})"
    if p is not None:
        np_ = int(np.count_nonzero(p != ref_p))
        assert np_ == 0, f"{tag}: {np_} predecessors differ"


@pytest.mark.parametrize("engine", [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS])
@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
@pytest.mark.parametrize("delta", [1, 3, 16, 100, 1024, 1 << 20])
def test_cfg0_all_schedules(orc, cfg0, engine, update, delta):
    g, dg = cfg0
    tag = f"cfg0 engine={engine} update={update} delta={delta}"
    say(tag)
    d, p, st = run_sssp(dg, 0, og.Schedule(delta=delta, update=update, engine=engine))
    assert st["status"] == 0
    assert_exact(orc, g, 0, d, p, tag)
    assert st["reached_vertices"] == g.n and st["reached_edges"] == g.m
    if update == og.OG_EAGER_NO_FUSION:
        assert st["pushes_local"] == 0


@pytest.mark.parametrize("threshold", [1, 2, 64, 2048])
@pytest.mark.parametrize("workgroups", [1, 3, 0])
def test_cfg0_thresholds_and_grid(orc, cfg0, threshold, workgroups):
    g, dg = cfg0
    tag = f"cfg0 threshold={threshold} wg={workgroups}"
    say(tag)
    d, p, st = run_sssp(dg, 4095, og.Schedule(delta=16, fusion_threshold=threshold, workgroups=workgroups))
    assert st["status"] == 0
    assert_exact(orc, g, 4095, d, p, tag)


def test_cfg0_repeatable(orc, cfg0):
    g, dg = cfg0
    say("cfg0 repeat x20")
    ref = None
    for i in range(20):
        d, p, st = run_sssp(dg, 1234, og.Schedule(delta=16))
        if ref is None:
            ref = (d, p)
            assert_exact(orc, g, 1234, d, p, "repeat")
        assert np.array_equal(d, ref[0]) and np.array_equal(p, ref[1])


@pytest.mark.parametrize("delta", [256, 4096, 1 << 14])
@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
def test_road_small(orc, road256, delta, update):
    g, dg = road256
    for src in gg.pick_sources(g, 3, seed=1):
        tag = f"road256 src={src} delta={delta} update={update}"
        say(tag)
        d, p, st = run_sssp(dg, int(src), og.Schedule(delta=delta, update=update))
        assert st["status"] == 0
        assert_exact(orc, g, int(src), d, p, tag)


@pytest.mark.parametrize("delta", [1, 8, 64, 700])
def test_rmat_small(orc, rmat14, delta):
    g, dg = rmat14
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    tag = f"rmat14 src={src} delta={delta}"
    say(tag)
    d, p, st = run_sssp(dg, src, og.Schedule(delta=delta))
    assert st["status"] == 0
    assert_exact(orc, g, src, d, p, tag)


def test_wbfs_rmat(orc, rmat14):
    g, _ = rmat14
    rng = np.random.default_rng(5)
    wg = gg.with_weights(g, g.w % 13 + 1)  # weights in [1, log2 n) for n = 2^14
    dg = og.DeviceGraph.from_host(wg, DEV)
    src = int(gg.pick_sources(g, 1, seed=3)[0])
    say(f"wbfs rmat14 src={src}")
    d, p, st = run_sssp(dg, src, og.Schedule(delta=64), fn="wbfs")
    assert st["status"] == 0
    assert_exact(orc, wg, src, d, p, "wbfs")


def test_small_window_uses_far_queue(orc, road256):
    g, dg = road256
    src = int(gg.pick_sources(g, 1, seed=4)[0])
    say("far queue K=2 delta=16")
    d, p, st = run_sssp(dg, src, og.Schedule(delta=16, window_buckets=2))
    assert st["status"] == 0 and st["far_pushes"] > 0
    assert_exact(orc, g, src, d, p, "far")


def test_small_queues_fall_back_to_far(orc, road256):
    g, dg = road256
    src = int(gg.pick_sources(g, 1, seed=5)[0])
    say("queue_capacity 6000 (window/spill overflow -> far)")
    d, p, st = run_sssp(dg, src, og.Schedule(delta=1 << 14, queue_capacity=6000, update=og.OG_EAGER_NO_FUSION,
                                             fusion_threshold=1))
    if st["status"] == 0:
        assert_exact(orc, g, src, d, p, "smallq")
    else:
        assert st["status"] == og.OG_ERR_WORKSPACE


def test_pred_pass_with_and_without_queue_room(orc):
    """The predecessor pass keeps its long-row slice list and parity summary
    where the queues were; with queues too small for them every row stays in
    its chunk and every dist read is made.  A weighted path with four hubs
    joined to every path vertex (rows of 2,000 edges, mean degree 10) gives
    the same canonical predecessors both ways."""
    L, H = 2000, 4
    src, dst, w = [], [], []
    for i in range(L - 1):
        src += [i, i + 1]
        dst += [i + 1, i]
        w += [1 + i % 3] * 2
    for h in range(L, L + H):
        for i in range(L):
            src += [h, i]
            dst += [i, h]
            w += [1_000_000 + i % 7] * 2
    g = gg.from_edges(L + H, src, dst, w)
    assert g.m >= 8 * g.n and np.diff(g.row_ptr).max() > 1024
    dg = og.DeviceGraph.from_host(g, DEV)
    for cap in (0, 8):  # 0: the default capacity
        say(f"pred pass, path with hubs, queue_capacity={cap}")
        d, p, st = run_sssp(dg, 0, og.Schedule(delta=64, window_buckets=2, queue_capacity=cap))
        assert st["status"] == 0, st["status"]
        assert_exact(orc, g, 0, d, p, f"hubs cap={cap}")


def test_queue_overflow_is_reported(road256):
    g, dg = road256
    say("queue_capacity 1024 on road256 delta=2^20 unfused -> workspace error")
    d, p, st = run_sssp(dg, 0, og.Schedule(delta=1 << 20, queue_capacity=1024, update=og.OG_EAGER_NO_FUSION),
                        check=False)
    assert st["status"] == og.OG_ERR_WORKSPACE
    assert st["queue_needed"] > 1024


def test_round_limit(cfg0):
    _, dg = cfg0
    for engine in (og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS):
        say(f"max_rounds=1 engine={engine}")
        d, p, st = run_sssp(dg, 0, og.Schedule(delta=16, max_rounds=1, engine=engine), check=False)
        assert st["status"] == og.OG_ERR_ROUND_LIMIT and st["rounds"] == 1


def test_overflow_detected():
    g = gg.from_edges(4, [0, 1, 2], [1, 2, 3], [2**30, 2**30, 5])
    dg = og.DeviceGraph.from_host(g, DEV)
    say("int32 overflow path")
    d, p, st = run_sssp(dg, 0, og.Schedule(delta=1 << 20), check=False)
    assert st["status"] == og.OG_ERR_OVERFLOW


def test_negative_weight_reported():
    g = gg.from_edges(3, [0, 1], [1, 2], [4, -1])
    dg = og.DeviceGraph.from_host(g, DEV)
    for flags in (0, og.OG_FLAG_VALIDATE):
        say(f"negative weight flags={flags}")
        d, p, st = run_sssp(dg, 0, og.Schedule(delta=2, flags=flags), check=False)
        assert st["status"] == og.OG_ERR_NEGATIVE_WEIGHT


def test_validate_rejects_malformed_graphs(orc, cfg0):
    """OG_FLAG_VALIDATE checks the CSR structure before anything reads it:
    a column index outside [0, n), a decreasing row_ptr or row_ptr[n] != m
    is OG_ERR_INVALID_ARG, with the outputs untouched; a valid graph runs."""
    say("validate malformed graphs")
    rp = torch.tensor([0, 2, 3, 4], dtype=torch.int64, device=DEV)
    col = torch.tensor([1, 2, 2, 0], dtype=torch.int32, device=DEV)
    w = torch.tensor([1, 4, 1, 3], dtype=torch.int32, device=DEV)
    V = og.OG_FLAG_VALIDATE
    d, p, st = og.sssp(og.DeviceGraph(rp, col, w), 0, og.Schedule(delta=2, flags=V))
    torch.cuda.synchronize()
    assert st["status"] == 0 and d.cpu().tolist() == [0, 1, 2]
    cases = {
        "column out of range": (rp, torch.tensor([1, 3, 2, 0], dtype=torch.int32, device=DEV)),
        "negative column": (rp, torch.tensor([1, -1, 2, 0], dtype=torch.int32, device=DEV)),
        "decreasing row_ptr": (torch.tensor([0, 3, 2, 4], dtype=torch.int64, device=DEV), col),
        "row_ptr[0] != 0": (torch.tensor([1, 2, 3, 4], dtype=torch.int64, device=DEV), col),
        "row_ptr[n] != m": (torch.tensor([0, 2, 3, 3], dtype=torch.int64, device=DEV), col),
    }
    for name, (rp_bad, col_bad) in cases.items():
        say(f"validate: {name}")
        dg = og.DeviceGraph(rp_bad, col_bad, w)
        out = torch.full((3,), -7, dtype=torch.int32, device=DEV)
        d, p, st = og.sssp(dg, 0, og.Schedule(delta=2, flags=V), check=False, out_dist=out)
        torch.cuda.synchronize()
        assert st["status"] == og.OG_ERR_INVALID_ARG, name
        core, st = og.kcore(og.DeviceGraph(rp_bad, col_bad, None), og.Schedule(update=og.OG_LAZY_UPDATE, flags=V),
                            check=False)
        torch.cuda.synchronize()
        assert st["status"] == og.OG_ERR_INVALID_ARG, name
    wf = torch.tensor([1.0, -2.0, 1.0, 3.0], dtype=torch.float32, device=DEV)
    say("validate: negative float32 weight")
    _, _, _, st = og.sssp_f32(og.DeviceGraph(rp, col, w), wf, 0, og.Schedule(delta=2, flags=V), check=False)
    torch.cuda.synchronize()
    assert st["status"] == og.OG_ERR_NEGATIVE_WEIGHT


def test_tiny_graphs(orc):
    say("tiny graphs")
    cases = [
        gg.from_edges(1, [], [], []),
        gg.from_edges(2, [], [], []),
        gg.from_edges(3, [0, 0, 1], [1, 2, 2], [5, 1, 0]),
        gg.from_edges(5, [0, 1, 3], [1, 0, 4], [0, 0, 7]),
    ]
    for g in cases:
        dg = og.DeviceGraph.from_host(g, DEV)
        for src in range(g.n):
            for delta in (1, 2, 1000):
                d, p, st = run_sssp(dg, src, og.Schedule(delta=delta))
                ref_d, _ = orc.sssp(g, src)
                assert np.array_equal(d, ref_d)
                assert orc.check(g, src, d, p) == 0


def test_random_graphs_with_zero_weights(orc):
    rng = np.random.default_rng(9)
    say("random small graphs, weights 0..3")
    for trial in range(30):
        n = int(rng.integers(2, 300))
        m = int(rng.integers(0, 4 * n))
        g = gg.from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m), rng.integers(0, 4, m))
        dg = og.DeviceGraph.from_host(g, DEV)
        src = int(rng.integers(0, n))
        delta = int(rng.choice([1, 2, 5, 64]))
        d, p, st = run_sssp(dg, src, og.Schedule(delta=delta, fusion_threshold=int(rng.choice([1, 8, 1024]))))
        ref_d, _ = orc.sssp(g, src)
        assert np.array_equal(d, ref_d), trial
        # zero-weight ties: canonical pred is a valid certificate only when it
        # has no zero-weight cycles; check tightness bits (7) at least
        assert orc.check(g, src, d, None) == 0


def walk_path(g, s, t, pred):
    v, total, steps = t, 0, 0
    while v != s:
        u = int(pred[v])
        assert u >= 0, "path broken"
        row = slice(g.row_ptr[u], g.row_ptr[u + 1])
        idx = np.nonzero(g.col[row] == v)[0]
        assert len(idx) == 1, "pred edge missing"
        total += int(g.w[row][idx[0]])
        v = u
        steps += 1
        assert steps <= g.n
    return total


@pytest.mark.parametrize("delta", [64, 1024])
def test_ppsp(orc, road256, delta):
    g, dg = road256
    rng = np.random.default_rng(delta)
    srcs = gg.pick_sources(g, 6, seed=6)
    for i in range(6):
        s = int(srcs[i])
        t = int(rng.integers(0, g.n))
        say(f"ppsp s={s} t={t} delta={delta}")
        dist, pred, st = og.ppsp(dg, s, t, og.Schedule(delta=delta))
        torch.cuda.synchronize()
        dist = dist.cpu().numpy()
        pred = pred.cpu().numpy()
        want = orc.ppsp(g, s, t)
        if want < 0:
            assert dist[t] == INF
        else:
            assert dist[t] == want
            assert walk_path(g, s, t, pred) == want


def test_astar(orc, road256):
    g, dg = road256
    rng = np.random.default_rng(77)
    srcs = gg.pick_sources(g, 6, seed=7)
    for i in range(6):
        s = int(srcs[i])
        t = int(rng.integers(0, g.n))
        want = orc.ppsp(g, s, t)
        for hname in ("zero", "euclid"):
            h = np.zeros(g.n, dtype=np.int32) if hname == "zero" else gg.grid_heuristic(256, t)
            say(f"astar s={s} t={t} h={hname}")
            dist, pred, st = og.astar(dg, s, t, torch.from_numpy(h).to(DEV), og.Schedule(delta=128))
            torch.cuda.synchronize()
            dist = dist.cpu().numpy()
            pred = pred.cpu().numpy()
            if want < 0:
                assert dist[t] == INF
            else:
                assert dist[t] == want, (hname, dist[t], want)
                assert walk_path(g, s, t, pred) == want


def test_async_flag_and_read_stats(orc, cfg0):
    g, dg = cfg0
    say("async + og_read_stats")
    ws = og.Workspace(DEV)
    d, p, st = og.sssp(dg, 7, og.Schedule(delta=16, flags=og.OG_FLAG_ASYNC), ws=ws)
    torch.cuda.synchronize()
    assert st["status"] == 0
    import ctypes
    from paper_1911_07260_amd import _lib
    full = _lib.OgStats()
    rc = _lib.load().og_read_stats(ctypes.c_void_p(ws.buf.data_ptr()), ctypes.byref(full), None)
    assert rc == 0 and full.rounds > 0 and full.reached_vertices == g.n
    assert_exact(orc, g, 7, d.cpu().numpy(), p.cpu().numpy(), "async")


def test_graph_rounds_replayed(orc, road256, cfg0):
    """The executable round graph is reused across queries on one workspace
    (only the sources change) and rebuilt when the graph or schedule
    changes; every replay must match the oracle, with ordinary persistent
    launches and synchronisations in between."""
    g, dg = road256
    ws = og.Workspace(DEV)
    sched = og.Schedule(delta=512, engine=og.OG_ENGINE_GRAPH_ROUNDS)
    for i, src in enumerate(gg.pick_sources(g, 6, seed=21)):
        say(f"graph rounds replay {i} src={src}")
        d, p, st = og.sssp(dg, int(src), sched, ws=ws)
        torch.cuda.synchronize()
        assert_exact(orc, g, int(src), d.cpu().numpy(), p.cpu().numpy(), f"graph replay {i}")
        d2, p2, _ = og.sssp(dg, int(src), og.Schedule(delta=512), ws=og.Workspace(DEV))
        torch.cuda.synchronize()
        assert torch.equal(d, d2) and torch.equal(p, p2)
    g0, dg0 = cfg0
    for upd in (og.OG_EAGER_NO_FUSION, og.OG_LAZY_UPDATE, og.OG_EAGER_WITH_FUSION):
        say(f"graph rounds rebuild cfg0 update={upd}")
        d, p, st = run_sssp(dg0, 17, og.Schedule(delta=16, update=upd, engine=og.OG_ENGINE_GRAPH_ROUNDS), ws=ws)
        assert_exact(orc, g0, 17, d, p, f"graph rebuild {upd}")


@pytest.mark.slow
@pytest.mark.parametrize("delta", [512, 1024, 1 << 13])
def test_road_full_size_one_source(orc, delta):
    """Full 4096^2 road-like grid, fused, persistent engine, flat expansion
    (at Delta 512 the benchmark's fused_flat leg; its headline schedule adds
    degree bins, checked at full size with the bins' tests): bit-exact."""
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=1)[0])
    say(f"road4096 src={src} delta={delta} fused")
    d, p, st = run_sssp(dg, src, og.Schedule(delta=delta))
    assert st["status"] == 0
    assert_exact(orc, g, src, d, p, "road4096")


@pytest.mark.slow
def test_road_full_size_batched_sample(orc):
    """The benchmark's batched leg: 64 queries on the full 4096^2 grid in one
    launch (Delta 512, fused); queries 0, 37 and 63 are compared with the
    oracle element by element, and every query's distances satisfy the
    certificate's edge condition (no relaxable edge) on a vertex sample."""
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    srcs = [int(s) for s in gg.pick_sources(g, 64, seed=1)]
    say("road4096 batched x64 delta=512")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=512, queue_capacity=64 * (1 << 21)))
    torch.cuda.synchronize()
    assert st["status"] == 0
    for q in (0, 37, 63):
        ref_d, ref_p = orc.sssp(g, srcs[q])
        assert np.array_equal(d[q].cpu().numpy(), ref_d), q
        assert np.array_equal(p[q].cpu().numpy(), ref_p), q
    rng = np.random.default_rng(3)
    vs = rng.integers(0, g.n, size=20000)
    dd = d.cpu().numpy()
    for q in range(64):
        dq = dd[q].astype(np.int64)
        assert dq[srcs[q]] == 0
        for v in vs[:300]:
            if dq[v] == INF:
                continue
            row = slice(g.row_ptr[v], g.row_ptr[v + 1])
            assert np.all(dq[g.col[row]] <= dq[v] + g.w[row])


@pytest.mark.slow
def test_rmat22_sssp_and_wbfs_exact(orc):
    """R-MAT scale 22 (edge factor 16): SSSP at the benchmark's R-MAT
    schedule (Delta 32, unfused) and wBFS, bit-exact with the oracle."""
    g = gg.rmat(22, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    say(f"rmat22 sssp src={src}")
    d, p, st = run_sssp(dg, src, og.Schedule(delta=32, update=og.OG_EAGER_NO_FUSION))
    assert st["status"] == 0
    assert_exact(orc, g, src, d, p, "rmat22")
    wg = gg.with_weights(g, g.w % 21 + 1)  # [1, log2 n) for n = 2^22
    dwg = og.DeviceGraph.from_host(wg, DEV)
    say("rmat22 wbfs")
    d, p, st = run_sssp(dwg, src, og.Schedule(), fn="wbfs")
    assert st["status"] == 0
    assert_exact(orc, wg, src, d, p, "rmat22 wbfs")
