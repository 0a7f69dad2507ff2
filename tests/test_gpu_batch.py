"""GPU parity of the batched (many queries per launch) and multi-source
entry points against the CPU oracle, element by element."""
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
def road128():
    g = gg.road(128, seed=3)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
@pytest.mark.parametrize("delta", [16, 300])
def test_sssp_batch_grid(orc, update, delta):
    g = gg.grid(64, 64, 1, 100, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    srcs = [0, 4095, 2080, 17, 17, 999, 3000, 64]
    say(f"sssp_batch grid64 nq=8 delta={delta} update={update}")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=delta, update=update))
    torch.cuda.synchronize()
    assert d.shape == (8, g.n) and st["status"] == 0
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for q, s in enumerate(srcs):
        rd, rp = orc.sssp(g, s)
        assert np.array_equal(d[q], rd), q
        assert np.array_equal(p[q], rp), q
    assert st["reached_vertices"] == 8 * g.n


@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
def test_sssp_batch_and_multi_power_law(orc, update):
    """A power-law graph in one launch: R-MAT 14 has rows longer than the
    predecessor pass's per-chunk limit (up to 3,627 edges, listed as slices)
    and a mean degree that turns on its parity filter, in every query copy;
    distances and canonical predecessors of every query, and the
    multi-source distances, equal the oracle's."""
    g = gg.rmat(14, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    srcs = [int(x) for x in gg.pick_sources(g, 6, seed=12)]
    say(f"sssp_batch rmat14 nq=6 update={update}")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=32, update=update))
    torch.cuda.synchronize()
    assert st["status"] == 0
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for q, s in enumerate(srcs):
        rd, rp = orc.sssp(g, s)
        assert np.array_equal(d[q], rd), q
        assert np.array_equal(p[q], rp), q
    say(f"sssp_multi rmat14 nsrc=6 update={update}")
    dm, pm, st = og.sssp_multi(dg, srcs, og.Schedule(delta=32, update=update))
    torch.cuda.synchronize()
    assert st["status"] == 0
    ref = np.min(np.stack([orc.sssp(g, s)[0] for s in srcs]), axis=0)
    dm, pm = dm.cpu().numpy(), pm.cpu().numpy()
    assert np.array_equal(dm, ref)
    # canonical predecessors under the multi-source distances, by brute force
    # over every edge: the smallest tight in-neighbour, each source its own
    src_of = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    du = ref.astype(np.int64)
    tight = (du[src_of] < INF) & (du[src_of] + g.w == du[g.col])
    want = np.full(g.n, np.iinfo(np.int64).max)
    np.minimum.at(want, g.col[tight], src_of[tight])
    want[ref == INF] = -1
    want[srcs] = srcs
    assert np.array_equal(pm.astype(np.int64), want)


@pytest.mark.parametrize("nq", [1, 5, 32])
def test_sssp_batch_road(orc, road128, nq):
    g, dg = road128
    srcs = gg.pick_sources(g, nq, seed=11)
    say(f"sssp_batch road128 nq={nq}")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=256))
    torch.cuda.synchronize()
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for q, s in enumerate(srcs):
        rd, rp = orc.sssp(g, int(s))
        assert np.array_equal(d[q], rd), q
        assert np.array_equal(p[q], rp), q


def test_sssp_batch_matches_single(road128):
    g, dg = road128
    srcs = gg.pick_sources(g, 4, seed=12)
    say("sssp_batch vs og_sssp")
    d, p, _ = og.sssp_batch(dg, srcs, og.Schedule(delta=128))
    for q, s in enumerate(srcs):
        d1, p1, _ = og.sssp(dg, int(s), og.Schedule(delta=128))
        assert torch.equal(d[q], d1) and torch.equal(p[q], p1)


def walk(g, s, t, pred):
    v, total, steps = t, 0, 0
    while v != s:
        u = int(pred[v])
        assert u >= 0
        row = slice(g.row_ptr[u], g.row_ptr[u + 1])
        idx = np.nonzero(g.col[row] == v)[0]
        assert len(idx) == 1
        total += int(g.w[row][idx[0]])
        v = u
        steps += 1
        assert steps <= g.n
    return total


def test_ppsp_batch(orc, road128):
    g, dg = road128
    nq = 12
    srcs = gg.pick_sources(g, nq, seed=13)
    dsts = gg.uniform(14, gg.STREAM_TARGETS, nq, g.n)
    say("ppsp_batch road128 nq=12")
    d, p, st = og.ppsp_batch(dg, srcs, dsts, og.Schedule(delta=64))
    torch.cuda.synchronize()
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for q in range(nq):
        s, t = int(srcs[q]), int(dsts[q])
        want = orc.ppsp(g, s, t)
        if want < 0:
            assert d[q, t] == INF
        else:
            assert d[q, t] == want
            assert walk(g, s, t, p[q]) == want


def test_astar_batch(orc, road128):
    g, dg = road128
    nq = 10
    srcs = gg.pick_sources(g, nq, seed=15)
    dsts = gg.uniform(16, gg.STREAM_TARGETS, nq, g.n)
    h = np.stack([gg.grid_heuristic(128, int(t)) for t in dsts])
    say("astar_batch road128 nq=10")
    d, p, st = og.astar_batch(dg, srcs, dsts, torch.from_numpy(h).to(DEV), og.Schedule(delta=64))
    torch.cuda.synchronize()
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for q in range(nq):
        s, t = int(srcs[q]), int(dsts[q])
        want = orc.ppsp(g, s, t)
        if want < 0:
            assert d[q, t] == INF
        else:
            assert d[q, t] == want
            assert walk(g, s, t, p[q]) == want


def block_diagonal(graphs):
    """Disjoint union of CSR graphs (vertex ids offset by the preceding sizes)."""
    n = sum(g.n for g in graphs)
    row_ptr = [np.zeros(1, dtype=np.int64)]
    cols, ws = [], []
    voff = eoff = 0
    for g in graphs:
        row_ptr.append(g.row_ptr[1:] + eoff)
        cols.append(g.col + voff)
        ws.append(g.w)
        voff += g.n
        eoff += g.m
    return gg.Graph(n=n, row_ptr=np.concatenate(row_ptr), col=np.concatenate(cols).astype(np.int32),
                    w=np.concatenate(ws).astype(np.int32), name="union")


def test_multi_source_disjoint_graphs(orc):
    rng = np.random.default_rng(3)
    sizes = [int(x) for x in rng.integers(200, 3000, size=24)]
    parts = [gg.rgg(sz, 6.0, seed=100 + i)[0] for i, sz in enumerate(sizes)]
    u = block_diagonal(parts)
    offs = np.concatenate([[0], np.cumsum([p.n for p in parts])[:-1]])
    local_src = [int(rng.integers(0, p.n)) for p in parts]
    srcs = [int(o + s) for o, s in zip(offs, local_src)]
    du = og.DeviceGraph.from_host(u, DEV)
    say(f"multi-source on {len(parts)} disjoint RGGs, n={u.n}")
    d, p, st = og.sssp_multi(du, srcs, og.Schedule(delta=2000))
    torch.cuda.synchronize()
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for i, part in enumerate(parts):
        rd, rp = orc.sssp(part, local_src[i])
        sl = slice(int(offs[i]), int(offs[i]) + part.n)
        assert np.array_equal(d[sl], rd), i
        got_p = p[sl]
        want_p = np.where(rp >= 0, rp + offs[i], -1)
        assert np.array_equal(got_p, want_p), i


def test_multi_source_super_source_reduction(orc, road128):
    """Multi-source distances equal single-source distances from an added
    super-source joined to every source by a zero-weight edge."""
    g, dg = road128
    srcs = [int(s) for s in gg.pick_sources(g, 7, seed=17)]
    say("multi-source road128 vs super-source reduction")
    d, p, st = og.sssp_multi(dg, srcs, og.Schedule(delta=256))
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    src = np.repeat(np.arange(g.n), g.degrees())
    big = gg.from_edges(g.n + 1, np.concatenate([src, np.full(len(srcs), g.n)]),
                        np.concatenate([g.col, srcs]), np.concatenate([g.w, np.zeros(len(srcs), dtype=np.int32)]))
    rd, _ = orc.sssp(big, g.n)
    assert np.array_equal(d, rd[:g.n])
    assert orc.check(big, g.n, np.concatenate([d, [0]]).astype(np.int32), None) == 0


@pytest.mark.parametrize("fn", ["sssp", "ppsp", "astar"])
def test_batch_waves_beyond_one_launch(orc, fn):
    """A batch of more queries than one launch holds (1,024 per launch) runs
    as consecutive launches on one workspace: 1,100 queries on the 64 x 64
    grid (two launches), every sampled query exact, including both sides of
    the cut, and the counters summed over the launches."""
    side = 64
    g = gg.road(side, seed=0)  # weights >= 10 * length: floor(10 * euclid) is admissible
    dg = og.DeviceGraph.from_host(g, DEV)
    nq = 1100
    srcs = gg.pick_sources(g, nq, seed=31)
    dsts = gg.pick_sources(g, nq, seed=32)
    sched = og.Schedule(delta=64)
    assert og.workspace_bytes(dg, sched, batch=nq) == og.workspace_bytes(dg, sched, batch=1024)
    say(f"{fn}_batch waves nq={nq}")
    if fn == "sssp":
        d, p, st = og.sssp_batch(dg, srcs, sched)
    elif fn == "ppsp":
        d, p, st = og.ppsp_batch(dg, srcs, dsts, sched)
    else:
        hs = [gg.grid_heuristic_device(side, dsts[q0:q0 + 275], DEV) for q0 in range(0, nq, 275)]
        h = torch.cat(hs).contiguous()
        d, p, st = og.astar_batch(dg, srcs, dsts, h, sched)
    torch.cuda.synchronize()
    assert st["status"] == 0 and d.shape == (nq, g.n)
    dn, pn = d.cpu().numpy(), p.cpu().numpy()
    for q in (0, 511, 1023, 1024, 1050, 1099):
        if fn == "sssp":
            rd, rp = orc.sssp(g, int(srcs[q]))
            assert np.array_equal(dn[q], rd) and np.array_equal(pn[q], rp), q
        else:
            want = orc.ppsp(g, int(srcs[q]), int(dsts[q]))
            if want < 0:
                assert dn[q, dsts[q]] == INF, q
                continue
            assert dn[q, dsts[q]] == want, q
            assert walk(g, int(srcs[q]), int(dsts[q]), pn[q]) == want, q
    if fn == "sssp":
        assert st["reached_vertices"] == int(np.count_nonzero(dn != INF))


def walk(g, s, t, pred):
    v, total = t, 0
    while v != s:
        u = int(pred[v])
        row = slice(g.row_ptr[u], g.row_ptr[u + 1])
        idx = np.nonzero(g.col[row] == v)[0]
        assert len(idx) >= 1
        total += int(g.w[row][idx].min())
        v = u
    return total


@pytest.mark.slow
def test_road4096_batch256(orc):
    """256 single-source queries on the full 4096^2 road-like grid in one
    og_sssp_batch call (virtual ids 256 * n >= 2^31: launches of 127
    queries), queries on both sides of each launch boundary compared with
    the oracle element by element."""
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    srcs = [int(s) for s in gg.pick_sources(g, 256, seed=1)]
    say("road4096 batch x256")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=512, queue_capacity=127 * (1 << 21)))
    torch.cuda.synchronize()
    assert st["status"] == 0
    for q in (0, 126, 127, 253, 254, 255):
        ref_d, ref_p = orc.sssp(g, srcs[q])
        assert np.array_equal(d[q].cpu().numpy(), ref_d), q
        assert np.array_equal(p[q].cpu().numpy(), ref_p), q
    del d, p
    torch.cuda.empty_cache()
