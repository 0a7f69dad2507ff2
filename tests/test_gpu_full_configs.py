"""Full-size GPU parity of the configurations the benchmark lines run.

Each test builds its configuration at full size and compares the HIP path,
through the C ABI, with the CPU oracle element by element (distances and
canonical predecessors are integers: bit-exact), or, for point-to-point
queries, the target distance plus a walk of the predecessor chain.

  - R-MAT scale 24 (edge factor 16): plain Delta-stepping SSSP, unfused and
    fused, and wBFS with weights in [1, 24) (Delta = 1);
  - the road-like 4096^2 grid: degree-binned SSSP at Delta 2^8 and 2^14 (the
    ends of the benchmark's sweep), and one launch of 64 A* queries with the
    estimate floor(10 * euclid);
  - 1,024 random geometric graphs of uneven size in one multi-source launch,
    16 of them compared with the oracle;
  - R-MAT scale 22 with float32 weights: forward bit-exact against the
    float32 oracle, backward exact against the oracle's subtree sums.
"""
import concurrent.futures as cf
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

INF = og.INF
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_refs = {}


def exact(orc, g, src, d, p, tag, key=None):
    say(f"{tag}: oracle")
    if key is not None and key in _refs:
        ref_d, ref_p = _refs[key]
    else:
        ref_d, ref_p = orc.sssp(g, src)
        if key is not None:
            _refs[key] = (ref_d, ref_p)
    d = d.cpu().numpy()
    p = p.cpu().numpy()
    nd = int(np.count_nonzero(d != ref_d))
    assert nd == 0, f"{tag}: {nd} distances differ (first at {np.nonzero(d != ref_d)[0][:5]})"
    npd = int(np.count_nonzero(p != ref_p))
    assert npd == 0, f"{tag}: {npd} predecessors differ"
    say(f"{tag}: exact")


def walk_path(g, s, t, pred):
    """Length of the predecessor chain from t back to s (every step must be
    an edge of the graph)."""
    v, total, steps = t, 0, 0
    while v != s:
        u = int(pred[v])
        assert u >= 0, "path broken"
        row = slice(g.row_ptr[u], g.row_ptr[u + 1])
        idx = np.nonzero(g.col[row] == v)[0]
        assert len(idx) >= 1, "pred edge missing"
        total += int(g.w[row][idx].min())
        v = u
        steps += 1
        assert steps <= g.n
    return total


@pytest.fixture(scope="module")
def rmat24():
    say("rmat24: generating")
    g = gg.rmat(24, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    say(f"rmat24: n={g.n} m={g.m}")
    yield g, dg
    del dg
    torch.cuda.empty_cache()


@pytest.mark.parametrize("update", [og.OG_EAGER_NO_FUSION, og.OG_EAGER_WITH_FUSION])
def test_rmat24_sssp_delta32(orc, rmat24, update):
    """The benchmark's plain R-MAT schedule (Delta 32), unfused and fused."""
    g, dg = rmat24
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    tag = f"rmat24 sssp src={src} delta=32 update={update}"
    say(tag)
    d, p, st = og.sssp(dg, src, og.Schedule(delta=32, update=update))
    torch.cuda.synchronize()
    assert st["status"] == 0
    exact(orc, g, src, d, p, tag, key=("rmat24", src))


def test_rmat24_wbfs(orc, rmat24):
    """wBFS on R-MAT 24 with weights in [1, log2 n) = [1, 24), Delta = 1."""
    g, dg = rmat24
    wg = gg.with_weights(g, g.w % 23 + 1)
    dwg = og.DeviceGraph(dg.row_ptr, dg.col, torch.from_numpy(wg.w).to(DEV))
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    tag = f"rmat24 wbfs src={src}"
    say(tag)
    d, p, st = og.wbfs(dwg, src, og.Schedule())
    torch.cuda.synchronize()
    assert st["status"] == 0
    exact(orc, wg, src, d, p, tag)


@pytest.fixture(scope="module")
def road4096():
    say("road4096: generating")
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    yield g, dg
    del dg
    torch.cuda.empty_cache()


@pytest.mark.parametrize("delta", [1 << 8, 1 << 14])
def test_road4096_bins_delta_range(orc, road4096, delta):
    """The ends of the benchmark's Delta sweep with its load balancing."""
    g, dg = road4096
    src = int(gg.pick_sources(g, 1, seed=1)[0])
    tag = f"road4096 bins src={src} delta={delta}"
    say(tag)
    d, p, st = og.sssp(dg, src, og.Schedule(delta=delta, flags=og.OG_FLAG_DEGREE_BINS))
    torch.cuda.synchronize()
    assert st["status"] == 0
    exact(orc, g, src, d, p, tag, key=("road4096", src))


def test_road4096_astar_batch64(orc, road4096):
    """One launch of 64 A* queries (the A* line's launch size), estimate
    floor(10 * euclid) to each query's target: every target distance equals
    the oracle's point-to-point distance and every predecessor chain from
    the target back to the source sums to it."""
    g, dg = road4096
    nq = 64
    srcs = gg.pick_sources(g, nq, seed=3)
    dsts = gg.pick_sources(g, nq, seed=4)
    h = gg.grid_heuristic_device(4096, dsts, DEV)
    say("road4096 astar batch x64")
    d, p, st = og.astar_batch(dg, srcs, dsts, h, og.Schedule(delta=512, queue_capacity=nq * (1 << 20)))
    torch.cuda.synchronize()
    assert st["status"] == 0
    q = torch.arange(nq, device=DEV)
    tt = torch.as_tensor(dsts, device=DEV)
    got = d[q, tt].cpu().numpy()
    del h
    say("road4096 astar batch x64: oracle (8 threads)")
    with cf.ThreadPoolExecutor(8) as ex:
        want = list(ex.map(lambda i: orc.ppsp(g, int(srcs[i]), int(dsts[i])), range(nq)))
    for i in range(nq):
        if want[i] < 0:
            assert got[i] == INF, i
            continue
        assert got[i] == want[i], (i, got[i], want[i])
        assert walk_path(g, int(srcs[i]), int(dsts[i]), p[i].cpu().numpy()) == want[i], i
    say("road4096 astar batch x64: exact")
    del d, p


def test_rgg1024_one_launch(orc):
    """The 1,024 random geometric graphs of the RGG line (sizes log-uniform in
    [1000, 64000], mean degree 6) solved in one multi-source launch over
    their block-diagonal union at the line's Delta; 16 graphs spread over
    the family are compared with the oracle element by element."""
    say("rgg1024: generating")
    fam = gg.rgg_family(1024, seed=5)
    u, offs = gg.block_diagonal(fam)
    loc = [int(gg.uniform(6 + i, gg.STREAM_SOURCES, 1, p.n)[0]) for i, p in enumerate(fam)]
    srcs = [int(o) + s for o, s in zip(offs, loc)]
    du = og.DeviceGraph.from_host(u, DEV)
    say(f"rgg1024 multi n={u.n} m={u.m}")
    d, p, st = og.sssp_multi(du, srcs, og.Schedule(delta=131072))
    torch.cuda.synchronize()
    assert st["status"] == 0
    dn, pn = d.cpu().numpy(), p.cpu().numpy()
    for i in range(0, 1024, 64):
        rd, rp = orc.sssp(fam[i], loc[i])
        o = int(offs[i])
        assert np.array_equal(dn[o:o + fam[i].n], rd), i
        # predecessors are union ids; the oracle's are the graph's own
        want_p = np.where(rp >= 0, rp + o, -1)
        assert np.array_equal(pn[o:o + fam[i].n], want_p), i
    say("rgg1024: 16 graphs exact")


def test_rmat22_float32_forward_backward(orc):
    """R-MAT 22 with float32 weights U(1, 1000) and 1,024 targets: the
    forward distances equal the float32 oracle bit for bit, and the
    backward pass equals the oracle's subtree sums on the oracle's tree."""
    say("rmat22 f32: generating")
    g = gg.rmat(22, 16, seed=0)
    w = gg.float_weights(g, 1.0, 1000.0, seed=3)
    dg = og.DeviceGraph.from_host(g, DEV)
    wt = torch.from_numpy(w).to(DEV)
    s = int(gg.pick_sources(g, 1, seed=1)[0])
    say(f"rmat22 f32 forward + backward src={s}")
    d, p, pe, st = og.sssp_f32(dg, wt, s, og.Schedule(delta=64))
    assert st["status"] == 0
    targets = gg.pick_sources(g, 1024, seed=3)
    up = np.bincount(targets, minlength=g.n).astype(np.float32)
    gw = og.sssp_backward_f32(dg, wt, p, pe, torch.from_numpy(up).to(DEV))
    torch.cuda.synchronize()
    say("rmat22 f32: oracle")
    ref = orc.dijkstra_real(g, w, s, f32=True)
    fin = np.isfinite(ref)
    dn = d.cpu().numpy()
    assert np.array_equal(dn[fin], ref[fin].astype(np.float32)) and np.all(np.isinf(dn[~fin]))
    rp, rpe = orc.tree_real(g, w, s, ref, f32=True)
    assert np.array_equal(p.cpu().numpy(), rp) and np.array_equal(pe.cpu().numpy(), rpe)
    want = orc.subtree_grad(g, ref, rp, rpe, np.where(fin, up, 0).astype(np.float64))
    assert np.array_equal(gw.cpu().numpy(), want.astype(np.float32))
    say("rmat22 f32: exact")
