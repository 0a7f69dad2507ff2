"""GPU parity of the vertex-block engine (OG_FLAG_VERTEX_BLOCKS): bucket
fusion inside LDS-resident blocks, with blocks improved across their
boundary queued for any workgroup within the round.

Distances and canonical predecessors must equal the oracle's bit for bit
for every Delta, block size (from one vertex per block, where every edge
leaves its block, to the 4,096-vertex cap), workgroup count and graph
shape; PPSP and wBFS use the same engine.  A blocked copy kept across calls
must give the same answers as a fresh one.
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
BLK = og.OG_FLAG_VERTEX_BLOCKS


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check(orc, g, src, d, p, tag):
    ref_d, ref_p = orc.sssp(g, src)
    d = d.cpu().numpy()
    p = p.cpu().numpy()
    nd = int(np.count_nonzero(d != ref_d))
    assert nd == 0, f"{tag}: {nd} distances differ (first at {np.nonzero(d != ref_d)[0][:5]})"
    npd = int(np.count_nonzero(p != ref_p))
    assert npd == 0, f"{tag}: {npd} predecessors differ"


@pytest.fixture(scope="module")
def cfg0():
    g = gg.grid(64, 64, 1, 100, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.fixture(scope="module")
def road256():
    g = gg.road(256, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.mark.parametrize("block_size", [1, 4, 64, 2048, 4096])
@pytest.mark.parametrize("delta", [1, 16, 100, 1 << 20])
def test_cfg0_block_sizes(orc, cfg0, block_size, delta):
    g, dg = cfg0
    tag = f"blocks cfg0 block_size={block_size} delta={delta}"
    say(tag)
    d, p, st = og.sssp(dg, 0, og.Schedule(delta=delta, flags=BLK, block_size=block_size))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check(orc, g, 0, d, p, tag)
    assert 1 <= st["blocks"] <= g.n
    if block_size == 1:
        assert st["blocks"] == g.n  # every vertex seeds its own cell
    assert st["reached_vertices"] == g.n


@pytest.mark.parametrize("workgroups", [1, 3, 0])
def test_cfg0_workgroups(orc, cfg0, workgroups):
    g, dg = cfg0
    for bs in (16, 1024):
        tag = f"blocks cfg0 wg={workgroups} block_size={bs}"
        say(tag)
        d, p, st = og.sssp(dg, 4095, og.Schedule(delta=64, flags=BLK, workgroups=workgroups, block_size=bs))
        torch.cuda.synchronize()
        assert st["status"] == 0
        check(orc, g, 4095, d, p, tag)


@pytest.mark.parametrize("delta", [256, 1024, 4096, 1 << 14])
def test_road256(orc, road256, delta):
    g, dg = road256
    for src in gg.pick_sources(g, 3, seed=1):
        tag = f"blocks road256 src={src} delta={delta}"
        say(tag)
        d, p, st = og.sssp(dg, int(src), og.Schedule(delta=delta, flags=BLK))
        torch.cuda.synchronize()
        assert st["status"] == 0
        check(orc, g, int(src), d, p, tag)


def test_road256_kept_copy(orc, road256):
    """A kept blocked copy: built by the first call, reused by the next ones
    (no build time), with the same block count and exact answers; a call
    with another block size rebuilds."""
    g, dg = road256
    ws = og.Workspace(DEV)
    fl = BLK | og.OG_FLAG_KEEP_BLOCKS | og.OG_FLAG_TIMING
    blocks = None
    for i, src in enumerate(gg.pick_sources(g, 4, seed=9)):
        say(f"blocks kept copy call {i}")
        d, p, st = og.sssp(dg, int(src), og.Schedule(delta=512, flags=fl), ws=ws)
        torch.cuda.synchronize()
        assert st["status"] == 0
        check(orc, g, int(src), d, p, f"kept {i}")
        if i == 0:
            blocks = st["blocks"]
            assert st["prep_ms"] > 0
        else:
            assert st["blocks"] == blocks and st["prep_ms"] == 0
    d, p, st = og.sssp(dg, 5, og.Schedule(delta=512, flags=fl, block_size=512), ws=ws)
    torch.cuda.synchronize()
    assert st["prep_ms"] > 0 and st["blocks"] > blocks
    check(orc, g, 5, d, p, "kept, other block size")
    # another engine on the workspace drops the record: the next block call rebuilds
    og.sssp(dg, 5, og.Schedule(delta=512), ws=ws)
    d, p, st = og.sssp(dg, 6, og.Schedule(delta=512, flags=fl, block_size=512), ws=ws)
    torch.cuda.synchronize()
    assert st["prep_ms"] > 0
    check(orc, g, 6, d, p, "rebuilt")


@pytest.mark.parametrize("delta", [1, 8, 64, 700])
def test_rmat14(orc, delta):
    """A power-law graph (hubs, little locality): still exact."""
    g = gg.rmat(14, 16, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=2)[0])
    tag = f"blocks rmat14 src={src} delta={delta}"
    say(tag)
    d, p, st = og.sssp(dg, src, og.Schedule(delta=delta, flags=BLK))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check(orc, g, src, d, p, tag)


def test_wbfs_ppsp_multi(orc, road256):
    g, dg = road256
    wg = gg.with_weights(g, g.w % 15 + 1)
    dwg = og.DeviceGraph.from_host(wg, DEV)
    src = int(gg.pick_sources(g, 1, seed=4)[0])
    say("blocks wbfs road256")
    d, p, st = og.wbfs(dwg, src, og.Schedule(flags=BLK))
    torch.cuda.synchronize()
    check(orc, wg, src, d, p, "blocks wbfs")
    rng = np.random.default_rng(11)
    for i in range(4):
        t = int(rng.integers(0, g.n))
        say(f"blocks ppsp {src}->{t}")
        d, p, st = og.ppsp(dg, src, t, og.Schedule(delta=256, flags=BLK))
        torch.cuda.synchronize()
        want = orc.ppsp(g, src, t)
        assert int(d[t].item()) == (INF if want < 0 else want)
    srcs = [int(s) for s in gg.pick_sources(g, 5, seed=12)]
    say("blocks multi-source road256")
    d, p, st = og.sssp_multi(dg, srcs, og.Schedule(delta=256, flags=BLK))
    torch.cuda.synchronize()
    assert st["status"] == 0
    ref = np.min(np.stack([orc.sssp(g, s)[0].astype(np.int64) for s in srcs]), axis=0)
    assert np.array_equal(d.cpu().numpy().astype(np.int64), ref)


def test_edge_cases(orc):
    """Heavy internal edges (weight >= 65536 is kept as a leaving edge even
    inside a block), zero weights, isolated vertices and self-loops, a
    one-vertex graph, a graph without edges."""
    rng = np.random.default_rng(5)
    n = 3000
    src = rng.integers(0, n, 12000)
    dst = (src + rng.integers(-40, 41, 12000)) % n
    w = rng.integers(0, 200, 12000)
    w[rng.random(12000) < 0.05] = 70000
    w[rng.random(12000) < 0.05] = 0
    s2 = np.concatenate([src, dst, [7, 7]])
    d2 = np.concatenate([dst, src, [7, 7]])
    w2 = np.concatenate([w, w, [3, 0]])
    g = gg.from_edges(n + 50, s2, d2, w2)  # the last 50 vertices are isolated
    dg = og.DeviceGraph.from_host(g, DEV)
    for bs in (1, 32, 4096):
        for delta in (1, 300, 1 << 22):
            tag = f"blocks edge cases bs={bs} delta={delta}"
            say(tag)
            d, p, st = og.sssp(dg, 7, og.Schedule(delta=delta, flags=BLK, block_size=bs))
            torch.cuda.synchronize()
            assert st["status"] == 0
            ref_d, _ = orc.sssp(g, 7)
            assert np.array_equal(d.cpu().numpy(), ref_d), tag
            assert orc.check(g, 7, d.cpu().numpy(), None) == 0
    one = gg.from_edges(1, [], [], [])
    d, p, st = og.sssp(og.DeviceGraph.from_host(one, DEV), 0, og.Schedule(delta=4, flags=BLK))
    torch.cuda.synchronize()
    assert st["status"] == 0 and d.cpu().tolist() == [0] and p.cpu().tolist() == [0]
    empty = gg.from_edges(100, [], [], [])
    d, p, st = og.sssp(og.DeviceGraph.from_host(empty, DEV), 42, og.Schedule(delta=4, flags=BLK))
    torch.cuda.synchronize()
    dn = d.cpu().numpy()
    assert dn[42] == 0 and np.all(np.delete(dn, 42) == INF)


def test_errors(cfg0):
    """A negative weight reached by the search, and a path that overflows
    int32, are reported through the status."""
    g, _ = cfg0
    w = g.w.copy()
    w[g.row_ptr[0]] = -5
    bad = og.DeviceGraph.from_host(gg.with_weights(g, w), DEV)
    _, _, st = og.sssp(bad, 0, og.Schedule(delta=16, flags=BLK), check=False)
    assert st["status"] == og.OG_ERR_NEGATIVE_WEIGHT
    big = og.DeviceGraph.from_host(gg.with_weights(g, np.full_like(g.w, 1 << 26)), DEV)
    _, _, st = og.sssp(big, 0, og.Schedule(delta=1 << 20, flags=BLK), check=False)
    assert st["status"] == og.OG_ERR_OVERFLOW


@pytest.mark.slow
def test_road4096_full_size(orc):
    """The full 4096^2 road-like grid with the headline's block schedule,
    the copy kept across two sources."""
    g = gg.road(4096, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    ws = og.Workspace(DEV)
    for src in gg.pick_sources(g, 2, seed=1):
        for delta in (1 << 10, 1 << 12):
            tag = f"blocks road4096 src={src} delta={delta}"
            say(tag)
            d, p, st = og.sssp(dg, int(src), og.Schedule(delta=delta, flags=BLK | og.OG_FLAG_KEEP_BLOCKS),
                               ws=ws)
            torch.cuda.synchronize()
            assert st["status"] == 0
            check(orc, g, int(src), d, p, tag)
