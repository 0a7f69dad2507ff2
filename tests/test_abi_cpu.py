"""C ABI checks that need no GPU: every symbol declared in include/*.h is
exported by libog.so, struct layouts agree with the header, and argument
validation rejects bad calls before anything is launched."""
import ctypes
import glob
import os
import re

import pytest

import paper_1911_07260_amd as og
from paper_1911_07260_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(og_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = declared_functions()
    assert "og_sssp" in names and "og_astar" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_no_oracle_in_product():
    """The product library links no oracle code and the package never
    imports it."""
    src = open(os.path.join(ROOT, "paper_1911_07260_amd", "csrc", "og_engine.hip")).read()
    assert "oracle" not in src
    for py in glob.glob(os.path.join(ROOT, "paper_1911_07260_amd", "*.py")):
        assert "import oracle" not in open(py).read()
    lib = _lib.load()
    assert not hasattr(lib, "oracle_dijkstra")


def test_version_and_strings():
    assert og.version() >> 16 == 1
    assert og.status_string(0) == "ok"
    assert "workspace" in og.status_string(og.OG_ERR_WORKSPACE)
    assert "internal" in og.status_string(og.OG_ERR_INTERNAL)
    assert og.status_string(12345) == "unknown status"


def test_default_schedule():
    lib = _lib.load()
    s = _lib.OgSchedule()
    assert lib.og_default_schedule(ctypes.byref(s)) == 0
    assert s.delta == 1 and s.update == 1 and s.window_buckets == 16 and s.fusion_threshold == 1024
    assert s.bin_thread == 4 and s.bin_wave == 64 and s.block_size == 2048
    assert lib.og_default_schedule(None) == og.OG_ERR_INVALID_ARG


def _fake_graph(n=10, m=20):
    # never dereferenced: these calls must fail validation first
    return _lib.OgGraph(n, m, 0x1000, 0x2000, 0x3000)


CTL = 131072  # the control block: counters, flags, each team's control state and queue tails


def _queues(cap, k, nsrc=1, pool=0, teams=1):
    """Bytes of the global queues: per-queue chunk tables (K + 4 queues per
    team), the free stack and the pool of 4,096-entry chunks (default: twice
    one queue's capacity plus one chunk per queue, at most every queue full,
    at least the sources' chunks plus one and one chunk per team), each
    region 256-byte aligned."""
    ck = 4096
    lists = teams * (k + 4)
    tch = -(-cap // ck)
    pre = -(-nsrc // ck)
    ch = -(-pool // ck) if pool > 0 else -(-2 * cap // ck) + lists
    ch = max(min(ch, lists * tch), pre + 1, teams)

    def v(nbytes):
        return (nbytes + 255) // 256 * 256

    return v(4 * lists * tch) + v(4 * ch) + v(8 * ch * ck)


def test_workspace_bytes():
    lib = _lib.load()
    g = _fake_graph(1000, 4000)
    s = og.Schedule(delta=4).to_c()
    b = lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(s))
    assert b % 256 == 0 and b >= CTL + (16 + 4) * 1024 * 8
    s2 = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000).to_c()
    Q = _queues(5000, 8)
    assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(s2)) == CTL + 256 + Q
    # an explicit pool size, rounded up to whole chunks and clamped to the queues' total
    for pool, want in ((1, 2), (9000, 3), (10 ** 9, 24)):
        sp = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000, queue_pool=pool).to_c()
        assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(sp)) == CTL + 256 + _queues(5000, 8, pool=pool)
        assert _queues(5000, 8, pool=pool) == 256 + (4 * want + 255) // 256 * 256 + 8 * 4096 * want
    neg = og.Schedule(delta=4, queue_pool=-1).to_c()
    assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(neg)) == 0
    # lazy update: + change flags and change buffer, one int per vertex each
    s3 = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000, update=og.OG_LAZY_UPDATE).to_c()
    vec = (g.n * 4 + 255) // 256 * 256
    assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(s3)) == CTL + 256 + Q + 2 * vec
    # k-core: no source table; + peel marks (and the lazy arrays)
    base = CTL + Q
    assert lib.og_workspace_bytes_kcore(ctypes.byref(g), ctypes.byref(s2)) == base + vec
    assert lib.og_workspace_bytes_kcore(ctypes.byref(g), ctypes.byref(s3)) == base + 3 * vec
    # light/heavy split: + split copy of col and w, light counts, long-row
    # list, bucket stamps and two heavy lists of (v, slice) entries, each
    # n + m / 4096 + 1 long (a heavy part is filed once per 4,096 edges)
    s4 = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000, flags=og.OG_FLAG_LIGHT_HEAVY).to_c()
    for gs in (g, _fake_graph(1000, 100_000)):
        evec = (gs.m * 4 + 255) // 256 * 256
        hvec = ((gs.n + gs.m // 4096 + 1) * 4 + 255) // 256 * 256
        assert lib.og_workspace_bytes(ctypes.byref(gs), ctypes.byref(s4)) == (CTL + 256 + Q
                                                                              + 2 * evec + 3 * vec + 4 * hvec)
    # pull direction (lazy only): + frontier marks (SSSP: 8 bytes per vertex; k-core: one bit) and the
    # long rows' slice list
    for fl in (og.OG_FLAG_DENSE_PULL, og.OG_FLAG_HYBRID_DIRECTION):
        s5 = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000, update=og.OG_LAZY_UPDATE, flags=fl).to_c()
        marks = (g.n * 8 + 255) // 256 * 256
        bits = ((g.n + 31) // 32 * 4 + 255) // 256 * 256
        slices = ((g.m // 2048 + g.m // 8192 + 1) * 8 + 255) // 256 * 256
        assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(s5)) == (CTL + 256 + Q + 2 * vec
                                                                             + marks + slices)
        assert lib.og_workspace_bytes_kcore(ctypes.byref(g), ctypes.byref(s5)) == base + 3 * vec + bits + slices
    lazy_split = og.Schedule(delta=4, update=og.OG_LAZY_UPDATE, flags=og.OG_FLAG_LIGHT_HEAVY).to_c()
    assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(lazy_split)) == 0
    assert lib.og_workspace_bytes_kcore(ctypes.byref(g), ctypes.byref(s4)) == base + vec
    bad = og.Schedule(delta=0).to_c()
    assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(bad)) == 0
    g0 = _lib.OgGraph(0, 0, 0x1000, None, None)
    assert lib.og_workspace_bytes(ctypes.byref(g0), ctypes.byref(s)) == 0


def test_batch_workspace_holds_every_teams_queues():
    """A batched call of the eager push engine sizes its queues for its teams
    (schedule.teams; by default 8; at most 8 and one per query); the lazy
    update and the split, pull and block variants keep one team."""
    lib = _lib.load()
    g = _fake_graph(1000, 4000)
    table = lambda nq: (4 * (nq + nq) + 255) // 256 * 256  # sources and targets
    per = 1000 + 4000 // 8
    for nq, teams, want in ((8, 0, 8), (3, 0, 3), (7, 0, 7), (16, 0, 8), (64, 0, 8), (8, 1, 1), (8, 4, 4),
                            (8, 99, 8), (3, 8, 3)):
        s = og.Schedule(delta=4, window_buckets=8, teams=teams).to_c()
        got = lib.og_workspace_bytes_batch(ctypes.byref(g), ctypes.byref(s), nq)
        assert got == CTL + table(nq) + _queues(nq * per + nq, 8, nsrc=nq, teams=want), (nq, teams)
    # a tiny pool still gives every team's share a chunk (8 chunks, not the
    # sources' one plus one)
    tiny = og.Schedule(delta=4, window_buckets=8, teams=8, queue_pool=1).to_c()
    assert lib.og_workspace_bytes_batch(ctypes.byref(g), ctypes.byref(tiny), 8) == (
        CTL + table(8) + _queues(8 * per + 8, 8, nsrc=8, pool=1, teams=8))
    lazy = og.Schedule(delta=4, window_buckets=8, update=og.OG_LAZY_UPDATE).to_c()
    vec = (8 * 1000 * 4 + 255) // 256 * 256
    assert lib.og_workspace_bytes_batch(ctypes.byref(g), ctypes.byref(lazy), 8) == (
        CTL + table(8) + _queues(8 * per + 8, 8, nsrc=8, teams=1) + 2 * vec)
    neg = og.Schedule(delta=4, teams=-1).to_c()
    assert lib.og_workspace_bytes_batch(ctypes.byref(g), ctypes.byref(neg), 8) == 0


@pytest.mark.parametrize("field,value", [
    ("delta", 0), ("update", 3), ("window_buckets", 1), ("window_buckets", 65), ("engine", 7),
    ("max_rounds", -1), ("flags", 1024), ("fusion_threshold", -2),
    # a pull direction needs lazy updates, and takes one direction flag
    ("flags", 16), ("flags", 32),
    # degree bins: non-negative cut-offs, not with the split or a pull direction
    ("bin_thread", -1), ("bin_wave", -1), ("flags", 64 | 8), ("flags", 64 | 16),
    # vertex blocks: not with the split, the degree bins or a pull direction; a non-negative block size
    ("flags", 256 | 8), ("flags", 256 | 64), ("flags", 256 | 16), ("block_size", -1),
    # queue pool and teams: non-negative
    ("queue_pool", -1), ("teams", -1),
])
def test_invalid_schedule_rejected(field, value):
    lib = _lib.load()
    g = _fake_graph()
    s = og.Schedule(delta=4)
    setattr(s, field, value)
    sc = s.to_c()
    st = _lib.OgStats()
    rc = lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(sc), ctypes.c_void_p(0x4000), None,
                     ctypes.c_void_p(0x10000), ctypes.c_size_t(1 << 40), ctypes.byref(st), None)
    assert rc == og.OG_ERR_INVALID_ARG and st.status == rc


def test_pull_direction_rules():
    lib = _lib.load()
    g = _fake_graph()
    st = _lib.OgStats()
    d = ctypes.c_void_p(0x4000)
    ws = ctypes.c_void_p(0x10000)
    big = ctypes.c_size_t(1 << 40)
    E = og.OG_ERR_INVALID_ARG
    both = og.Schedule(delta=4, update=og.OG_LAZY_UPDATE,
                       flags=og.OG_FLAG_DENSE_PULL | og.OG_FLAG_HYBRID_DIRECTION).to_c()
    assert lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(both), d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(both)) == 0
    for fl in (og.OG_FLAG_DENSE_PULL, og.OG_FLAG_HYBRID_DIRECTION):
        eager = og.Schedule(delta=4, flags=fl).to_c()
        assert lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(eager), d, None, ws, big, ctypes.byref(st), None) == E
        assert lib.og_kcore(ctypes.byref(g), ctypes.byref(eager), d, ws, big, ctypes.byref(st), None) == E
        split = og.Schedule(delta=4, update=og.OG_LAZY_UPDATE, flags=fl | og.OG_FLAG_LIGHT_HEAVY).to_c()
        assert lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(split), d, None, ws, big, ctypes.byref(st), None) == E
        # float32 weights have no pull instantiation
        lazy = og.Schedule(delta=4, update=og.OG_LAZY_UPDATE, flags=fl).to_c()
        gf = _lib.OgGraphF32(10, 20, 0x1000, 0x2000, 0x3000)
        assert lib.og_sssp_f32(ctypes.byref(gf), 0, ctypes.byref(lazy), d, None, None, ws, big,
                               ctypes.byref(st), None) == E


def test_invalid_calls_rejected():
    lib = _lib.load()
    g = _fake_graph()
    sc = og.Schedule(delta=4).to_c()
    st = _lib.OgStats()
    ws = ctypes.c_void_p(0x10000)
    big = ctypes.c_size_t(1 << 40)
    d = ctypes.c_void_p(0x4000)
    E = og.OG_ERR_INVALID_ARG
    assert lib.og_sssp(ctypes.byref(g), -1, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_sssp(ctypes.byref(g), 10, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_sssp(None, 0, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_sssp(ctypes.byref(g), 0, None, d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(sc), None, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(sc), d, None, None, big, ctypes.byref(st), None) == E
    # misaligned workspace
    assert lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(sc), d, None, ctypes.c_void_p(0x10008), big,
                       ctypes.byref(st), None) == E
    # ppsp / astar targets and estimate
    assert lib.og_ppsp(ctypes.byref(g), 0, 10, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_ppsp(ctypes.byref(g), 0, -1, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st), None) == E
    assert lib.og_astar(ctypes.byref(g), 0, 3, None, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st),
                        None) == E
    # bad graphs
    for bad in (_lib.OgGraph(5, 3, None, 0x1, 0x1), _lib.OgGraph(5, 3, 0x1, None, 0x1),
                _lib.OgGraph(5, -1, 0x1, 0x1, 0x1), _lib.OgGraph(5, 1 << 31, 0x1, 0x1, 0x1)):
        assert lib.og_sssp(ctypes.byref(bad), 0, ctypes.byref(sc), d, None, ws, big, ctypes.byref(st),
                           None) == E


def test_workspace_too_small():
    lib = _lib.load()
    g = _fake_graph()
    sc = og.Schedule(delta=4).to_c()
    st = _lib.OgStats()
    need = lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(sc))
    rc = lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(sc), ctypes.c_void_p(0x4000), None,
                     ctypes.c_void_p(0x10000), ctypes.c_size_t(need - 256), ctypes.byref(st), None)
    assert rc == og.OG_ERR_WORKSPACE


def test_binding_argument_checks_survive_optimisation():
    """Wrong tensor types are rejected by a raised ValueError, not an
    assert that python -O would strip (CPU tensors: nothing is launched)."""
    import torch
    rp = torch.tensor([0, 1, 2], dtype=torch.int64)
    col = torch.tensor([1, 0], dtype=torch.int32)
    w = torch.tensor([3, 3], dtype=torch.int32)
    og.DeviceGraph(rp, col, w)  # well formed
    with pytest.raises(ValueError):
        og.DeviceGraph(rp.to(torch.int32), col, w)
    with pytest.raises(ValueError):
        og.DeviceGraph(rp, col.to(torch.int64), w)
    with pytest.raises(ValueError):
        og.DeviceGraph(rp, col, w.to(torch.float32))
    with pytest.raises(ValueError):
        og.DeviceGraph(rp, col, w[:1])
    with pytest.raises(ValueError):
        og.DeviceGraph(torch.zeros(1, dtype=torch.int64), col[:0], w[:0])
    src = open(os.path.join(ROOT, "paper_1911_07260_amd", "__init__.py")).read()
    src += open(os.path.join(ROOT, "paper_1911_07260_amd", "diff.py")).read()
    assert not re.search(r"^\s*assert\b", src, flags=re.M)


@pytest.mark.parametrize("kw", [
    dict(update=og.OG_EAGER_NO_FUSION), dict(update=og.OG_LAZY_UPDATE),
    dict(engine=og.OG_ENGINE_HOST_ROUNDS), dict(engine=og.OG_ENGINE_GRAPH_ROUNDS),
])
def test_vertex_blocks_need_fused_persistent(kw):
    """The vertex-block engine is bucket fusion in a persistent launch: any
    other update or engine is rejected before anything is launched."""
    lib = _lib.load()
    g = _fake_graph()
    sc = og.Schedule(delta=4, flags=og.OG_FLAG_VERTEX_BLOCKS, **kw).to_c()
    st = _lib.OgStats()
    rc = lib.og_sssp(ctypes.byref(g), 0, ctypes.byref(sc), ctypes.c_void_p(0x4000), None,
                     ctypes.c_void_p(0x10000), ctypes.c_size_t(1 << 40), ctypes.byref(st), None)
    assert rc == og.OG_ERR_INVALID_ARG


def test_vertex_blocks_single_query_only():
    """Batches and A* estimates are rejected with the block engine."""
    import numpy as np
    lib = _lib.load()
    g = _fake_graph()
    sc = og.Schedule(delta=4, flags=og.OG_FLAG_VERTEX_BLOCKS).to_c()
    st = _lib.OgStats()
    srcs = np.array([0, 1], dtype=np.int32)
    rc = lib.og_sssp_batch(ctypes.byref(g), ctypes.c_void_p(srcs.ctypes.data), 2, ctypes.byref(sc),
                           ctypes.c_void_p(0x4000), None, ctypes.c_void_p(0x10000), ctypes.c_size_t(1 << 40),
                           ctypes.byref(st), None)
    assert rc == og.OG_ERR_INVALID_ARG
    rc = lib.og_astar(ctypes.byref(g), 0, 1, ctypes.c_void_p(0x8000), ctypes.byref(sc), ctypes.c_void_p(0x4000),
                      None, ctypes.c_void_p(0x10000), ctypes.c_size_t(1 << 40), ctypes.byref(st), None)
    assert rc == og.OG_ERR_INVALID_ARG


def test_vertex_blocks_workspace_bytes():
    """The block engine's workspace: the plain layout, then the blocked copy
    (block starts, per-block offsets and sizes, vertices in block order,
    block of each vertex, internal
    and leaving row offsets, internal edges, leaving edges' targets, weights
    and target blocks), the per-query state (processed labels, block states,
    a ring of a power of two above n entries) and the build's temporaries."""
    lib = _lib.load()
    for n, m in ((1000, 4000), (4096, 16128), (5000, 100_000)):
        g = _fake_graph(n, m)
        plain = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000).to_c()
        blk = og.Schedule(delta=4, window_buckets=8, queue_capacity=5000, flags=og.OG_FLAG_VERTEX_BLOCKS).to_c()
        base = lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(plain))

        def v(nbytes):
            return (nbytes + 255) // 256 * 256

        ring = 1
        while ring < n + 1:
            ring *= 2
        copy = v(4 * (n + 1)) + v(16 * n) + 2 * v(4 * n) + 2 * v(4 * (n + 1)) + 4 * v(4 * m)
        query = 2 * v(4 * n) + v(8 * ring)
        build = (v(8 * n) + 3 * v(4 * n) + v(8 * n) + v(4 * n) + 2 * v(4 * (n + 1)) + 2 * v(4 * n)
                 + 2 * v(4 * (n + 1)) + v(4 * ((n + 1) // 2048 + 2)) + 256)
        assert lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(blk)) == base + copy + query + build


def test_noalloc_refusals_need_no_gpu():
    """og_sssp_noalloc refuses, before touching the device, a schedule that
    would create HIP objects and a graph whose workspace exceeds its fixed
    array."""
    lib = _lib.load()
    st = _lib.OgStats()
    small = _fake_graph(100, 400)
    for sc in (og.Schedule(delta=4, flags=og.OG_FLAG_TIMING), og.Schedule(delta=4, engine=og.OG_ENGINE_GRAPH_ROUNDS),
               og.Schedule(delta=0)):
        c = sc.to_c()
        rc = lib.og_sssp_noalloc(ctypes.byref(small), 0, ctypes.byref(c), ctypes.c_void_p(0x4000), None,
                                 ctypes.byref(st), None)
        assert rc == og.OG_ERR_INVALID_ARG and st.status == rc
    big = _fake_graph(4_000_000, 16_000_000)
    c = og.Schedule(delta=4).to_c()
    assert lib.og_workspace_bytes(ctypes.byref(big), ctypes.byref(c)) > og.OG_SCRATCH_BYTES
    rc = lib.og_sssp_noalloc(ctypes.byref(big), 0, ctypes.byref(c), ctypes.c_void_p(0x4000), None,
                             ctypes.byref(st), None)
    assert rc == og.OG_ERR_WORKSPACE and st.status == rc
