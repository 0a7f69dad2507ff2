"""Pins for the CPU oracle: it is checked against things other than itself.

* exhaustive simple-path enumeration on tiny graphs (the definition itself),
* Bellman-Ford brute force and scipy's independent Dijkstra,
* closed forms (uniform grid -> scaled Manhattan distance, path -> prefix
  sums, unit weights -> breadth-first depth),
* a hand-worked 3x3 grid fixture (tests/golden/grid3x3.txt),
* planted bugs in the oracle's source, each of which must fail a pin.
"""
import itertools
import os
from collections import deque

import numpy as np
import pytest

import graphgen as gg
import oracle

INF64 = oracle.INF64
INF32 = oracle.INF32
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_graph(rng, n, p, wlo, whi, directed=True):
    src, dst, w = [], [], []
    for u in range(n):
        for v in range(n):
            if u != v and rng.random() < p:
                src.append(u)
                dst.append(v)
                w.append(int(rng.integers(wlo, whi)))
    if not directed:
        src, dst, w = src + dst, dst + src, w + w
    return gg.from_edges(n, src, dst, w)


def brute_force_paths(g, s):
    """min over simple s->v paths of the weight sum, by enumeration."""
    n = g.n
    best = [INF64] * n
    best[s] = 0
    adj = [[(int(g.col[e]), int(g.w[e])) for e in range(g.row_ptr[u], g.row_ptr[u + 1])] for u in range(n)]

    def dfs(u, d, seen):
        for v, w in adj[u]:
            if v in seen:
                continue
            nd = d + w
            if nd < best[v]:
                best[v] = nd
            seen.add(v)
            dfs(v, nd, seen)
            seen.discard(v)

    dfs(s, 0, {s})
    return np.array(best, dtype=np.int64)


def brute_force_pred(g, s, d):
    n = g.n
    pred = np.full(n, -1, dtype=np.int32)
    for u in range(n):
        if d[u] == INF64:
            continue
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[e])
            if v != s and d[v] != INF64 and d[u] + int(g.w[e]) == d[v]:
                if pred[v] < 0 or u < pred[v]:
                    pred[v] = u
    pred[s] = s
    return pred


def load_golden(name):
    edges, vals = [], {}
    mode = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            if line == "edges":
                mode = "edges"
                continue
            head, *rest = line.split()
            if head in ("source", "dist", "pred"):
                vals[head] = [int(x) for x in rest]
                mode = None
            elif mode == "edges":
                edges.append(tuple(int(x) for x in line.split()))
    return edges, vals


def test_enumeration_tiny(orc):
    rng = np.random.default_rng(7)
    for trial in range(150):
        n = int(rng.integers(2, 7))
        g = random_graph(rng, n, 0.45, 0, 6)
        s = int(rng.integers(0, n))
        ref = brute_force_paths(g, s)
        assert np.array_equal(orc.dijkstra64(g, s), ref), trial
        d = orc.dijkstra64(g, s)
        assert np.array_equal(orc.canonical_pred(g, s, d), brute_force_pred(g, s, d)), trial


@pytest.mark.parametrize("wlo,whi", [(0, 4), (1, 100), (0, 1)])
def test_bellman_ford_random(orc, wlo, whi):
    rng = np.random.default_rng(11 + whi)
    for trial in range(300):
        n = int(rng.integers(1, 65))
        p = float(rng.choice([0.02, 0.08, 0.3]))
        g = random_graph(rng, n, p, wlo, whi, directed=bool(trial % 2))
        s = int(rng.integers(0, n))
        assert np.array_equal(orc.dijkstra64(g, s), orc.bellman_ford64(g, s)), trial


def test_scipy_independent(orc):
    sp = pytest.importorskip("scipy.sparse")
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    rng = np.random.default_rng(3)
    for trial in range(20):
        g = gg.rgg(int(rng.integers(200, 3000)), 6.0, seed=trial)[0]
        mat = sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.n, g.n))
        s = int(rng.integers(0, g.n))
        ref = csgraph.dijkstra(mat, directed=True, indices=s)
        mine = orc.dijkstra64(g, s)
        fin = np.isfinite(ref)
        assert np.array_equal(fin, mine != INF64)
        assert np.array_equal(ref[fin].astype(np.int64), mine[fin])


@pytest.mark.parametrize("c", [1, 7])
def test_closed_form_uniform_grid(orc, c):
    R, C = 17, 23
    g = gg.grid(R, C, 1, 2, seed=0)
    g = gg.with_weights(g, np.full(g.m, c, dtype=np.int32))
    for s in (0, 8 * C + 11, R * C - 1):
        d = orc.dijkstra64(g, s)
        rs, cs = divmod(s, C)
        r, cc = np.divmod(np.arange(R * C), C)
        assert np.array_equal(d, c * (np.abs(r - rs) + np.abs(cc - cs)))


def test_closed_form_path(orc):
    rng = np.random.default_rng(5)
    k = 200
    w = rng.integers(0, 1000, size=k - 1)
    g = gg.from_edges(k, np.arange(k - 1), np.arange(1, k), w)
    d = orc.dijkstra64(g, 0)
    assert np.array_equal(d, np.concatenate([[0], np.cumsum(w)]))
    d = orc.dijkstra64(g, k - 1)  # directed path: nothing reachable backwards
    assert d[k - 1] == 0 and np.all(d[:-1] == INF64)


def test_closed_form_unit_weights_bfs_depth(orc):
    g = gg.rmat(10, 8, seed=4)
    g = gg.with_weights(g, np.ones(g.m, dtype=np.int32))
    s = int(np.argmax(g.degrees()))
    depth = np.full(g.n, -1)
    depth[s] = 0
    q = deque([s])
    while q:
        u = q.popleft()
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            if depth[v] < 0:
                depth[v] = depth[u] + 1
                q.append(v)
    d = orc.dijkstra64(g, s)
    assert np.array_equal(np.where(d == INF64, -1, d), depth)


def test_hand_worked_grid(orc):
    edges, vals = load_golden("grid3x3.txt")
    u, v, w = zip(*edges)
    g = gg.from_edges(9, list(u) + list(v), list(v) + list(u), list(w) + list(w))
    s = vals["source"][0]
    d32, p = orc.sssp(g, s)
    assert d32.tolist() == vals["dist"]
    assert p.tolist() == vals["pred"]
    assert orc.check(g, s, d32, p) == 0


def test_unreachable_and_int32(orc):
    g = gg.from_edges(5, [0, 1, 3], [1, 2, 4], [5, 2**31 - 4, 1])
    d64 = orc.dijkstra64(g, 0)
    assert d64.tolist() == [0, 5, 2**31 + 1, INF64, INF64]
    d32, over = orc.to_i32(d64)
    assert over == 1 and d32[2] == INF32 and d32[3] == INF32
    g2 = gg.from_edges(3, [0, 1], [1, 2], [5, 2**31 - 7])
    d32, over = orc.to_i32(orc.dijkstra64(g2, 0))
    assert over == 0 and d32.tolist() == [0, 5, 2**31 - 2]
    g3 = gg.from_edges(3, [0, 1], [1, 2], [5, 2**31 - 6])  # sum == INT32_MAX: not representable
    d32, over = orc.to_i32(orc.dijkstra64(g3, 0))
    assert over == 1


def test_ppsp_and_astar(orc):
    g = gg.road(96, seed=2)
    rng = np.random.default_rng(0)
    for _ in range(12):
        s, t = (int(x) for x in rng.integers(0, g.n, size=2))
        full = orc.dijkstra64(g, s)
        want = -1 if full[t] == INF64 else int(full[t])
        assert orc.ppsp(g, s, t) == want
        h0 = np.zeros(g.n, dtype=np.int32)
        assert orc.astar(g, s, t, h0)[0] == want
        h = gg.grid_heuristic(96, t)
        got, expanded = orc.astar(g, s, t, h)
        assert got == want
        assert expanded <= orc.astar(g, s, t, h0)[1]


def test_grid_heuristic_consistent():
    """floor(10*euclid) never exceeds w(u,v) + h(v) on the road generator's
    edges (the long-range weight floor makes it consistent), so A* stays
    exact."""
    side = 128
    g = gg.road(side, seed=9)
    t = 5000
    h = gg.grid_heuristic(side, t).astype(np.int64)
    src = np.repeat(np.arange(g.n), g.degrees())
    assert np.all(h[src] <= g.w.astype(np.int64) + h[g.col])
    assert h[t] == 0


def mutation_detected(m, orc_ok):
    """True if some pin distinguishes mutated oracle m from the definition."""
    bad = oracle.mutated(m)
    rng = np.random.default_rng(100 + m)
    for trial in range(60):
        n = int(rng.integers(2, 7))
        g = random_graph(rng, n, 0.5, 1, 6)
        s = int(rng.integers(0, n))
        ref = brute_force_paths(g, s)
        d = bad.dijkstra64(g, s)
        if not np.array_equal(d, ref):
            return True
        if not np.array_equal(bad.canonical_pred(g, s, ref), brute_force_pred(g, s, ref)):
            return True
    return False


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_planted_bugs_are_caught(orc, m):
    assert mutation_detected(m, orc), f"planted oracle bug {m} slipped through the pins"
