"""Pins for the real-valued (float32-weight) oracle functions.

* float64 Dijkstra == exact rational shortest paths (path enumeration with
  fractions.Fraction) on tiny graphs;
* float32-arithmetic Dijkstra == a numpy float32 Bellman-Ford fixed point;
* the tree is tight in the matching arithmetic and uses the smallest
  tight predecessor;
* subtree gradients == central finite differences of the float64 loss
  (h = 1e-2) wherever the tree is stable, and == brute-force path counts.
"""
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg


def rand_graph(rng, n, p):
    src, dst = [], []
    for u in range(n):
        for v in range(n):
            if u != v and rng.random() < p:
                src.append(u)
                dst.append(v)
    g = gg.from_edges(n, src, dst, np.zeros(len(src), dtype=np.int64))
    w = rng.uniform(1.0, 20.0, size=g.m).astype(np.float32)
    return g, w


def exact_paths(g, w, s):
    best = [None] * g.n
    best[s] = Fraction(0)
    adj = [[(int(g.col[e]), Fraction(float(w[e]))) for e in range(g.row_ptr[u], g.row_ptr[u + 1])] for u in range(g.n)]

    def dfs(u, d, seen):
        for v, wt in adj[u]:
            if v in seen:
                continue
            nd = d + wt
            if best[v] is None or nd < best[v]:
                best[v] = nd
            seen.add(v)
            dfs(v, nd, seen)
            seen.discard(v)

    dfs(s, Fraction(0), {s})
    return best


def f32_bellman_ford(g, w, s):
    d = np.full(g.n, np.inf, dtype=np.float32)
    d[s] = np.float32(0)
    src = np.repeat(np.arange(g.n), g.degrees())
    for _ in range(g.n + 1):
        cand = (d[src] + w).astype(np.float32)  # float32 + float32: one rounding
        nd = d.copy()
        np.minimum.at(nd, g.col, cand)
        if np.array_equal(nd, d):
            break
        d = nd
    return d


def test_f64_equals_exact_rationals(orc):
    rng = np.random.default_rng(21)
    for trial in range(120):
        g, w = rand_graph(rng, int(rng.integers(2, 7)), 0.5)
        s = int(rng.integers(0, g.n))
        d = orc.dijkstra_real(g, w, s, f32=False)
        ex = exact_paths(g, w, s)
        for v in range(g.n):
            if ex[v] is None:
                assert np.isinf(d[v])
            else:
                assert Fraction(d[v]) == ex[v], (trial, v)


def test_f32_equals_numpy_float32_fixed_point(orc):
    rng = np.random.default_rng(22)
    for trial in range(40):
        g = gg.rgg(int(rng.integers(50, 400)), 5.0, seed=trial)[0]
        w = gg.float_weights(g, 1.0, 1000.0, seed=trial)
        s = int(rng.integers(0, g.n))
        d = orc.dijkstra_real(g, w, s, f32=True)
        ref = f32_bellman_ford(g, w, s)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(d), fin)
        assert np.array_equal(d[fin].astype(np.float32), ref[fin]), trial


@pytest.mark.parametrize("f32", [False, True])
def test_tree_is_canonical_and_tight(orc, f32):
    g = gg.road(64, seed=4)
    w = gg.float_weights(g, seed=4)
    s = 100
    d = orc.dijkstra_real(g, w, s, f32)
    p, pe = orc.tree_real(g, w, s, d, f32)
    assert p[s] == s and pe[s] == -1
    src = np.repeat(np.arange(g.n), g.degrees())
    if f32:
        tight = (d[src].astype(np.float32) + w).astype(np.float32) == d[g.col].astype(np.float32)
    else:
        tight = d[src] + w.astype(np.float64) == d[g.col]
    tight &= np.isfinite(d[src]) & (g.col != s)
    want = np.full(g.n, -1)
    for e in np.nonzero(tight)[0]:
        v, u = g.col[e], src[e]
        if want[v] < 0 or u < want[v]:
            want[v] = u
    want[s] = s
    assert np.array_equal(p, want)
    has = pe >= 0
    assert np.array_equal(src[pe[has]], p[has]) and np.array_equal(g.col[pe[has]], np.nonzero(has)[0])


def loss64(orc, g, w, s, targets):
    d = orc.dijkstra_real(g, w, s, f32=False)
    return float(np.sum(d[targets]))


def test_subtree_grad_matches_finite_differences(orc):
    g = gg.road(24, seed=6)
    w = gg.float_weights(g, seed=6)
    s = 5
    rng = np.random.default_rng(7)
    targets = rng.integers(0, g.n, size=40)
    d = orc.dijkstra_real(g, w, s, f32=False)
    targets = targets[np.isfinite(d[targets])]
    p, pe = orc.tree_real(g, w, s, d, f32=False)
    up = np.bincount(targets, minlength=g.n).astype(np.float64)
    grad = orc.subtree_grad(g, d, p, pe, up)
    # brute force: count targets whose tree path uses each edge
    bf = np.zeros(g.m)
    for t in targets:
        v = int(t)
        while pe[v] >= 0:
            bf[pe[v]] += 1
            v = int(p[v])
    assert np.array_equal(grad, bf)
    h = 1e-2
    checked = 0
    for e in rng.choice(g.m, size=120, replace=False):
        wp, wm = w.astype(np.float64).copy(), w.astype(np.float64).copy()
        wp[e] += h
        wm[e] -= h
        fd = (loss64(orc, g, wp.astype(np.float32), s, targets) - loss64(orc, g, wm.astype(np.float32), s,
                                                                         targets))
        # the float32 cast of w +- h moves w_e by a few ulps off +-h
        step = float(np.float32(wp[e]) - np.float32(wm[e]))
        fd /= step
        if abs(fd - round(fd)) < 1e-3:  # tree stable over [w - h, w + h]
            assert abs(fd - grad[e]) <= 1e-3 * max(1.0, abs(grad[e])), (e, fd, grad[e])
            checked += 1
    assert checked > 100


def test_float_weights_symmetric():
    g = gg.road(32, seed=1)
    w = gg.float_weights(g, 1.0, 1000.0, seed=2)
    assert w.dtype == np.float32 and w.min() >= 1.0 and w.max() < 1000.0
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    fwd = {(int(a), int(b)): x for a, b, x in zip(src, g.col, w)}
    assert all(fwd[(b, a)] == x for (a, b), x in fwd.items())
    assert len(np.unique(w)) > 0.99 * (g.m // 2)
