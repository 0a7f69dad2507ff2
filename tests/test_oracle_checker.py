"""The certificate checker fires on each kind of corrupted result."""
import numpy as np
import pytest

import graphgen as gg
import oracle

INF32 = oracle.INF32


@pytest.fixture(scope="module")
def case(orc):
    g = gg.road(40, seed=1)
    s = int(gg.pick_sources(g, 1, seed=1)[0])
    d, p = orc.sssp(g, s)
    assert orc.check(g, s, d, p) == 0
    return g, s, d, p


def bits(orc, g, s, d, p):
    return orc.check(g, s, d, p)


def test_clean(orc, case):
    g, s, d, p = case
    assert bits(orc, g, s, d, p) == 0
    assert bits(orc, g, s, d, None) == 0


def test_src_nonzero(orc, case):
    g, s, d, p = case
    d2 = d.copy()
    d2[s] = 1
    assert bits(orc, g, s, d2, None) & (1 << 0)


def test_not_relaxed(orc, case):
    g, s, d, p = case
    v = int(np.nonzero((d != INF32) & (np.arange(g.n) != s))[0][5])
    d2 = d.copy()
    d2[v] += 1000
    assert bits(orc, g, s, d2, None) & (1 << 1)


def test_too_small_breaks_tightness(orc, case):
    g, s, d, p = case
    v = int(np.nonzero((d != INF32) & (np.arange(g.n) != s))[0][7])
    d2 = d.copy()
    d2[v] -= 1
    assert bits(orc, g, s, d2, p) & ((1 << 7) | (1 << 1))


def test_negative(orc, case):
    g, s, d, p = case
    d2 = d.copy()
    d2[int(np.nonzero(d == INF32)[0][0])] = -3
    assert bits(orc, g, s, d2, None) & (1 << 2)


def test_reachability(orc, case):
    g, s, d, p = case
    d2 = d.copy()
    unreach = int(np.nonzero(d == INF32)[0][0])
    d2[unreach] = 5
    assert bits(orc, g, s, d2, None) & (1 << 3)


def test_pred_errors(orc, case):
    g, s, d, p = case
    reach = np.nonzero((d != INF32) & (np.arange(g.n) != s))[0]
    p2 = p.copy(); p2[s] = -1
    assert bits(orc, g, s, d, p2) & (1 << 4)
    p2 = p.copy(); p2[reach[3]] = -1
    assert bits(orc, g, s, d, p2) & (1 << 5)
    p2 = p.copy(); p2[int(np.nonzero(d == INF32)[0][0])] = s
    assert bits(orc, g, s, d, p2) & (1 << 6)
    p2 = p.copy(); p2[reach[3]] = (reach[3] + 2) % g.n
    assert bits(orc, g, s, d, p2) & (1 << 7)
    p2 = p.copy(); p2[reach[3]] = g.n + 5
    assert bits(orc, g, s, d, p2) & (1 << 9)


def test_pred_cycle(orc):
    # zero-weight 2-cycle hanging off the source: tight edges but no root
    g = gg.from_edges(3, [0, 1, 2], [1, 2, 1], [4, 0, 0])
    d = np.array([0, 4, 4], dtype=np.int32)
    p = np.array([0, 2, 1], dtype=np.int32)
    assert orc.check(g, 0, d, p) & (1 << 8)
    p_ok = np.array([0, 0, 1], dtype=np.int32)
    assert orc.check(g, 0, d, p_ok) == 0
