"""Generator properties: sizes, symmetry, simple graphs, ranges, determinism."""
import numpy as np
import pytest

import graphgen as gg


def assert_simple_symmetric(g):
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.col.astype(np.int64)
    assert np.all(src != dst), "self-loop"
    key = src * g.n + dst
    # rows sorted by destination and no duplicates
    assert np.all(np.diff(key) > 0)
    rkey = dst * g.n + src
    order = np.argsort(rkey)
    assert np.array_equal(rkey[order], key), "not symmetric"
    assert np.array_equal(g.w[order], g.w), "asymmetric weights"


def test_grid_config0_exact():
    g = gg.grid(64, 64, 1, 100, seed=0)
    assert g.n == 4096 and g.m == 16128
    assert g.w.min() >= 1 and g.w.max() <= 99
    assert_simple_symmetric(g)
    g2 = gg.grid(64, 64, 1, 100, seed=0)
    assert np.array_equal(g.w, g2.w) and np.array_equal(g.col, g2.col)
    g3 = gg.grid(64, 64, 1, 100, seed=1)
    assert not np.array_equal(g.w, g3.w)


def test_road_small():
    g = gg.road(256, seed=0)
    assert g.n == 65536
    assert_simple_symmetric(g)
    grid_edges = 2 * 256 * 255
    und = g.m // 2
    assert 0.73 * grid_edges < und < 0.77 * grid_edges
    assert g.w.min() >= 10
    assert gg.road(256, seed=0).w.tolist() == g.w.tolist()


@pytest.mark.slow
def test_road_full_size():
    g = gg.road(4096, seed=0)
    assert g.n == 16_777_216
    expect = 2 * 0.75 * 2 * 4096 * 4095
    assert abs(g.m - expect) / expect < 0.01
    assert g.degrees().max() <= 8
    # long-range edges: weight above a unit grid step's maximum of 20
    assert (g.w > 20).sum() > 0


def test_rmat_small():
    g = gg.rmat(12, 16, seed=0)
    assert g.n == 4096
    assert_simple_symmetric(g)
    assert 1 <= g.w.min() and g.w.max() <= 999
    d = g.degrees()
    assert d.max() > 20 * d.mean()  # skewed


def test_rgg():
    g, x, y = gg.rgg(5000, 6.0, seed=1)
    assert_simple_symmetric(g)
    assert 4.5 < g.m / g.n < 7.5
    src = np.repeat(np.arange(g.n), g.degrees())
    L = np.sqrt((x[src] - x[g.col]).astype(np.float64) ** 2 + (y[src] - y[g.col]).astype(np.float64) ** 2)
    assert np.array_equal(g.w, np.maximum(1, np.floor(L + 0.5)).astype(np.int32))  # llround, half away from 0


def test_uniform_and_sources():
    a = gg.uniform(1, 5, 1000, 17)
    assert a.min() >= 0 and a.max() < 17
    assert np.array_equal(a, gg.uniform(1, 5, 1000, 17))
    g = gg.road(64, seed=0)
    s = gg.pick_sources(g, 8, seed=1)
    assert np.all(g.degrees()[s] >= 1)
