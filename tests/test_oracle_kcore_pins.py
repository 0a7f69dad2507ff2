"""Pins for the k-core oracle (section 6.1, k-core decomposition).

The oracle peels a vertex of minimum remaining degree at a time.  It is
checked against:
* the definition itself on tiny random graphs: for every k, the k-core is
  what remains after repeatedly deleting vertices with fewer than k live
  neighbours, and coreness[v] is the largest k whose k-core keeps v;
* closed forms: complete graphs, cycles, paths, stars, complete bipartite
  graphs, full grids, the Petersen graph;
* a hand-worked fixture (tests/golden/kcore8.txt);
* the certificate on generated graphs: every v keeps at least core[v]
  neighbours u with core[u] >= core[v];
* a planted bug (the peeling level allowed to go down) that these pins catch.
"""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def undirected(n, pairs):
    pairs = [(int(a), int(b)) for a, b in pairs]
    src = [a for a, b in pairs] + [b for a, b in pairs]
    dst = [b for a, b in pairs] + [a for a, b in pairs]
    return gg.from_edges(n, src, dst, np.ones(len(src), dtype=np.int64))


def core_by_definition(g):
    n = g.n
    nbrs = [g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist() for v in range(n)]
    core = np.zeros(n, dtype=np.int32)
    for k in range(1, n + 1):
        alive = np.ones(n, dtype=bool)
        changed = True
        while changed:
            changed = False
            for v in range(n):
                if alive[v] and sum(alive[u] for u in nbrs[v]) < k:
                    alive[v] = False
                    changed = True
        if not alive.any():
            break
        core[alive] = k
    return core


def random_simple(rng, n, p):
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    return undirected(n, pairs)


def certificate_ok(g, core):
    src = np.repeat(np.arange(g.n), g.degrees())
    strong = core[g.col] >= core[src]
    support = np.bincount(src[strong], minlength=g.n)
    return bool(np.all(support >= core))


def test_definition_brute_force(orc):
    rng = np.random.default_rng(31)
    for trial in range(150):
        n = int(rng.integers(1, 11))
        g = random_simple(rng, n, float(rng.uniform(0.1, 0.9)))
        assert np.array_equal(orc.kcore(g), core_by_definition(g)), trial


def test_closed_forms(orc):
    for n in (2, 3, 5, 9):
        k = undirected(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
        assert orc.kcore(k).tolist() == [n - 1] * n
    for n in (3, 4, 10):
        assert orc.kcore(undirected(n, [(i, (i + 1) % n) for i in range(n)])).tolist() == [2] * n
        assert orc.kcore(undirected(n, [(i, i + 1) for i in range(n - 1)])).tolist() == [1] * n
        assert orc.kcore(undirected(n + 1, [(0, i) for i in range(1, n + 1)])).tolist() == [1] * (n + 1)
    for a, b in ((1, 4), (2, 3), (3, 3), (4, 6)):
        kab = undirected(a + b, [(i, a + j) for i in range(a) for j in range(b)])
        assert orc.kcore(kab).tolist() == [min(a, b)] * (a + b)
    for r, c in ((2, 2), (3, 5), (8, 8)):
        g = gg.grid(r, c, 1, 2, seed=0) if r == c else None
        pairs = [(i * c + j, i * c + j + 1) for i in range(r) for j in range(c - 1)]
        pairs += [(i * c + j, (i + 1) * c + j) for i in range(r - 1) for j in range(c)]
        assert orc.kcore(undirected(r * c, pairs)).tolist() == [2] * (r * c)
        if g is not None:
            assert orc.kcore(g).tolist() == [2] * (r * c)
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    assert orc.kcore(undirected(10, outer + spokes + inner)).tolist() == [3] * 10
    assert orc.kcore(undirected(4, [])).tolist() == [0] * 4


def test_hand_worked_fixture(orc):
    pairs, n, want = [], None, None
    with open(os.path.join(GOLDEN, "kcore8.txt")) as f:
        mode = None
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            if line == "edges":
                mode = "edges"
                continue
            head, *rest = line.split()
            if head == "n":
                n = int(rest[0])
            elif head == "core":
                want = [int(x) for x in rest]
            elif mode == "edges":
                pairs.append((int(head), int(rest[0])))
    assert orc.kcore(undirected(n, pairs)).tolist() == want


@pytest.mark.parametrize("kind", ["road", "rmat"])
def test_certificate_on_generated(orc, kind):
    g = gg.road(128, seed=3) if kind == "road" else gg.rmat(12, 16, seed=4)
    core = orc.kcore(g)
    assert certificate_ok(g, core)
    # maximality: peeling {core >= k} with threshold k + 1 by the definition
    # leaves exactly {core >= k + 1}
    src = np.repeat(np.arange(g.n), g.degrees())
    for k in sorted(set(np.unique(core).tolist()))[:6]:
        alive = core >= k
        while True:
            live_deg = np.bincount(src[alive[src] & alive[g.col]], minlength=g.n)
            drop = alive & (live_deg < k + 1)
            if not drop.any():
                break
            alive &= ~drop
        assert np.array_equal(alive, core >= k + 1), k


def test_planted_bug_is_caught(orc):
    bad = oracle.mutated(5)
    rng = np.random.default_rng(77)
    caught = False
    for trial in range(150):
        g = random_simple(rng, int(rng.integers(2, 11)), float(rng.uniform(0.2, 0.9)))
        if not np.array_equal(bad.kcore(g), core_by_definition(g)):
            caught = True
            break
    assert caught, "planted k-core bug slipped through the pins"
