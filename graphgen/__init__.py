"""Seeded synthetic graph inputs (CSR, numpy arrays).

The generators live in ``graphgen.cpp`` (built into ``libgraphgen.so`` by
``build()``); this module only marshals arguments.  It is shared by the
oracle's tests and by the GPU path's tests and benchmark, and it contains no
shortest-path arithmetic.

Workload recipes (all integer weights, symmetric directed CSR):

* ``grid(64, 64, 1, 100, seed=0)``: full 4-neighbour grid, 4,096 vertices,
  16,128 directed edges, weights uniform in [1, 100).
* ``road(4096, seed=0)``: road-like percolated grid, 16,777,216 vertices,
  p_keep 0.75, 0.1 % long-range edges within 64 grid steps, weights
  ``llround(10 * len * U(1, 2))`` (long-range weights at least
  ``ceil(10 * len)``).
* ``rmat(24, 16, seed=0)``: R-MAT (0.57, 0.19, 0.19, 0.05), symmetrised,
  deduplicated, no self-loops.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.cpp")

# Random streams used by ``uniform`` (sources, targets, pairs).
STREAM_SOURCES = 101
STREAM_TARGETS = 102
STREAM_PAIRS = 103


def build() -> str:
    """Compile libgraphgen.so (g++, OpenMP)."""
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _SO + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    vp = ctypes.c_void_p
    lib.gg_n.restype = ctypes.c_int32
    lib.gg_n.argtypes = [vp]
    lib.gg_m.restype = ctypes.c_int64
    lib.gg_m.argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, vp, vp, vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_grid.restype = vp
    lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
    lib.gg_road.restype = vp
    lib.gg_road.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_uint64]
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
    lib.gg_rgg.restype = vp
    lib.gg_rgg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, vp, vp]
    lib.gg_grid_heuristic.restype = None
    lib.gg_grid_heuristic.argtypes = [ctypes.c_int32, ctypes.c_int32, vp]
    lib.gg_uniform.restype = None
    lib.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint64, vp]
    _lib = lib
    return lib


@dataclass
class Graph:
    """Directed CSR graph: row v's out-edges are col[row_ptr[v]:row_ptr[v+1]]
    with weights w[...], sorted by destination."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[m]
    w: np.ndarray        # int32[m]
    name: str = ""
    side: int = 0        # grid side for grid-based graphs (vertex (r,c) = r*side+c)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _take(handle, name: str, side: int = 0) -> Graph:
    lib = _load()
    if not handle:
        raise ValueError(f"graphgen: invalid arguments for {name}")
    try:
        n = lib.gg_n(handle)
        m = lib.gg_m(handle)
        row_ptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(max(m, 1), dtype=np.int32)
        w = np.empty(max(m, 1), dtype=np.int32)
        lib.gg_copy(handle, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data)
    finally:
        lib.gg_free(handle)
    return Graph(n=n, row_ptr=row_ptr, col=col[:m], w=w[:m], name=name, side=side)


def grid(rows: int, cols: int, wlo: int = 1, whi: int = 100, seed: int = 0) -> Graph:
    return _take(_load().gg_grid(rows, cols, wlo, whi, seed), f"grid{rows}x{cols}",
                 side=cols if rows == cols else 0)


def road(side: int, seed: int = 0, p_keep: float = 0.75, lr_frac: float = 0.001,
         lr_radius: int = 64) -> Graph:
    return _take(_load().gg_road(side, p_keep, lr_frac, lr_radius, seed), f"road{side}", side=side)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         wlo: int = 1, whi: int = 1000, seed: int = 0) -> Graph:
    return _take(_load().gg_rmat(scale, edge_factor, a, b, c, wlo, whi, seed), f"rmat{scale}")


def rgg(n: int, mean_degree: float = 6.0, seed: int = 0):
    """Random geometric graph; returns (Graph, x, y) with integer coordinates."""
    lib = _load()
    x = np.empty(n, dtype=np.int32)
    y = np.empty(n, dtype=np.int32)
    g = _take(lib.gg_rgg(n, mean_degree, seed, x.ctypes.data, y.ctypes.data), f"rgg{n}")
    return g, x, y


def grid_heuristic(side: int, target: int) -> np.ndarray:
    """A* heuristic floor(10 * euclid(v, target)) on a side x side grid."""
    h = np.empty(side * side, dtype=np.int32)
    _load().gg_grid_heuristic(side, target, h.ctypes.data)
    return h


def uniform(seed: int, stream: int, count: int, k: int) -> np.ndarray:
    """count counter-based draws uniform in [0, k)."""
    out = np.empty(count, dtype=np.int64)
    _load().gg_uniform(seed, stream, count, k, out.ctypes.data)
    return out


def with_weights(g: Graph, w: np.ndarray, name: str | None = None) -> Graph:
    return Graph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=np.ascontiguousarray(w, dtype=np.int32),
                 name=name or g.name, side=g.side)


def pick_sources(g: Graph, count: int, seed: int = 1, min_degree: int = 1) -> np.ndarray:
    """Seeded sources among vertices with out-degree >= min_degree."""
    cand = np.nonzero(g.degrees() >= min_degree)[0]
    idx = uniform(seed, STREAM_SOURCES, count, len(cand))
    return cand[idx].astype(np.int64)


def from_edges(n: int, src, dst, w, name: str = "edges") -> Graph:
    """Directed CSR from explicit edge lists (small test graphs).  Rows are
    sorted by destination; duplicate (src, dst) pairs keep the smallest
    weight.  Self-loops are kept (they never shorten a path)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.int64)
    order = np.lexsort((w, dst, src))
    src, dst, w = src[order], dst[order], w[order]
    if len(src):
        keep = np.ones(len(src), dtype=bool)
        keep[1:] = (src[1:] != src[:-1]) | (dst[1:] != dst[:-1])
        src, dst, w = src[keep], dst[keep], w[keep]
    counts = np.bincount(src, minlength=n) if len(src) else np.zeros(n, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32), w=w.astype(np.int32), name=name)


def grid_heuristic_device(side: int, targets, device="cuda"):
    """A* estimates for a batch of targets on a side x side grid, computed on
    the device: [len(targets), side*side] int32, h_q[v] = floor(10 *
    euclid(v, t_q)) evaluated in float64.  Distances are integers and every
    edge weight is at least ceil(10 * length), so even a last-bit rounding
    up in the device square root keeps h admissible."""
    import torch
    t = torch.as_tensor(np.asarray(targets, dtype=np.int64), device=device)
    v = torch.arange(side * side, device=device, dtype=torch.int64)
    r, c = (v // side).to(torch.float64), (v % side).to(torch.float64)
    rt, ct = (t // side).to(torch.float64)[:, None], (t % side).to(torch.float64)[:, None]
    h = torch.floor(10.0 * torch.sqrt((r[None, :] - rt) ** 2 + (c[None, :] - ct) ** 2))
    return h.to(torch.int32).contiguous()


def block_diagonal(graphs, name: str = "union") -> "tuple[Graph, np.ndarray]":
    """Disjoint union of CSR graphs; returns (union, vertex offsets)."""
    offs = np.zeros(len(graphs), dtype=np.int64)
    n = 0
    for i, g in enumerate(graphs):
        offs[i] = n
        n += g.n
    row_ptr = [np.zeros(1, dtype=np.int64)]
    cols, ws = [], []
    eoff = 0
    for g, o in zip(graphs, offs):
        row_ptr.append(g.row_ptr[1:] + eoff)
        cols.append(g.col.astype(np.int64) + o)
        ws.append(g.w)
        eoff += g.m
    return Graph(n=n, row_ptr=np.concatenate(row_ptr), col=np.concatenate(cols).astype(np.int32),
                 w=np.concatenate(ws).astype(np.int32), name=name), offs


def rgg_family(count: int, nmin: int = 1000, nmax: int = 64000, mean_degree: float = 6.0, seed: int = 0):
    """`count` random geometric graphs with sizes log-uniform in [nmin, nmax]
    (graph i uses seed `seed*100003 + i`); returns the list of graphs."""
    u = uniform(seed, STREAM_PAIRS, count, 1 << 30) / float(1 << 30)
    sizes = np.exp(np.log(nmin) + u * (np.log(nmax) - np.log(nmin))).astype(np.int64)
    return [rgg(int(sz), mean_degree, seed=seed * 100003 + i)[0] for i, sz in enumerate(sizes)]


def _sm64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on uint64 arrays (wrapping arithmetic)."""
    x = x + np.uint64(0x9E3779B97F4A7C15)
    x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


STREAM_FLOAT_W = 104


def float_weights(g: Graph, lo: float = 1.0, hi: float = 1000.0, seed: int = 3) -> np.ndarray:
    """float32 weights, continuous uniform in [lo, hi), one draw per
    undirected pair {u, v} (both directions equal): u01 of
    sm64(sm64(sm64(seed) + stream) + min*n + max), scaled in float64 and
    rounded to float32."""
    with np.errstate(over="ignore"):
        src = np.repeat(np.arange(g.n, dtype=np.uint64), g.degrees())
        dst = g.col.astype(np.uint64)
        a = np.minimum(src, dst)
        b = np.maximum(src, dst)
        key = _sm64(_sm64(np.array([seed], dtype=np.uint64))[0:1] + np.uint64(STREAM_FLOAT_W))[0]
        x = _sm64(key + a * np.uint64(g.n) + b)
    u = (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (lo + (hi - lo) * u).astype(np.float32)
