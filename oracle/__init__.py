"""CPU oracle (plain C, built with gcc) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU product path
(``paper_1911_07260_amd``) never imports, loads or calls it, and the two
share no code.

See ``oracle.c`` for what each function computes and which passage of the
paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

INF64 = np.iinfo(np.int64).max
INF32 = np.iinfo(np.int32).max

CHECK_BITS = {
    0: "dist[src] != 0",
    1: "edge not relaxed: dist[v] > dist[u] + w",
    2: "negative distance",
    3: "reachability mismatch",
    4: "pred[src] != src",
    5: "reachable vertex without pred",
    6: "unreachable vertex with pred",
    7: "pred edge not tight",
    8: "pred chain does not reach src",
    9: "pred out of range",
}


def build(out: str = _SO, mutation: int = 0) -> str:
    """Compile the oracle with gcc.  ``mutation`` > 0 plants one of the
    numbered bugs in ``oracle.c`` (used only by the pin tests, which must
    catch each of them)."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", f"-DORACLE_MUTATION={int(mutation)}",
           _SRC, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib):
    vp = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_dijkstra.restype = ctypes.c_int
    lib.oracle_dijkstra.argtypes = [i32, vp, vp, vp, i32, vp]
    lib.oracle_bellman_ford.restype = ctypes.c_int
    lib.oracle_bellman_ford.argtypes = [i32, vp, vp, vp, i32, vp]
    lib.oracle_bfs_reach.restype = ctypes.c_int
    lib.oracle_bfs_reach.argtypes = [i32, vp, vp, i32, vp]
    lib.oracle_canonical_pred.restype = ctypes.c_int
    lib.oracle_canonical_pred.argtypes = [i32, vp, vp, vp, i32, vp, vp]
    lib.oracle_to_i32.restype = i64
    lib.oracle_to_i32.argtypes = [i32, vp, vp]
    lib.oracle_ppsp.restype = i64
    lib.oracle_ppsp.argtypes = [i32, vp, vp, vp, i32, i32]
    lib.oracle_astar.restype = i64
    lib.oracle_astar.argtypes = [i32, vp, vp, vp, i32, i32, vp, vp]
    lib.oracle_check.restype = ctypes.c_uint32
    lib.oracle_check.argtypes = [i32, vp, vp, vp, i32, vp, vp]
    lib.oracle_dijkstra_f64.restype = ctypes.c_int
    lib.oracle_dijkstra_f64.argtypes = [i32, vp, vp, vp, i32, vp]
    lib.oracle_dijkstra_f32.restype = ctypes.c_int
    lib.oracle_dijkstra_f32.argtypes = [i32, vp, vp, vp, i32, vp]
    lib.oracle_tree_real.restype = ctypes.c_int
    lib.oracle_tree_real.argtypes = [i32, vp, vp, vp, i32, vp, ctypes.c_int, vp, vp]
    lib.oracle_subtree_grad.restype = ctypes.c_int
    lib.oracle_subtree_grad.argtypes = [i32, i64, vp, vp, vp, vp, vp]
    lib.oracle_kcore.restype = ctypes.c_int
    lib.oracle_kcore.argtypes = [i32, vp, vp, vp]
    return lib


class Oracle:
    """ctypes view of one build of liboracle."""

    def __init__(self, path: str):
        self.lib = _bind(ctypes.CDLL(path))

    @staticmethod
    def _csr(g):
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        w = np.ascontiguousarray(g.w, dtype=np.int32)
        return rp, col, w

    def dijkstra64(self, g, src: int) -> np.ndarray:
        """Shortest-path distances, int64, INF64 where unreachable."""
        rp, col, w = self._csr(g)
        d = np.empty(g.n, dtype=np.int64)
        rc = self.lib.oracle_dijkstra(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src),
                                      d.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_dijkstra: bad arguments")
        return d

    def bellman_ford64(self, g, src: int) -> np.ndarray:
        rp, col, w = self._csr(g)
        d = np.empty(g.n, dtype=np.int64)
        rc = self.lib.oracle_bellman_ford(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data,
                                          int(src), d.ctypes.data)
        if rc < 0:
            raise ValueError("oracle_bellman_ford: bad arguments")
        return d

    def reach(self, g, src: int) -> np.ndarray:
        rp, col, _ = self._csr(g)
        r = np.empty(g.n, dtype=np.uint8)
        self.lib.oracle_bfs_reach(g.n, rp.ctypes.data, col.ctypes.data, int(src), r.ctypes.data)
        return r.astype(bool)

    def to_i32(self, d64: np.ndarray):
        d64 = np.ascontiguousarray(d64, dtype=np.int64)
        d32 = np.empty(len(d64), dtype=np.int32)
        over = self.lib.oracle_to_i32(len(d64), d64.ctypes.data, d32.ctypes.data)
        return d32, int(over)

    def canonical_pred(self, g, src: int, d64: np.ndarray) -> np.ndarray:
        rp, col, w = self._csr(g)
        d64 = np.ascontiguousarray(d64, dtype=np.int64)
        p = np.empty(g.n, dtype=np.int32)
        self.lib.oracle_canonical_pred(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src),
                                       d64.ctypes.data, p.ctypes.data)
        return p

    def sssp(self, g, src: int):
        """(dist int32 with INF32, canonical pred int32)."""
        d64 = self.dijkstra64(g, src)
        d32, over = self.to_i32(d64)
        if over:
            raise OverflowError(f"{over} distances do not fit in int32")
        return d32, self.canonical_pred(g, src, d64)

    def ppsp(self, g, src: int, dst: int) -> int:
        """s-d shortest distance; -1 if unreachable."""
        rp, col, w = self._csr(g)
        r = self.lib.oracle_ppsp(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src), int(dst))
        if r < -1:
            raise ValueError("oracle_ppsp: bad arguments")
        return int(r)

    def astar(self, g, src: int, dst: int, h: np.ndarray):
        """(s-d distance or -1, expanded vertex count) by textbook A*."""
        rp, col, w = self._csr(g)
        h = np.ascontiguousarray(h, dtype=np.int32)
        ex = ctypes.c_int64(0)
        r = self.lib.oracle_astar(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src),
                                  int(dst), h.ctypes.data, ctypes.byref(ex))
        if r < -1:
            raise ValueError("oracle_astar: bad arguments")
        return int(r), int(ex.value)

    # ---- real-valued weights (float32 w) --------------------------------
    def _csr_f(self, g, wf):
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        w = np.ascontiguousarray(wf, dtype=np.float32)
        return rp, col, w

    def dijkstra_real(self, g, wf, src: int, f32: bool) -> np.ndarray:
        """Shortest distances (float64 array, inf unreachable): exact
        arithmetic (f32=False) or every addition rounded to float32."""
        rp, col, w = self._csr_f(g, wf)
        d = np.empty(g.n, dtype=np.float64)
        fn = self.lib.oracle_dijkstra_f32 if f32 else self.lib.oracle_dijkstra_f64
        if fn(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src), d.ctypes.data) != 0:
            raise ValueError("oracle_dijkstra_real: bad arguments")
        return d

    def tree_real(self, g, wf, src: int, dist: np.ndarray, f32: bool):
        """(pred, pred_edge) of the canonical tree (float32 or exact tightness)."""
        rp, col, w = self._csr_f(g, wf)
        dist = np.ascontiguousarray(dist, dtype=np.float64)
        p = np.empty(g.n, dtype=np.int32)
        pe = np.empty(g.n, dtype=np.int32)
        self.lib.oracle_tree_real(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src), dist.ctypes.data,
                                  int(bool(f32)), p.ctypes.data, pe.ctypes.data)
        return p, pe

    def subtree_grad(self, g, dist, pred, pred_edge, upstream) -> np.ndarray:
        """dL/dw for L = sum_v upstream[v] * D(v) on the given tree."""
        dist = np.ascontiguousarray(dist, dtype=np.float64)
        pred = np.ascontiguousarray(pred, dtype=np.int32)
        pe = np.ascontiguousarray(pred_edge, dtype=np.int32)
        up = np.ascontiguousarray(upstream, dtype=np.float64)
        gw = np.empty(g.m, dtype=np.float64)
        if self.lib.oracle_subtree_grad(g.n, g.m, dist.ctypes.data, pred.ctypes.data, pe.ctypes.data,
                                        up.ctypes.data, gw.ctypes.data) != 0:
            raise MemoryError("oracle_subtree_grad")
        return gw

    def kcore(self, g) -> np.ndarray:
        """Coreness of every vertex (int32) by minimum-degree peeling."""
        rp, col, _ = self._csr(g)
        core = np.empty(g.n, dtype=np.int32)
        if self.lib.oracle_kcore(g.n, rp.ctypes.data, col.ctypes.data, core.ctypes.data) != 0:
            raise ValueError("oracle_kcore: bad arguments")
        return core

    def check(self, g, src: int, dist32: np.ndarray, pred: np.ndarray | None = None) -> int:
        """Bitmask of violated shortest-path certificate invariants."""
        rp, col, w = self._csr(g)
        d = np.ascontiguousarray(dist32, dtype=np.int32)
        p = None if pred is None else np.ascontiguousarray(pred, dtype=np.int32)
        return int(self.lib.oracle_check(g.n, rp.ctypes.data, col.ctypes.data, w.ctypes.data, int(src),
                                         d.ctypes.data, None if p is None else p.ctypes.data))


_default = None


def get() -> Oracle:
    """The unmutated oracle, built on first use if missing or stale."""
    global _default
    if _default is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _default = Oracle(_SO)
    return _default


def mutated(mutation: int) -> Oracle:
    """A throw-away build with planted bug ``mutation`` (pin tests only)."""
    d = tempfile.mkdtemp(prefix="oracle_mut")
    return Oracle(build(os.path.join(d, f"liboracle_m{mutation}.so"), mutation))


def describe(bits: int) -> list[str]:
    return [msg for b, msg in CHECK_BITS.items() if bits & (1 << b)]
