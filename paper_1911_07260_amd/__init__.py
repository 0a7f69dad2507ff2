"""Ordered (bucketed) shortest-path processing on MI355X.

Python face of libog.so (include/og.h).  PyTorch supplies device memory and
streams only; every step of the computation runs in the library's HIP
kernels.  Functions mirror the C ABI:

    sssp(graph, src, schedule)        og_sssp
    wbfs(graph, src, schedule)        og_wbfs   (Delta forced to 1)
    ppsp(graph, src, dst, schedule)   og_ppsp
    astar(graph, src, dst, h, sched)  og_astar
    kcore(graph, schedule)            og_kcore  (coreness of every vertex)
    sssp_batch / ppsp_batch / astar_batch
                                      og_*_batch (many queries, one launch)
    sssp_multi(graph, srcs, schedule) og_sssp_multi (several sources at 0)

The Schedule selects the update mode (eager with or without bucket fusion,
lazy), the engine (persistent kernel, one launch per round, or rounds
replayed from a captured hipGraph) and flags (structure validation, light /
heavy edge split, dense-pull or hybrid traversal direction with lazy
updates, degree-binned load balancing, LDS-resident vertex blocks).  ``diff`` holds the FP32 forward and backward passes
(og_sssp_f32, og_sssp_backward_f32) and an autograd Function over them;
``autotune`` searches the schedule on the device (Delta, update strategy
and direction, fusion threshold, window, workgroups, degree bins).

Each shortest-path call returns ``(dist, pred, stats)`` with int32 device
tensors (pred is None when not requested) and a dict of counters.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field, fields

import torch

from . import _lib
from ._lib import (OG_EAGER_NO_FUSION, OG_EAGER_WITH_FUSION, OG_ENGINE_GRAPH_ROUNDS, OG_ENGINE_HOST_ROUNDS,
                   OG_ENGINE_PERSISTENT, OG_ERR_HIP, OG_ERR_INTERNAL, OG_ERR_INVALID_ARG, OG_ERR_NEGATIVE_WEIGHT,
                   OG_ERR_OVERFLOW, OG_ERR_ROUND_LIMIT, OG_ERR_WORKSPACE, OG_FLAG_ASYNC, OG_FLAG_DEGREE_BINS,
                   OG_FLAG_DENSE_PULL, OG_FLAG_HYBRID_DIRECTION, OG_FLAG_KEEP_BLOCKS, OG_FLAG_KEEP_SPLIT,
                   OG_FLAG_LIGHT_HEAVY, OG_FLAG_TIMING, OG_FLAG_VALIDATE, OG_FLAG_VERTEX_BLOCKS, OG_LAZY_UPDATE, OG_OK,
                   OG_SCRATCH_BYTES,
                   OgError, OgGraph, OgSchedule, OgStats)

INF = 2**31 - 1


def _require(ok: bool, what: str) -> None:
    """Argument check that survives python -O (a failed check never reaches
    the library with a buffer of the wrong type or size)."""
    if not ok:
        raise ValueError(what)

__all__ = [
    "DeviceGraph", "Schedule", "Workspace", "sssp", "sssp_noalloc", "wbfs", "ppsp", "astar", "sssp_batch", "ppsp_batch",
    "astar_batch", "sssp_multi", "kcore", "workspace_bytes", "status_string", "version", "release", "INF",
    "OgError",
]


@dataclass
class Schedule:
    """og_schedule (section 4.2 scheduling options).  Zero = library default."""
    delta: int = 1
    update: int = OG_EAGER_WITH_FUSION
    fusion_threshold: int = 0
    window_buckets: int = 0
    engine: int = OG_ENGINE_PERSISTENT
    max_rounds: int = 0
    workgroups: int = 0
    flags: int = 0
    queue_capacity: int = 0
    bin_thread: int = 0
    bin_wave: int = 0
    block_size: int = 0
    queue_pool: int = 0
    teams: int = 0

    @property
    def fused(self) -> bool:
        return self.update == OG_EAGER_WITH_FUSION

    def to_c(self) -> OgSchedule:
        return OgSchedule(**{f.name: int(getattr(self, f.name)) for f in fields(self)})


class DeviceGraph:
    """Directed CSR graph resident on a device (int64 row_ptr, int32 col, w)."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, w: torch.Tensor | None):
        _require(row_ptr.dtype == torch.int64 and col.dtype == torch.int32,
                 "DeviceGraph: row_ptr must be int64 and col int32")
        _require(row_ptr.is_contiguous() and col.is_contiguous(), "DeviceGraph: row_ptr and col must be contiguous")
        _require(w is None or (w.dtype == torch.int32 and w.is_contiguous()),
                 "DeviceGraph: w must be a contiguous int32 tensor")
        _require(row_ptr.numel() >= 2, "DeviceGraph: row_ptr needs n + 1 >= 2 entries")
        _require(w is None or w.numel() == col.numel(), "DeviceGraph: w and col must have the same length")
        self.row_ptr, self.col, self.w = row_ptr, col, w
        self.n = row_ptr.numel() - 1
        self.m = col.numel()

    @classmethod
    def from_host(cls, g, device="cuda", weights: bool = True):
        """From any object with numpy row_ptr / col / w (e.g. graphgen.Graph);
        weights=False leaves w out (og_kcore does not read it)."""
        rp = torch.from_numpy(g.row_ptr).to(device=device, dtype=torch.int64).contiguous()
        col = torch.from_numpy(g.col).to(device=device, dtype=torch.int32).contiguous()
        w = torch.from_numpy(g.w).to(device=device, dtype=torch.int32).contiguous() if weights else None
        return cls(rp, col, w)

    @property
    def device(self):
        return self.row_ptr.device

    def to_c(self) -> OgGraph:
        return OgGraph(self.n, self.m, self.row_ptr.data_ptr(),
                       self.col.data_ptr() if self.m else None,
                       self.w.data_ptr() if (self.m and self.w is not None) else None)


def version() -> int:
    return int(_lib.load().og_version())


def release() -> None:
    """og_release: waits for the device and frees what the library keeps per
    host thread (timing events, the replayed round graph)."""
    lib = _lib.load()
    status = lib.og_release()
    if status != OG_OK:
        raise OgError(status, "og_release", lib)


def status_string(status: int) -> str:
    return _lib.load().og_status_string(int(status)).decode()


def workspace_bytes(graph: DeviceGraph, schedule: Schedule, batch: int = 0, multi: int = 0) -> int:
    """og_workspace_bytes (single query), ..._batch (batch = nq queries) or
    ..._multi (multi = number of sources)."""
    lib = _lib.load()
    g = graph.to_c()
    s = schedule.to_c()
    if batch:
        return int(lib.og_workspace_bytes_batch(ctypes.byref(g), ctypes.byref(s), int(batch)))
    if multi:
        return int(lib.og_workspace_bytes_multi(ctypes.byref(g), ctypes.byref(s), int(multi)))
    return int(lib.og_workspace_bytes(ctypes.byref(g), ctypes.byref(s)))


class Workspace:
    """A device byte buffer reused across calls (grown on demand)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf: torch.Tensor | None = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws: dict = {}


def _workspace(graph: DeviceGraph, schedule: Schedule, ws: Workspace | None, batch: int = 0, multi: int = 0):
    nbytes = workspace_bytes(graph, schedule, batch=batch, multi=multi)
    if nbytes == 0:
        raise OgError(OG_ERR_INVALID_ARG, "og_workspace_bytes", _lib.load())
    if ws is None:
        key = str(graph.device)
        ws = _default_ws.setdefault(key, Workspace(graph.device))
    return ws.get(nbytes), nbytes


def _call(fn_name, graph, args_mid, schedule, want_pred, ws, stream, out_dist=None, out_pred=None,
          check=True, nq=1, batch=0, multi=0):
    lib = _lib.load()
    schedule = schedule or Schedule()
    n = graph.n * nq
    dev = graph.device
    shape = (nq, graph.n) if batch else (graph.n,)
    dist = out_dist if out_dist is not None else torch.empty(shape, dtype=torch.int32, device=dev)
    pred = out_pred if out_pred is not None else (
        torch.empty(shape, dtype=torch.int32, device=dev) if want_pred else None)
    _require(dist.numel() == n and dist.dtype == torch.int32 and dist.is_contiguous(),
             f"output dist must be a contiguous int32 tensor of {n} entries")
    _require(pred is None or (pred.numel() == n and pred.dtype == torch.int32 and pred.is_contiguous()),
             f"output pred must be a contiguous int32 tensor of {n} entries")
    buf, nbytes = _workspace(graph, schedule, ws, batch=batch, multi=multi)
    g = graph.to_c()
    s = schedule.to_c()
    st = OgStats()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    handle = ctypes.c_void_p(stream.cuda_stream)
    fn = getattr(lib, fn_name)
    status = fn(ctypes.byref(g), *args_mid, ctypes.byref(s), ctypes.c_void_p(dist.data_ptr()),
                ctypes.c_void_p(pred.data_ptr()) if pred is not None else None,
                ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(buf.numel()), ctypes.byref(st), handle)
    stats = st.as_dict()
    stats["status"] = int(status)
    if check and status != OG_OK:
        raise OgError(status, fn_name, lib)
    return dist, pred, stats


def sssp(graph: DeviceGraph, src: int, schedule: Schedule | None = None, pred: bool = True,
         ws: Workspace | None = None, stream=None, **kw):
    """Single-source shortest paths (og_sssp)."""
    return _call("og_sssp", graph, [int(src)], schedule, pred, ws, stream, **kw)


def sssp_noalloc(graph: DeviceGraph, src: int, schedule: Schedule | None = None, pred: bool = True,
                 stream=None, out_dist: torch.Tensor | None = None, out_pred: torch.Tensor | None = None,
                 check: bool = True):
    """og_sssp_noalloc: og_sssp on the library's fixed per-device workspace
    (OG_SCRATCH_BYTES); no device allocation by the library.  Calls that
    overlap on one device must not be made."""
    lib = _lib.load()
    schedule = schedule or Schedule()
    dev = graph.device
    dist = out_dist if out_dist is not None else torch.empty(graph.n, dtype=torch.int32, device=dev)
    pr = out_pred if out_pred is not None else (torch.empty(graph.n, dtype=torch.int32, device=dev) if pred else None)
    _require(dist.numel() == graph.n and dist.dtype == torch.int32 and dist.is_contiguous(),
             f"output dist must be a contiguous int32 tensor of {graph.n} entries")
    _require(pr is None or (pr.numel() == graph.n and pr.dtype == torch.int32 and pr.is_contiguous()),
             f"output pred must be a contiguous int32 tensor of {graph.n} entries")
    g = graph.to_c()
    s = schedule.to_c()
    st = OgStats()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    status = lib.og_sssp_noalloc(ctypes.byref(g), int(src), ctypes.byref(s), ctypes.c_void_p(dist.data_ptr()),
                                 ctypes.c_void_p(pr.data_ptr()) if pr is not None else None, ctypes.byref(st),
                                 ctypes.c_void_p(stream.cuda_stream))
    stats = st.as_dict()
    stats["status"] = int(status)
    if check and status != OG_OK:
        raise OgError(status, "og_sssp_noalloc", lib)
    return dist, pr, stats


def wbfs(graph: DeviceGraph, src: int, schedule: Schedule | None = None, pred: bool = True,
         ws: Workspace | None = None, stream=None, **kw):
    """Weighted BFS (og_wbfs): Delta = 1."""
    return _call("og_wbfs", graph, [int(src)], schedule, pred, ws, stream, **kw)


def ppsp(graph: DeviceGraph, src: int, dst: int, schedule: Schedule | None = None, pred: bool = True,
         ws: Workspace | None = None, stream=None, **kw):
    """Point-to-point shortest path (og_ppsp): only dist[dst] and dst's
    predecessor chain are defined."""
    return _call("og_ppsp", graph, [int(src), int(dst)], schedule, pred, ws, stream, **kw)


def astar(graph: DeviceGraph, src: int, dst: int, h: torch.Tensor, schedule: Schedule | None = None,
          pred: bool = True, ws: Workspace | None = None, stream=None, **kw):
    """A* (og_astar) with per-vertex estimate h (int32 device tensor)."""
    _require(h.dtype == torch.int32 and h.is_contiguous() and h.numel() == graph.n,
             f"h must be a contiguous int32 tensor of {graph.n} entries")
    return _call("og_astar", graph, [int(src), int(dst), ctypes.c_void_p(h.data_ptr())], schedule, pred,
                 ws, stream, **kw)


def _host_ids(a) -> "np.ndarray":
    import numpy as np
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


def sssp_batch(graph: DeviceGraph, srcs, schedule: Schedule | None = None, pred: bool = True,
               ws: Workspace | None = None, stream=None, **kw):
    """nq single-source queries in one launch (og_sssp_batch); dist and pred
    are [nq, n]."""
    s_ = _host_ids(srcs)
    return _call("og_sssp_batch", graph, [ctypes.c_void_p(s_.ctypes.data), len(s_)], schedule, pred, ws, stream,
                 nq=len(s_), batch=len(s_), **kw)


def ppsp_batch(graph: DeviceGraph, srcs, dsts, schedule: Schedule | None = None, pred: bool = True,
               ws: Workspace | None = None, stream=None, **kw):
    """nq point-to-point queries in one launch (og_ppsp_batch)."""
    s_, t_ = _host_ids(srcs), _host_ids(dsts)
    _require(len(s_) == len(t_), "ppsp_batch: srcs and dsts must have the same length")
    return _call("og_ppsp_batch", graph, [ctypes.c_void_p(s_.ctypes.data), ctypes.c_void_p(t_.ctypes.data), len(s_)],
                 schedule, pred, ws, stream, nq=len(s_), batch=len(s_), **kw)


def astar_batch(graph: DeviceGraph, srcs, dsts, h: torch.Tensor, schedule: Schedule | None = None,
                pred: bool = True, ws: Workspace | None = None, stream=None, **kw):
    """nq A* queries in one launch (og_astar_batch); h is [nq, n] int32."""
    s_, t_ = _host_ids(srcs), _host_ids(dsts)
    _require(len(s_) == len(t_), "astar_batch: srcs and dsts must have the same length")
    _require(h.dtype == torch.int32 and h.is_contiguous() and h.numel() == graph.n * len(s_),
             f"h must be a contiguous int32 tensor of {graph.n * len(s_)} entries")
    return _call("og_astar_batch", graph, [ctypes.c_void_p(s_.ctypes.data), ctypes.c_void_p(t_.ctypes.data), len(s_),
                                           ctypes.c_void_p(h.data_ptr())],
                 schedule, pred, ws, stream, nq=len(s_), batch=len(s_), **kw)


def sssp_multi(graph: DeviceGraph, srcs, schedule: Schedule | None = None, pred: bool = True,
               ws: Workspace | None = None, stream=None, **kw):
    """Multi-source shortest paths (og_sssp_multi): dist[v] = min over srcs."""
    s_ = _host_ids(srcs)
    return _call("og_sssp_multi", graph, [ctypes.c_void_p(s_.ctypes.data), len(s_)], schedule, pred, ws, stream,
                 multi=len(s_), **kw)


def kcore(graph: DeviceGraph, schedule: Schedule | None = None, ws: Workspace | None = None, stream=None,
          out: torch.Tensor | None = None, check: bool = True):
    """k-core decomposition (og_kcore): (coreness int32 [n], stats).  The
    graph must store both directions of every edge; weights are not read.
    schedule.update: OG_LAZY_UPDATE (histogram reduction) or an eager mode;
    delta is ignored."""
    lib = _lib.load()
    schedule = schedule or Schedule(update=OG_LAZY_UPDATE)
    g = graph.to_c()
    s = schedule.to_c()
    nbytes = int(lib.og_workspace_bytes_kcore(ctypes.byref(g), ctypes.byref(s)))
    if nbytes == 0:
        raise OgError(OG_ERR_INVALID_ARG, "og_workspace_bytes_kcore", lib)
    if ws is None:
        ws = _default_ws.setdefault(str(graph.device), Workspace(graph.device))
    buf = ws.get(nbytes)
    core = out if out is not None else torch.empty(graph.n, dtype=torch.int32, device=graph.device)
    _require(core.numel() == graph.n and core.dtype == torch.int32 and core.is_contiguous(),
             f"output core must be a contiguous int32 tensor of {graph.n} entries")
    st = OgStats()
    if stream is None:
        stream = torch.cuda.current_stream(graph.device)
    status = lib.og_kcore(ctypes.byref(g), ctypes.byref(s), ctypes.c_void_p(core.data_ptr()),
                          ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(buf.numel()), ctypes.byref(st),
                          ctypes.c_void_p(stream.cuda_stream))
    stats = st.as_dict()
    stats["status"] = int(status)
    if check and status != OG_OK:
        raise OgError(status, "og_kcore", lib)
    return core, stats


from .diff import ShortestPathDistances, shortest_path_distances, sssp_backward_f32, sssp_f32  # noqa: E402
