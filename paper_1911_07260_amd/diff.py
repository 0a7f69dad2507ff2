"""Differentiable shortest-path distances (float32 weights).

`shortest_path_distances(w, graph, src)` returns float32 distances D(v) from
`src` for edge weights `w` (a float32 tensor of the graph's m edges) and is
differentiable in `w`: with unique shortest paths, D(t) is the sum of the
weights on the tree path to t, so dD(t)/dw_e = 1 on that path and 0 off it,
and the gradient of any loss of the distances is, for the tree edge e into
v, the sum of dL/dD over v's subtree.  Forward = og_sssp_f32 (the bucket
engine in float32 arithmetic, recording the tree); backward =
og_sssp_backward_f32 (subtree sums accumulated leaf to root on the device).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import OG_OK, OgError, OgGraphF32, OgStats

__all__ = ["sssp_f32", "sssp_backward_f32", "ShortestPathDistances", "shortest_path_distances"]


def _graph_f32(graph, w: torch.Tensor) -> OgGraphF32:
    if not (w.dtype == torch.float32 and w.is_contiguous() and w.numel() == graph.m):
        raise ValueError(f"w must be a contiguous float32 tensor of the graph's {graph.m} edges")
    return OgGraphF32(graph.n, graph.m, graph.row_ptr.data_ptr(), graph.col.data_ptr() if graph.m else None,
                      w.data_ptr() if graph.m else None)


def sssp_f32(graph, w: torch.Tensor, src: int, schedule=None, pred: bool = True, ws=None, stream=None,
             check: bool = True):
    """og_sssp_f32: (dist float32 [n], pred int32 [n], pred_edge int32 [n],
    stats).  pred/pred_edge are None when pred=False."""
    from . import Schedule, Workspace
    lib = _lib.load()
    schedule = schedule or Schedule()
    g = _graph_f32(graph, w)
    s = schedule.to_c()
    nbytes = int(lib.og_workspace_bytes_f32(ctypes.byref(g), ctypes.byref(s)))
    if nbytes == 0:
        raise OgError(_lib.OG_ERR_INVALID_ARG, "og_workspace_bytes_f32", lib)
    ws = ws or Workspace(graph.device)
    buf = ws.get(nbytes)
    dev = graph.device
    dist = torch.empty(graph.n, dtype=torch.float32, device=dev)
    p = torch.empty(graph.n, dtype=torch.int32, device=dev) if pred else None
    pe = torch.empty(graph.n, dtype=torch.int32, device=dev) if pred else None
    st = OgStats()
    stream = stream or torch.cuda.current_stream(dev)
    rc = lib.og_sssp_f32(ctypes.byref(g), int(src), ctypes.byref(s), ctypes.c_void_p(dist.data_ptr()),
                         ctypes.c_void_p(p.data_ptr()) if pred else None,
                         ctypes.c_void_p(pe.data_ptr()) if pred else None,
                         ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(buf.numel()), ctypes.byref(st),
                         ctypes.c_void_p(stream.cuda_stream))
    stats = st.as_dict()
    stats["status"] = int(rc)
    if check and rc != OG_OK:
        raise OgError(rc, "og_sssp_f32", lib)
    return dist, p, pe, stats


def sssp_backward_f32(graph, w: torch.Tensor, pred: torch.Tensor, pred_edge: torch.Tensor,
                      grad_dist: torch.Tensor, ws=None, stream=None) -> torch.Tensor:
    """og_sssp_backward_f32: dL/dw (float32 [m]) from dL/dD (float32 [n])."""
    from . import Workspace
    lib = _lib.load()
    g = _graph_f32(graph, w)
    grad_dist = grad_dist.to(dtype=torch.float32).contiguous()
    grad_w = torch.empty(graph.m, dtype=torch.float32, device=graph.device)
    ws = ws or Workspace(graph.device)
    buf = ws.get(int(lib.og_backward_workspace_bytes(graph.n)))
    stream = stream or torch.cuda.current_stream(graph.device)
    rc = lib.og_sssp_backward_f32(ctypes.byref(g), ctypes.c_void_p(pred.data_ptr()),
                                  ctypes.c_void_p(pred_edge.data_ptr()), ctypes.c_void_p(grad_dist.data_ptr()),
                                  ctypes.c_void_p(grad_w.data_ptr()), ctypes.c_void_p(buf.data_ptr()),
                                  ctypes.c_size_t(buf.numel()), ctypes.c_void_p(stream.cuda_stream))
    if rc != OG_OK:
        raise OgError(rc, "og_sssp_backward_f32", lib)
    return grad_w


class ShortestPathDistances(torch.autograd.Function):
    """dist = D(w) with dL/dw from reverse subtree sums over the tree."""

    @staticmethod
    def forward(ctx, w, graph, src, schedule):
        dist, pred, pe, _ = sssp_f32(graph, w.detach().contiguous(), src, schedule)
        ctx.save_for_backward(w, pred, pe)
        ctx.graph = graph
        return dist

    @staticmethod
    def backward(ctx, grad_dist):
        w, pred, pe = ctx.saved_tensors
        grad_w = sssp_backward_f32(ctx.graph, w.detach().contiguous(), pred, pe, grad_dist)
        return grad_w, None, None, None


def shortest_path_distances(w: torch.Tensor, graph, src: int, schedule=None) -> torch.Tensor:
    """Differentiable single-source distances (see the module docstring)."""
    return ShortestPathDistances.apply(w, graph, int(src), schedule)
