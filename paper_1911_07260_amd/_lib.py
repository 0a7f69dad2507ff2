"""ctypes declarations for libog.so (the C ABI in include/og.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the ABI.  Importing this module fails loudly when the
library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libog.so")

OG_OK = 0
OG_ERR_INVALID_ARG = -1
OG_ERR_NEGATIVE_WEIGHT = -2
OG_ERR_OVERFLOW = -3
OG_ERR_WORKSPACE = -4
OG_ERR_HIP = -5
OG_ERR_ROUND_LIMIT = -6
OG_ERR_INTERNAL = -7

OG_FLAG_VALIDATE = 1
OG_FLAG_ASYNC = 2
OG_FLAG_TIMING = 4
OG_FLAG_LIGHT_HEAVY = 8
OG_FLAG_DENSE_PULL = 16
OG_FLAG_HYBRID_DIRECTION = 32
OG_FLAG_DEGREE_BINS = 64
OG_FLAG_KEEP_SPLIT = 128
OG_FLAG_VERTEX_BLOCKS = 256
OG_FLAG_KEEP_BLOCKS = 512

OG_SCRATCH_BYTES = 32 << 20  # og_sssp_noalloc's fixed workspace per device

OG_EAGER_NO_FUSION = 0
OG_EAGER_WITH_FUSION = 1
OG_LAZY_UPDATE = 2

OG_ENGINE_PERSISTENT = 0
OG_ENGINE_GRAPH_ROUNDS = 2
OG_ENGINE_HOST_ROUNDS = 1


class OgGraph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
    ]


class OgGraphF32(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
    ]


class OgSchedule(ctypes.Structure):
    _fields_ = [
        ("delta", ctypes.c_int32),
        ("update", ctypes.c_int32),
        ("fusion_threshold", ctypes.c_int32),
        ("window_buckets", ctypes.c_int32),
        ("engine", ctypes.c_int32),
        ("max_rounds", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("queue_capacity", ctypes.c_int64),
        ("bin_thread", ctypes.c_int32),
        ("bin_wave", ctypes.c_int32),
        ("block_size", ctypes.c_int32),
        ("queue_pool", ctypes.c_int64),
        ("teams", ctypes.c_int32),
    ]


class OgStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("rounds", ctypes.c_int64),
        ("buckets", ctypes.c_int64),
        ("relaxations", ctypes.c_int64),
        ("improvements", ctypes.c_int64),
        ("pushes_local", ctypes.c_int64),
        ("pushes_global", ctypes.c_int64),
        ("far_pushes", ctypes.c_int64),
        ("reached_vertices", ctypes.c_int64),
        ("reached_edges", ctypes.c_int64),
        ("queue_needed", ctypes.c_int64),
        ("init_ms", ctypes.c_double),
        ("engine_ms", ctypes.c_double),
        ("pred_ms", ctypes.c_double),
        ("batches", ctypes.c_int64),
        ("chain", ctypes.c_int64),
        ("barriers", ctypes.c_int64),
        ("blocks", ctypes.c_int64),
        ("prep_ms", ctypes.c_double),
        ("pool_needed", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: (float(getattr(self, name)) if name.endswith("_ms") else int(getattr(self, name)))
                for name, _ in self._fields_}


class OgError(RuntimeError):
    def __init__(self, status: int, where: str, lib=None):
        msg = lib.og_status_string(status).decode() if lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


_lib = None


def load():
    """The loaded libog.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first (python -c "
            "'import __graft_entry__ as g; g.build()'); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.og_version.restype = i32
    lib.og_version.argtypes = []
    lib.og_status_string.restype = ctypes.c_char_p
    lib.og_status_string.argtypes = [i32]
    lib.og_default_schedule.restype = i32
    lib.og_default_schedule.argtypes = [P(OgSchedule)]
    lib.og_workspace_bytes.restype = ctypes.c_size_t
    lib.og_workspace_bytes.argtypes = [P(OgGraph), P(OgSchedule)]
    common = [P(OgSchedule), vp, vp, vp, ctypes.c_size_t, P(OgStats), vp]
    lib.og_sssp.restype = i32
    lib.og_sssp.argtypes = [P(OgGraph), i32] + common
    lib.og_wbfs.restype = i32
    lib.og_wbfs.argtypes = [P(OgGraph), i32] + common
    lib.og_ppsp.restype = i32
    lib.og_ppsp.argtypes = [P(OgGraph), i32, i32] + common
    lib.og_astar.restype = i32
    lib.og_astar.argtypes = [P(OgGraph), i32, i32, vp] + common
    lib.og_workspace_bytes_batch.restype = ctypes.c_size_t
    lib.og_workspace_bytes_batch.argtypes = [P(OgGraph), P(OgSchedule), i32]
    lib.og_workspace_bytes_multi.restype = ctypes.c_size_t
    lib.og_workspace_bytes_multi.argtypes = [P(OgGraph), P(OgSchedule), i32]
    lib.og_sssp_batch.restype = i32
    lib.og_sssp_batch.argtypes = [P(OgGraph), vp, i32] + common
    lib.og_ppsp_batch.restype = i32
    lib.og_ppsp_batch.argtypes = [P(OgGraph), vp, vp, i32] + common
    lib.og_astar_batch.restype = i32
    lib.og_astar_batch.argtypes = [P(OgGraph), vp, vp, i32, vp] + common
    lib.og_sssp_multi.restype = i32
    lib.og_sssp_multi.argtypes = [P(OgGraph), vp, i32] + common
    lib.og_workspace_bytes_f32.restype = ctypes.c_size_t
    lib.og_workspace_bytes_f32.argtypes = [P(OgGraphF32), P(OgSchedule)]
    lib.og_sssp_f32.restype = i32
    lib.og_sssp_f32.argtypes = [P(OgGraphF32), i32, P(OgSchedule), vp, vp, vp, vp, ctypes.c_size_t, P(OgStats), vp]
    lib.og_backward_workspace_bytes.restype = ctypes.c_size_t
    lib.og_backward_workspace_bytes.argtypes = [i32]
    lib.og_sssp_backward_f32.restype = i32
    lib.og_sssp_backward_f32.argtypes = [P(OgGraphF32), vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.og_workspace_bytes_kcore.restype = ctypes.c_size_t
    lib.og_workspace_bytes_kcore.argtypes = [P(OgGraph), P(OgSchedule)]
    lib.og_kcore.restype = i32
    lib.og_kcore.argtypes = [P(OgGraph), P(OgSchedule), vp, vp, ctypes.c_size_t, P(OgStats), vp]
    lib.og_sssp_noalloc.restype = i32
    lib.og_sssp_noalloc.argtypes = [P(OgGraph), i32, P(OgSchedule), vp, vp, P(OgStats), vp]
    lib.og_release.restype = i32
    lib.og_release.argtypes = []
    lib.og_read_stats.restype = i32
    lib.og_read_stats.argtypes = [vp, P(OgStats), vp]
    _lib = lib
    return lib
