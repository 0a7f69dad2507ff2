"""og_sssp_noalloc (the entry point that allocates nothing) against og_sssp
(the same engine with a caller-provided workspace), through the C ABI:
identical distances and predecessors on two calls in a row, the second on
a smaller graph (the fixed array keeps the first call's contents), both
also equal to the CPU oracle; a graph too large for the fixed array is
refused with nothing launched."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og
from paper_1911_07260_amd import _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def noalloc(lib, dg, src, sched):
    d = torch.full((dg.n,), -7, dtype=torch.int32, device=DEV)
    p = torch.full((dg.n,), -7, dtype=torch.int32, device=DEV)
    g = dg.to_c()
    s = sched.to_c()
    st = _lib.OgStats()
    rc = lib.og_sssp_noalloc(ctypes.byref(g), int(src), ctypes.byref(s), ctypes.c_void_p(d.data_ptr()),
                             ctypes.c_void_p(p.data_ptr()), ctypes.byref(st),
                             ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    torch.cuda.synchronize()
    return rc, st, d.cpu().numpy(), p.cpu().numpy()


@pytest.mark.parametrize("flags", [0, og.OG_FLAG_DEGREE_BINS])
def test_noalloc_matches_workspace_call(orc, flags):
    lib = _lib.load()
    sched = og.Schedule(delta=256, flags=flags)
    for side in (1024, 96):  # the second call is smaller
        g = gg.road(side, seed=0)
        dg = og.DeviceGraph.from_host(g, DEV)
        src = int(gg.pick_sources(g, 1, seed=1)[0])
        need = og.workspace_bytes(dg, sched)
        assert need <= og.OG_SCRATCH_BYTES
        say(f"noalloc road{side} src={src} flags={flags} (workspace {need} bytes)")
        rc, st, d, p = noalloc(lib, dg, src, sched)
        assert rc == og.OG_OK and st.status == og.OG_OK
        ref_d, ref_p, ref_st = og.sssp(dg, src, sched)
        torch.cuda.synchronize()
        assert np.array_equal(d, ref_d.cpu().numpy()) and np.array_equal(p, ref_p.cpu().numpy())
        want_d, want_p = orc.sssp(g, src)
        assert np.array_equal(d, want_d) and np.array_equal(p, want_p)
        assert st.reached_vertices == ref_st["reached_vertices"] and st.reached_edges == ref_st["reached_edges"]


def test_noalloc_refuses_oversized_and_object_creating_calls():
    lib = _lib.load()
    g = gg.road(2048, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    sched = og.Schedule(delta=256)
    assert og.workspace_bytes(dg, sched) > og.OG_SCRATCH_BYTES
    rc, st, d, _ = noalloc(lib, dg, 0, sched)
    assert rc == og.OG_ERR_WORKSPACE and st.status == rc
    assert np.all(d == -7)  # nothing was launched
    for bad in (og.Schedule(delta=256, flags=og.OG_FLAG_TIMING),
                og.Schedule(delta=256, engine=og.OG_ENGINE_GRAPH_ROUNDS)):
        small = og.DeviceGraph.from_host(gg.road(64, seed=0), DEV)
        rc, st, d, _ = noalloc(lib, small, 0, bad)
        assert rc == og.OG_ERR_INVALID_ARG and np.all(d == -7)
