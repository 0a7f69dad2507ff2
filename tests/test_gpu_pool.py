"""The shared queue pool: every global queue draws 4,096-entry chunks from
one pool and returns them once consumed, so a pool far smaller than the
entries a call pushes in total suffices.

  - chunks are recycled: with a pool of twice the peak a call reports, the
    call pushes many times the pool's entries and still matches the oracle
    bit for bit;
  - every engine and instantiation (persistent / host rounds / graph
    rounds, fused / unfused, degree bins, light/heavy split, lazy with a
    pull direction, vertex blocks, k-core, batches) runs exact on twice its
    own measured peak;
  - an exhausted pool ends the call with OG_ERR_WORKSPACE and a peak above
    the pool, and the next call on the same workspace is exact again.
Graphs: the 256 x 256 and 1024 x 1024 road-like grids and R-MAT scale 14
(edge factor 16).
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CHUNK = 4096


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def road256():
    g = gg.road(256, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.fixture(scope="module")
def rmat14():
    g = gg.rmat(14, 16, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


def exact(orc, g, src, d, p, tag):
    ref_d, ref_p = orc.sssp(g, src)
    d = d.cpu().numpy()
    nd = int(np.count_nonzero(d != ref_d))
    assert nd == 0, f"{tag}: {nd} distances differ"
    if p is not None:
        npd = int(np.count_nonzero(p.cpu().numpy() != ref_p))
        assert npd == 0, f"{tag}: {npd} predecessors differ"


def with_pool(s, pool):
    return og.Schedule(**{**s.__dict__, "queue_pool": pool})


def test_chunks_are_recycled(orc):
    """Delta 16, unfused, a window of 4 buckets, on the 1024 x 1024 road
    grid: thousands of buckets, each filed and consumed in turn, through a
    pool of a few chunks per queue."""
    g = gg.road(1024, seed=0)
    dg = og.DeviceGraph.from_host(g, DEV)
    src = int(gg.pick_sources(g, 1, seed=21)[0])
    s = og.Schedule(delta=16, update=og.OG_EAGER_NO_FUSION, window_buckets=4)
    say("pool: road1024 delta=16 unfused K=4, default pool")
    d, p, st = og.sssp(dg, src, s)
    torch.cuda.synchronize()
    assert st["status"] == 0
    peak = st["pool_needed"]
    assert peak > 0 and peak % CHUNK == 0
    pool = 2 * peak
    say(f"pool: peak {peak} entries, rerun with pool {pool}")
    d, p, st = og.sssp(dg, src, with_pool(s, pool))
    torch.cuda.synchronize()
    assert st["status"] == 0
    assert st["pool_needed"] <= pool
    # far more entries went through the queues than the pool holds
    assert st["pushes_global"] > 4 * pool, (st["pushes_global"], pool)
    exact(orc, g, src, d, p, "recycled")


SCHEDULES = {
    "persistent_fused": og.Schedule(delta=64),
    "persistent_unfused": og.Schedule(delta=64, update=og.OG_EAGER_NO_FUSION),
    "host_rounds": og.Schedule(delta=64, engine=og.OG_ENGINE_HOST_ROUNDS),
    "graph_rounds": og.Schedule(delta=64, engine=og.OG_ENGINE_GRAPH_ROUNDS, update=og.OG_EAGER_NO_FUSION),
    "bins": og.Schedule(delta=64, flags=og.OG_FLAG_DEGREE_BINS),
    "light_heavy": og.Schedule(delta=64, update=og.OG_EAGER_NO_FUSION, flags=og.OG_FLAG_LIGHT_HEAVY),
    "lazy_hybrid": og.Schedule(delta=64, update=og.OG_LAZY_UPDATE, flags=og.OG_FLAG_HYBRID_DIRECTION),
    "blocks": og.Schedule(delta=64, flags=og.OG_FLAG_VERTEX_BLOCKS),
    "small_window": og.Schedule(delta=8, window_buckets=2),
}


@pytest.mark.parametrize("kind", ["road", "rmat"])
@pytest.mark.parametrize("name", list(SCHEDULES))
def test_every_engine_on_twice_its_peak(orc, road256, rmat14, kind, name):
    g, dg = road256 if kind == "road" else rmat14
    src = int(gg.pick_sources(g, 1, seed=22)[0])
    s = SCHEDULES[name]
    say(f"pool: {kind} {name} default pool")
    d, p, st = og.sssp(dg, src, s)
    torch.cuda.synchronize()
    assert st["status"] == 0
    exact(orc, g, src, d, p, f"{kind} {name} default")
    pool = 2 * st["pool_needed"]
    say(f"pool: {kind} {name} pool {pool}")
    d, p, st = og.sssp(dg, src, with_pool(s, pool))
    torch.cuda.synchronize()
    assert st["status"] == 0
    assert st["pool_needed"] <= -(-pool // CHUNK) * CHUNK
    exact(orc, g, src, d, p, f"{kind} {name} pool={pool}")


def test_kcore_and_batch_on_small_pools(orc, road256, rmat14):
    g, dg = rmat14
    for update in (og.OG_LAZY_UPDATE, og.OG_EAGER_NO_FUSION):
        say(f"pool: kcore rmat14 update={update}")
        core, st = og.kcore(dg, og.Schedule(update=update))
        assert st["status"] == 0
        pool = 2 * st["pool_needed"]
        core, st = og.kcore(dg, og.Schedule(update=update, queue_pool=pool))
        assert st["status"] == 0
        assert np.array_equal(core.cpu().numpy(), orc.kcore(g))
    g, dg = road256
    srcs = gg.pick_sources(g, 16, seed=23)
    s = og.Schedule(delta=128)
    say("pool: road256 batch of 16")
    d, p, st = og.sssp_batch(dg, srcs, s)
    torch.cuda.synchronize()
    assert st["status"] == 0
    pool = 2 * st["pool_needed"]
    d, p, st = og.sssp_batch(dg, srcs, with_pool(s, pool))
    torch.cuda.synchronize()
    assert st["status"] == 0
    for i in (0, 7, 15):
        exact(orc, g, int(srcs[i]), d[i], p[i], f"batch query {i}")


@pytest.mark.parametrize("name", ["persistent_unfused", "host_rounds", "bins", "blocks"])
def test_exhausted_pool_is_reported(orc, rmat14, name):
    """Two chunks (the sources' one and one more) cannot hold the queues of
    Delta 1 on R-MAT 14 (each of the 16 window buckets takes a chunk of its
    own): OG_ERR_WORKSPACE, with a peak above the pool; the same workspace
    then serves a call with the default pool exactly."""
    g, dg = rmat14
    s = og.Schedule(**{**SCHEDULES[name].__dict__, "delta": 1, "queue_pool": 1})
    ws = og.Workspace(DEV)
    src = int(gg.pick_sources(g, 1, seed=24)[0])
    say(f"pool: exhausted {name} src={src}")
    d, p, st = og.sssp(dg, src, s, ws=ws, check=False)
    torch.cuda.synchronize()
    assert st["status"] == og.OG_ERR_WORKSPACE
    assert st["pool_needed"] > 2 * CHUNK
    say(f"pool: {name} after exhaustion, default pool")
    d, p, st = og.sssp(dg, src, og.Schedule(**{**s.__dict__, "queue_pool": 0}), ws=ws)
    torch.cuda.synchronize()
    assert st["status"] == 0
    exact(orc, g, src, d, p, f"{name} after exhaustion")
