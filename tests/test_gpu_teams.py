"""Batched launches split into teams of workgroups (workgroup b serves team
b % teams, query q belongs to team q % teams, each team with its own bucket
lists, pool share and rounds): every team count, load balancing, update,
engine and grid size gives the oracle's distances and canonical
predecessors for every query, also when teams finish at different times.

Graphs: the 128 x 128 road-like grid (seed 3) and R-MAT scale 12.
"""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_1911_07260_amd as og

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def road128():
    g = gg.road(128, seed=3)
    return g, og.DeviceGraph.from_host(g, DEV)


@pytest.fixture(scope="module")
def rmat12():
    g = gg.rmat(12, 16, seed=0)
    return g, og.DeviceGraph.from_host(g, DEV)


def check_all(orc, g, srcs, d, p, tag):
    d, p = d.cpu().numpy(), p.cpu().numpy()
    for q, s in enumerate(srcs):
        rd, rp = orc.sssp(g, int(s))
        assert np.array_equal(d[q], rd), f"{tag}: query {q} distances"
        assert np.array_equal(p[q], rp), f"{tag}: query {q} predecessors"


@pytest.mark.parametrize("teams", [1, 2, 3, 8])
@pytest.mark.parametrize("flags", [0, og.OG_FLAG_DEGREE_BINS])
@pytest.mark.parametrize("update", [og.OG_EAGER_WITH_FUSION, og.OG_EAGER_NO_FUSION])
def test_team_counts(orc, road128, teams, flags, update):
    g, dg = road128
    srcs = gg.pick_sources(g, 8, seed=31)
    tag = f"road128 nq=8 teams={teams} flags={flags} update={update}"
    say(tag)
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=64, teams=teams, flags=flags, update=update))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check_all(orc, g, srcs, d, p, tag)


@pytest.mark.parametrize("engine", [og.OG_ENGINE_HOST_ROUNDS, og.OG_ENGINE_GRAPH_ROUNDS])
def test_teams_host_driven_rounds(orc, road128, engine):
    g, dg = road128
    srcs = gg.pick_sources(g, 8, seed=32)
    tag = f"road128 nq=8 teams=8 engine={engine}"
    say(tag)
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=64, engine=engine, flags=og.OG_FLAG_DEGREE_BINS))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check_all(orc, g, srcs, d, p, tag)


@pytest.mark.parametrize("workgroups", [1, 3, 5, 13])
def test_fewer_workgroups_than_teams(orc, road128, workgroups):
    """A grid of fewer workgroups than 8 runs as many teams as workgroups;
    13 workgroups make teams of two and of one."""
    g, dg = road128
    srcs = gg.pick_sources(g, 8, seed=33)
    tag = f"road128 nq=8 workgroups={workgroups}"
    say(tag)
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=64, workgroups=workgroups))
    torch.cuda.synchronize()
    assert st["status"] == 0 and st["workgroups"] == workgroups
    check_all(orc, g, srcs, d, p, tag)


@pytest.mark.parametrize("nq", [2, 11, 37])
def test_uneven_queries_per_team(orc, rmat12, nq):
    """Query counts that do not divide among 8 teams (2: two teams; 11 and
    37: teams of unequal query counts), on a power-law graph."""
    g, dg = rmat12
    srcs = gg.pick_sources(g, nq, seed=34)
    tag = f"rmat12 nq={nq}"
    say(tag)
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=32, flags=og.OG_FLAG_DEGREE_BINS))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check_all(orc, g, srcs, d, p, tag)


def test_teams_point_to_point_and_astar(orc, road128):
    g, dg = road128
    srcs = gg.pick_sources(g, 16, seed=35)
    dsts = gg.pick_sources(g, 16, seed=36)
    say("road128 ppsp_batch nq=16 teams=8")
    d, p, st = og.ppsp_batch(dg, srcs, dsts, og.Schedule(delta=64))
    torch.cuda.synchronize()
    assert st["status"] == 0
    got = d[torch.arange(16, device=DEV), torch.as_tensor(dsts, device=DEV)].cpu().numpy()
    want = np.array([orc.ppsp(g, int(s), int(t)) for s, t in zip(srcs, dsts)])
    want = np.where(want < 0, og.INF, want)
    assert np.array_equal(got, want)
    say("road128 astar_batch nq=16 teams=8")
    h = gg.grid_heuristic_device(128, dsts, DEV)
    d, p, st = og.astar_batch(dg, srcs, dsts, h, og.Schedule(delta=64))
    torch.cuda.synchronize()
    assert st["status"] == 0
    got = d[torch.arange(16, device=DEV), torch.as_tensor(dsts, device=DEV)].cpu().numpy()
    assert np.array_equal(got, want)


def test_lazy_batch_runs_one_team(orc, road128):
    """teams is a request: the lazy update keeps one set of queues."""
    g, dg = road128
    srcs = gg.pick_sources(g, 8, seed=37)
    say("road128 nq=8 lazy teams=8")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=64, update=og.OG_LAZY_UPDATE, teams=8))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check_all(orc, g, srcs, d, p, "lazy")


def test_teams_exhausted_pool(orc, rmat12):
    """Two chunks cannot hold 8 teams' queues: OG_ERR_WORKSPACE, then an
    exact call on the same workspace."""
    g, dg = rmat12
    srcs = gg.pick_sources(g, 8, seed=38)
    ws = og.Workspace(DEV)
    say("rmat12 nq=8 queue_pool=1")
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=1, queue_pool=1), ws=ws, check=False)
    torch.cuda.synchronize()
    assert st["status"] == og.OG_ERR_WORKSPACE
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=1), ws=ws)
    torch.cuda.synchronize()
    assert st["status"] == 0
    check_all(orc, g, srcs, d, p, "after exhaustion")


def test_teams_finishing_at_different_times(orc, road128):
    """Eight teams of one query each, where team 0's source is isolated (its
    team is done after one round) and team 1's source lies in the main grid:
    the finished team's workgroups leave while the others run on."""
    g, dg = road128
    iso = int(np.where(g.degrees() == 0)[0][0])
    srcs = [iso] + [int(s) for s in gg.pick_sources(g, 7, seed=39)]
    tag = f"road128 nq=8 teams=8, query 0 from isolated vertex {iso}"
    say(tag)
    d, p, st = og.sssp_batch(dg, srcs, og.Schedule(delta=64, teams=8, flags=og.OG_FLAG_DEGREE_BINS))
    torch.cuda.synchronize()
    assert st["status"] == 0
    check_all(orc, g, srcs, d, p, tag)
    # the rounds and barriers of the team that took the most (one barrier per
    # eager round)
    assert st["rounds"] >= 2 and st["barriers"] == st["rounds"]


@pytest.mark.parametrize("engine", [og.OG_ENGINE_PERSISTENT, og.OG_ENGINE_HOST_ROUNDS])
def test_teams_stop_early_on_their_own_targets(orc, road128, engine):
    """Point-to-point queries, one team each: team 0's target is its source
    (settled at the first decision), the others' targets are far away."""
    g, dg = road128
    srcs = [int(s) for s in gg.pick_sources(g, 8, seed=40)]
    dsts = [srcs[0]] + [int(t) for t in gg.pick_sources(g, 7, seed=41)]
    say(f"road128 ppsp_batch nq=8 teams=8 engine={engine}, query 0 target = source")
    d, p, st = og.ppsp_batch(dg, srcs, dsts, og.Schedule(delta=64, teams=8, engine=engine))
    torch.cuda.synchronize()
    assert st["status"] == 0
    got = d[torch.arange(8, device=DEV), torch.as_tensor(dsts, device=DEV)].cpu().numpy()
    want = np.array([orc.ppsp(g, int(s), int(t)) for s, t in zip(srcs, dsts)])
    want = np.where(want < 0, og.INF, want)
    assert got[0] == 0 and np.array_equal(got, want)
