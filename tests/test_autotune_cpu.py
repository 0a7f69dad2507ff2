"""The schedule search finds the optimum of a synthetic cost surface (no
GPU: the runner is a plain function of the schedule)."""
import math

import pytest

from paper_1911_07260_amd import (OG_EAGER_NO_FUSION, OG_EAGER_WITH_FUSION, OG_ERR_HIP, OG_ERR_INTERNAL,
                                   OG_ERR_INVALID_ARG, OG_ERR_ROUND_LIMIT, OG_ERR_WORKSPACE, OG_FLAG_DEGREE_BINS,
                                   OG_FLAG_HYBRID_DIRECTION, OG_FLAG_VALIDATE, OG_LAZY_UPDATE, OgError, Schedule)
from paper_1911_07260_amd.autotune import Autotuner


def cost(s: Schedule) -> float:
    c = abs(math.log2(s.delta) - math.log2(724)) * 3.0        # best Delta ~ 724
    c += 0.0 if s.update == OG_EAGER_WITH_FUSION else 5.0
    c += {0: 0.5, 64: 2.0, 256: 0.0, 512: 0.3}.get(s.fusion_threshold, 1.0)
    c += {0: 0.2, 8: 0.4, 32: 0.0}.get(s.window_buckets, 1.0)
    c += {0: 0.0, 256: 1.0, 512: 0.5, 1024: 0.2}.get(s.workgroups, 1.0)
    return 10.0 + c


def test_search_finds_synthetic_optimum():
    tuner = Autotuner(cost)
    res = tuner.tune(weight_scale=15.0)
    assert res.best.update == OG_EAGER_WITH_FUSION
    assert res.best.fusion_threshold == 256
    assert res.best.delta in (724, 512, 1024)
    assert res.best_ms == min(t.engine_ms for t in res.trials)
    assert len(res.trials) < 60
    js = res.to_json()
    assert '"best_ms"' in js


@pytest.mark.parametrize("status", [OG_ERR_WORKSPACE, OG_ERR_ROUND_LIMIT])
def test_failing_candidates_are_skipped(status):
    """A candidate whose queues overflow the workspace, or that runs out of
    rounds, is a bad schedule: it is logged and the search goes on."""
    def runner(s):
        if s.update == OG_EAGER_NO_FUSION:
            raise OgError(status, "og_sssp")
        return cost(s)
    res = Autotuner(runner).tune(weight_scale=15.0)
    assert res.best.update == OG_EAGER_WITH_FUSION
    assert any(not t.ok for t in res.trials)


@pytest.mark.parametrize("status", [OG_ERR_INTERNAL, OG_ERR_HIP, OG_ERR_INVALID_ARG])
def test_library_errors_propagate(status):
    """A library bug (failed internal check), a HIP failure or an invalid
    argument is not tuned around: it leaves tune() at once."""
    calls = []

    def runner(s):
        calls.append(s)
        if len(calls) == 3:
            raise OgError(status, "og_sssp")
        return cost(s)
    with pytest.raises(OgError) as e:
        Autotuner(runner).tune(weight_scale=15.0)
    assert e.value.status == status
    assert len(calls) == 3


def test_other_exceptions_propagate():
    def runner(s):
        raise RuntimeError("not a library status")
    with pytest.raises(RuntimeError):
        Autotuner(runner).tune(weight_scale=15.0)


def test_lazy_and_direction_candidates():
    """With lazy=True the search also times the lazy update, pushing and with
    the hybrid direction, and returns the direction flag it chose next to the
    caller's own flags."""
    def runner(s):
        c = cost(Schedule(**{**s.__dict__, "update": OG_EAGER_WITH_FUSION}))
        if s.update == OG_LAZY_UPDATE:
            c -= 4.0 if s.flags & OG_FLAG_HYBRID_DIRECTION else 1.0
        return c
    res = Autotuner(runner, base=Schedule(flags=OG_FLAG_VALIDATE)).tune(weight_scale=15.0, lazy=True)
    assert res.best.update == OG_LAZY_UPDATE
    assert res.best.flags == OG_FLAG_VALIDATE | OG_FLAG_HYBRID_DIRECTION
    assert any(t.schedule["update"] == OG_LAZY_UPDATE and not t.schedule["flags"] & OG_FLAG_HYBRID_DIRECTION
               for t in res.trials)
    # without lazy=True the eager strategies only
    res = Autotuner(runner).tune(weight_scale=15.0)
    assert res.best.update == OG_EAGER_WITH_FUSION and res.best.flags == 0


def test_degree_bin_cutoffs():
    """The last stage times the degree bins at each pair of cut-offs and keeps
    the best, with its flag."""
    def runner(s):
        c = cost(s)
        if s.flags & OG_FLAG_DEGREE_BINS:
            c -= 0.5 + (0.5 if (s.bin_thread, s.bin_wave) == (4, 16) else 0.0)
        return c
    res = Autotuner(runner, base=Schedule(flags=OG_FLAG_VALIDATE)).tune(weight_scale=15.0)
    assert res.best.flags == OG_FLAG_VALIDATE | OG_FLAG_DEGREE_BINS
    assert (res.best.bin_thread, res.best.bin_wave) == (4, 16)
    # bins that do not pay are left out
    res = Autotuner(cost).tune(weight_scale=15.0)
    assert not res.best.flags & OG_FLAG_DEGREE_BINS


def test_team_count_for_batched_runners():
    """A batched runner's search ends with the team count; a single-query
    runner never varies it."""
    def runner(s):
        return cost(s) + {0: 0.3, 1: 1.0, 2: 0.6, 4: 0.0, 8: 0.2}[s.teams]
    res = Autotuner(runner, batched=True).tune(weight_scale=15.0)
    assert res.best.teams == 4
    assert {t.schedule["teams"] for t in res.trials} == {0, 1, 2, 4, 8}
    res = Autotuner(runner).tune(weight_scale=15.0)
    assert res.best.teams == 0 and all(t.schedule["teams"] == 0 for t in res.trials)
