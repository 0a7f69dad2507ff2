"""Schedule autotuner for the bucket engine.

The paper tunes its schedules with an ensemble search (section 5.3, OpenTuner
with an area-under-curve bandit) over the scheduling-language options.  This
is a smaller, deterministic search written for this engine: every candidate
is run through the C ABI on a few sample queries and timed with the
library's HIP events (`OG_FLAG_TIMING`, bucket-engine time only); the search
is

  1. Delta on a coarse power-of-two ladder around the weight scale, with
     and without bucket fusion (the two eager update strategies of section
     4.2), and optionally the lazy update pushing or with the
     SparsePush-DensePull hybrid direction (section 4.2; symmetric graphs);
  2. the fusion threshold and the window size around the best candidate;
  3. Delta refined by factors of sqrt(2) around the best value;
  4. the workgroup count;
  5. degree-binned load balancing and its two cut-offs (lane and wavefront
     bins; eager schedules);
  6. for batched runners, the number of workgroup teams (each team serves
     its own queries with rounds of its own).

Each stage keeps the best candidate (lowest median engine time).  Results
are returned as a `Schedule` plus a log of every candidate tried and can be
saved as JSON.
"""
from __future__ import annotations

import json
import math
import time
from dataclasses import asdict, dataclass, field

import numpy as np
import torch

from . import (OG_EAGER_NO_FUSION, OG_EAGER_WITH_FUSION, OG_ERR_ROUND_LIMIT, OG_ERR_WORKSPACE, OG_FLAG_DEGREE_BINS,
               OG_FLAG_DENSE_PULL, OG_FLAG_HYBRID_DIRECTION, OG_FLAG_TIMING, OG_LAZY_UPDATE, DeviceGraph, OgError,
               Schedule, Workspace, astar_batch, ppsp_batch, sssp, sssp_batch)

# Statuses that make a candidate a bad schedule rather than a failure: its
# queues overflowed the workspace, or it needed more rounds than the base
# schedule allows.  Every other error (an invalid argument, a HIP failure,
# an internal consistency check) is raised to the caller.
_CANDIDATE_ERRORS = (OG_ERR_WORKSPACE, OG_ERR_ROUND_LIMIT)

_DIRECTIONS = OG_FLAG_DENSE_PULL | OG_FLAG_HYBRID_DIRECTION
_CHOSEN = _DIRECTIONS | OG_FLAG_DEGREE_BINS  # flags the search may set


@dataclass
class Trial:
    schedule: dict
    engine_ms: float
    ok: bool


@dataclass
class TuneResult:
    best: Schedule
    best_ms: float
    trials: list = field(default_factory=list)
    seconds: float = 0.0

    def to_json(self) -> str:
        return json.dumps({"best": asdict(self.best), "best_ms": self.best_ms, "seconds": self.seconds,
                           "trials": [asdict(t) for t in self.trials]}, indent=1)

    def save(self, path: str) -> None:
        with open(path, "w") as f:
            f.write(self.to_json())


class Autotuner:
    """Times candidate schedules for one workload.

    `runner(schedule) -> engine_ms` may be given directly; `for_sssp`,
    `for_batch` and `for_ppsp_batch` build runners for the library's entry
    points on sample sources.
    """

    def __init__(self, runner, base: Schedule | None = None, repeats: int = 1, batched: bool = False):
        self.runner = runner
        self.base = base or Schedule()
        self.repeats = repeats
        self.batched = batched  # the runner launches several queries at once: the team count matters
        self.trials: list[Trial] = []
        self._cache: dict = {}

    # ---------------------------------------------------------- builders
    @classmethod
    def for_sssp(cls, graph: DeviceGraph, sources, **kw):
        ws = Workspace(graph.device)

        def run(s: Schedule) -> float:
            t = []
            for src in sources:
                _, _, st = sssp(graph, int(src), s, pred=False, ws=ws)
                t.append(st["engine_ms"])
            return float(np.median(t))

        return cls(run, **kw)

    @classmethod
    def for_batch(cls, graph: DeviceGraph, sources, **kw):
        ws = Workspace(graph.device)

        def run(s: Schedule) -> float:
            _, _, st = sssp_batch(graph, sources, s, pred=False, ws=ws)
            return float(st["engine_ms"])

        return cls(run, batched=len(sources) > 1, **kw)

    @classmethod
    def for_ppsp_batch(cls, graph: DeviceGraph, sources, targets, h: torch.Tensor | None = None, **kw):
        ws = Workspace(graph.device)

        def run(s: Schedule) -> float:
            if h is None:
                _, _, st = ppsp_batch(graph, sources, targets, s, pred=False, ws=ws)
            else:
                _, _, st = astar_batch(graph, sources, targets, h, s, pred=False, ws=ws)
            return float(st["engine_ms"])

        return cls(run, batched=len(sources) > 1, **kw)

    # ------------------------------------------------------------ search
    def measure(self, s: Schedule) -> float:
        key = tuple(sorted(asdict(s).items()))
        if key in self._cache:
            return self._cache[key]
        s = Schedule(**{**asdict(s), "flags": s.flags | OG_FLAG_TIMING})
        ms = []
        ok = True
        for _ in range(self.repeats):
            try:
                ms.append(self.runner(s))
            except OgError as e:
                if e.status not in _CANDIDATE_ERRORS:
                    raise
                ok = False
                break
        val = float(np.median(ms)) if ok else math.inf
        self._cache[key] = val
        self.trials.append(Trial(asdict(s), val, ok))
        return val

    def _best(self, cands):
        scored = [(self.measure(c), i, c) for i, c in enumerate(cands)]
        scored.sort(key=lambda x: (x[0], x[1]))
        return scored[0][2], scored[0][0]

    def tune(self, weight_scale: float, hop_weight: float | None = None, lazy: bool = False) -> TuneResult:
        """weight_scale: a typical edge weight (e.g. the median); the Delta
        ladder spans weight_scale/16 .. weight_scale*1024.  lazy: also try
        the lazy update, pushing and with the hybrid direction (the graph
        must then be symmetric)."""
        t0 = time.perf_counter()
        base = self.base
        lo = max(1, int(weight_scale / 16))
        deltas = sorted({1 << k for k in range(max(0, int(math.log2(lo))), int(math.log2(weight_scale * 1024)) + 1)})
        modes = [(OG_EAGER_WITH_FUSION, 0), (OG_EAGER_NO_FUSION, 0)]
        if lazy:
            modes += [(OG_LAZY_UPDATE, 0), (OG_LAZY_UPDATE, OG_FLAG_HYBRID_DIRECTION)]
        cands = [Schedule(**{**asdict(base), "delta": d, "update": u, "flags": (base.flags & ~_DIRECTIONS) | fl})
                 for d in deltas for u, fl in modes]
        best, best_ms = self._best(cands)
        # threshold / window around the best
        cands = [best]
        if best.update == OG_EAGER_WITH_FUSION:
            cands += [Schedule(**{**asdict(best), "fusion_threshold": t}) for t in (64, 256, 512)]
        cands += [Schedule(**{**asdict(best), "window_buckets": k}) for k in (8, 32)]
        best, best_ms = self._best(cands)
        # refine Delta by sqrt(2)
        cands = [best] + [Schedule(**{**asdict(best), "delta": max(1, int(round(best.delta * f)))})
                          for f in (0.5, 0.7071, 1.4142, 2.0)]
        best, best_ms = self._best(cands)
        # workgroups
        cands = [best] + [Schedule(**{**asdict(best), "workgroups": w}) for w in (256, 512, 1024)]
        best, best_ms = self._best(cands)
        # degree bins (not with a pull direction)
        if not best.flags & _DIRECTIONS:
            cands = [best] + [Schedule(**{**asdict(best), "flags": best.flags | OG_FLAG_DEGREE_BINS, "bin_thread": bt,
                                          "bin_wave": bw}) for bt in (2, 4) for bw in (16, 64, 256)]
            best, best_ms = self._best(cands)
        # teams of workgroups (batched launches of the eager engine; 0 = the
        # library's default, one per query up to 8)
        if self.batched and best.update != OG_LAZY_UPDATE:
            cands = [best] + [Schedule(**{**asdict(best), "teams": t}) for t in (1, 2, 4, 8) if t != best.teams]
            best, best_ms = self._best(cands)
        best = Schedule(**{**asdict(best), "flags": (base.flags & ~_CHOSEN) | (best.flags & _CHOSEN)})
        return TuneResult(best=best, best_ms=best_ms, trials=list(self.trials), seconds=time.perf_counter() - t0)
