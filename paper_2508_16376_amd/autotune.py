"""Autotuner for the two-dimensional schedule.

Chooses, per design (or campaign) and fault population, the parameters that
decide where work runs: whether idle wavefronts take handed-over faults
during the light launch (the unified schedule), the events-per-cycle
threshold of the light-lane monitor, the light-lane capacity, whether lanes
start their cycles in step, the number of resident wavefronts per compute
unit, how many of them share one structural workspace, how many wavefronts
simulate one structural fault together, how the head of the light queue
spreads over the wavefronts (dealt out, or taken in one batch per
wavefront), whether each XCD takes faults from its own queue, and (with a
predictor) the predicted-load quantile above which faults start on the
structural path.  The paper fixes its overload threshold by hand (Sec.
V-A); here candidates are timed and the fastest kept, one parameter at a
time (coordinate descent, with the unified schedule moved together with
workspace sharing), with the result cached by design hash.  Candidates run
on a seeded sample of the fault list (by default the whole list): the
sample must keep more faults than the chip has lanes, or it would hide the
contention of the structural path and pick thresholds that fail at full
scale; the parameters that depend on how many faults are in flight are then
descended again on the whole list.  A wall-clock budget bounds each
descent: once it is spent the best point so far is confirmed and kept.  No
parameter changes a result, only time.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import numpy as np

from . import riros

# Descent order: the monitor and capacity first (they decide how much work
# reaches the structural path), then whether light lanes start their cycles
# in step, whether idle wavefronts take handed-over work during the light
# launch, then occupancy, sharing and the structural workgroup size, and
# how the head of the light queue spreads over the wavefronts (dealt out, or
# taken a few to a wavefront).
SPACE = {
    "monitor_rate": [0.0, 1.0, 2.0, 4.0, 8.0],
    "light_cap": [4, 8],
    "lockstep": [1, 0],
    "unified": [1, 0],
    "waves_per_cu": [8, 12, 16],
    "struct_share": [1, 2, 4],
    "heavy_wg": [64, 128, 256],
    "deal": [0, 8, 32],
    "head_lanes": [0, 32, 16, 64],
    "xcd_queues": [0, 1],
    "heavy_quantile": [None, 0.99, 0.9, 0.6, 0.0],
}
# Parameters whose best value depends on how many faults are in flight (or,
# for the head batch, how many heavy faults there are to spread; for the
# monitor, how many faults reach the structural path, which pays together
# with the unified schedule or not at all).
SCALE_PARAMS = ("monitor_rate", "lockstep", "unified", "waves_per_cu", "struct_share", "heavy_wg", "head_lanes")
# Parameters that pay only together with another's value: the unified
# schedule needs workspaces shared by several wavefronts (one workspace per
# wavefront holds too few of them resident), so each unified value is tried
# with every sharing value.
JOINT = {"unified": "struct_share"}
# Candidate values on the whole list, where a low monitor rate hands most of
# a million faults to the structural path and a candidate takes seconds.
WHOLE_LIST_VALUES = {"monitor_rate": [0.0, 4.0, 8.0]}
DEFAULT = {"unified": 1, "monitor_rate": 2.0, "light_cap": 8, "waves_per_cu": 12, "struct_share": 1,
           "heavy_wg": 64, "lockstep": 1, "deal": 0, "head_lanes": 0,
           "xcd_queues": 0, "heavy_quantile": None}


def design_key(design, T: int, F: int, with_priority: bool) -> str:
    h = hashlib.sha1(np.ascontiguousarray(design.nodes).tobytes())
    h.update(np.ascontiguousarray(design.po).tobytes())
    return f"{h.hexdigest()[:16]}-T{T}-F{F}-p{int(with_priority)}"


def _opts(p, priority):
    theta = math.inf
    if priority is not None and p["heavy_quantile"] is not None:
        theta = float(np.quantile(priority, p["heavy_quantile"]))
    return {"monitor_rate": p["monitor_rate"], "light_cap": p["light_cap"], "waves_per_cu": p["waves_per_cu"],
            "unified": p.get("unified", 0), "struct_share": p.get("struct_share", 0),
            "heavy_wg": p.get("heavy_wg", 0), "lockstep": p.get("lockstep", 0), "deal": p.get("deal", 0),
            "head_lanes": p.get("head_lanes", 0), "xcd_queues": p.get("xcd_queues", 0), "theta": theta}


def _time_single(d, g, faults, priority, p, reps=2, drop=True):
    """Best of ``reps`` timed runs after one untimed run (the first launch of a
    kernel instance pays for loading its code object)."""
    kw = _opts(p, priority)
    riros.fault_sim(d, g, faults, mode=riros.MODE_TWO_D, drop=drop, priority=priority, with_events=False, **kw)
    best = math.inf
    for _ in range(reps):
        riros.fault_sim(d, g, faults, mode=riros.MODE_TWO_D, drop=drop, priority=priority, with_events=False, **kw)
        best = min(best, riros.last_kernel_ms())
    return best


class Autotuner:
    def __init__(self, cache_path: str | None = None, progress=None, budget_s: float | None = None):
        """progress: optional callable taking one line of text per timed
        point (a long tuning run then reports as it goes).  budget_s: wall
        time after which no new point is timed (the confirmation of the best
        points still runs)."""
        self.progress = progress
        self.budget_s = budget_s
        self.cache_path = cache_path
        self.cache: dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)
        self.log: list[dict] = []

    def _save(self):
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)

    def _descend(self, measure, with_priority: bool, confirm: int = 3, start=None, names=None, values=None):
        """Coordinate descent from ``start`` (default DEFAULT) over the
        parameters in ``names``, in that order (default every one of SPACE,
        in SPACE's order), with the
        candidate values of ``values`` where it names a parameter (default
        SPACE's).  A parameter of JOINT is tried with every value of its
        partner when the partner is descended too."""
        t_start = time.perf_counter()

        def spent():
            return self.budget_s is not None and time.perf_counter() - t_start > self.budget_s

        best = dict(DEFAULT if start is None else start)
        best_t = measure(best)
        self.log.append({"params": dict(best), "ms": best_t})
        timed = [(best_t, dict(best))]
        seen = {tuple(sorted(best.items(), key=lambda kv: kv[0]))}
        # Two passes at most: a parameter chosen early (say the monitor rate)
        # may lose its worth once a later one moves (most faults starting on
        # the structural path); the second pass only times unseen points.
        for _ in range(2):
            start = dict(best)
            for name in (SPACE if names is None else names):
                space_values = SPACE[name]
                if name == "heavy_quantile" and not with_priority:
                    continue
                vals = (values or {}).get(name, space_values)
                partner = JOINT.get(name)
                if partner is not None and names is not None and partner not in names:
                    partner = None
                moves = [{name: v} for v in vals] if partner is None else \
                    [{name: v, partner: w} for v in vals for w in (values or {}).get(partner, SPACE[partner])]
                for mv in moves:
                    cand = dict(best)
                    cand.update(mv)
                    key = tuple(sorted(cand.items(), key=lambda kv: kv[0]))
                    if key in seen or spent():
                        continue
                    seen.add(key)
                    t = measure(cand)
                    self.log.append({"params": dict(cand), "ms": t})
                    timed.append((t, dict(cand)))
                    if self.progress:
                        self.progress(f"[autotune] {cand} {t:.3f} ms")
                    if t < best_t:
                        best, best_t = cand, t
            if best == start or spent():
                break
        # The fastest few points are timed twice more and ranked by their
        # mean: a single lucky timing should not pick the schedule.
        if confirm > 1:
            top = sorted(timed, key=lambda x: x[0])[:confirm]
            scored = []
            for t0, p in top:
                ts = [t0] + [measure(p) for _ in range(2)]
                scored.append((sum(ts) / len(ts), min(ts), p))
                if self.progress:
                    self.progress(f"[autotune] confirm {p} mean {scored[-1][0]:.3f} ms")
            _, best_t, best = min(scored, key=lambda x: x[0])
        return best, best_t

    def tune_single(self, design_np, d, g, faults, priority=None, T=None, sample=None, drop=True, start=None,
                    names=None):
        """Parameters for riros_fault_sim(mode=TWO_D) on this design and fault
        list.  sample: time the candidates on these fault indexes only.  drop:
        the detect-and-drop convention the parameters are for.  start, names:
        descend from ``start`` over these parameters only (default: from
        DEFAULT over every one)."""
        key = design_key(design_np, T or 0, faults.size, priority is not None)
        if sample is not None:
            key += f"-s{len(sample)}"
        if not drop:
            key += "-nodrop"
        if names is not None:
            key += "-" + "-".join(names)
        if key in self.cache:
            return self.cache[key]["params"]
        full_ps = None if priority is None else np.ascontiguousarray(priority, dtype=np.float32)
        full = faults
        if sample is not None:
            faults = np.ascontiguousarray(faults[sample])
            priority = None if priority is None else priority[sample]
        ps = None if priority is None else np.ascontiguousarray(priority, dtype=np.float32)
        best, t = self._descend(lambda p: _time_single(d, g, faults, ps, p, drop=drop), priority is not None,
                                start=start, names=names)
        if sample is not None and names is None:
            # Occupancy, workspace sharing, the structural workgroup size and
            # lockstep trade against contention, which grows with the number
            # of faults in flight: a sample holding a fraction of the list
            # favours fewer resident wavefronts than the whole list does.  The
            # head batch's size decides how the heavy faults, a fixed share
            # of the list, spread over the wavefronts, and the monitor how
            # many faults the structural path takes, which pays only together
            # with the unified schedule.  These are descended again on the
            # whole list from the sample's best point; the capacity and the
            # queue options keep the sample's choice.
            best, t = self._descend(lambda p: _time_single(d, g, full, full_ps, p, drop=drop), priority is not None,
                                    start=best, names=SCALE_PARAMS, values=WHOLE_LIST_VALUES)
        self.cache[key] = {"params": best, "ms": t}
        self._save()
        return best

    def tune_batch(self, designs_np, ds, gs, fault_lists, priorities=None):
        """Parameters for a campaign (riros_batch_create)."""
        h = hashlib.sha1()
        for dn, fl in zip(designs_np, fault_lists):
            h.update(np.ascontiguousarray(dn.nodes).tobytes())
            h.update(np.int64(fl.size).tobytes())
        key = f"batch-{h.hexdigest()[:16]}-p{int(priorities is not None)}"
        if key in self.cache:
            return self.cache[key]["params"]
        prs = None if priorities is None else [np.ascontiguousarray(p, dtype=np.float32) for p in priorities]
        allp = None if prs is None else np.concatenate(prs)

        def measure(p):
            kw = _opts(p, allp)
            b = riros.Batch(ds, gs, fault_lists, prs, **kw)
            t = math.inf
            for _ in range(2):      # the first launch also loads code objects
                b.launch()
                b.read(0)
                t = min(t, riros.last_kernel_ms())
            b.close()
            return t

        best, t = self._descend(measure, priorities is not None)
        self.cache[key] = {"params": best, "sample_ms": t}
        self._save()
        return best


def batch_kwargs(params, priorities_concat=None):
    """riros.Batch keyword arguments for tuned parameters."""
    return _opts(params, priorities_concat)


def single_kwargs(params, priority=None):
    return _opts(params, priority)
