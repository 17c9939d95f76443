"""Host logic of the autotuner: coordinate descent over the schedule space."""
import numpy as np

from paper_2508_16376_amd import autotune


def test_descent_finds_the_coordinatewise_minimum():
    calls = []

    def cost(p):
        calls.append(dict(p))
        c = abs(p["monitor_rate"] - 4.0) + (0 if p["light_cap"] == 4 else 1) + abs(p["waves_per_cu"] - 16) / 4
        c += 0 if p["heavy_quantile"] == 0.99 else 0.5
        c += 0 if p["unified"] == 0 else 0.25
        c += 0 if p["heavy_wg"] == 128 else 0.125
        c += 0 if p["deal"] == 8 else 0.0625
        c += 0 if p["head_lanes"] == 16 else 0.03125
        c += 0 if p["xcd_queues"] == 1 else 0.015625
        return c

    t = autotune.Autotuner()
    best, bt = t._descend(cost, with_priority=True)
    assert best == {"unified": 0, "monitor_rate": 4.0, "light_cap": 4, "waves_per_cu": 16, "struct_share": 1,
                    "heavy_wg": 128, "lockstep": 1, "deal": 8, "head_lanes": 16,
                    "xcd_queues": 1, "heavy_quantile": 0.99}
    assert bt == 0
    # every candidate is a point of the space; the descent times no point
    # twice, and then the three fastest points are timed twice more each
    keys = [tuple(sorted(c.items(), key=lambda kv: kv[0])) for c in calls]
    distinct = len(set(keys))
    assert len(keys) == distinct + 2 * min(3, distinct)
    assert keys[:distinct] == list(dict.fromkeys(keys))
    for c in calls:
        for k, v in c.items():
            assert v in autotune.SPACE[k] or v == autotune.DEFAULT[k]


def test_no_predictor_keeps_every_fault_light_first():
    t = autotune.Autotuner()
    best, _ = t._descend(lambda p: 1.0 if p["heavy_quantile"] is None else 0.0, with_priority=False)
    assert best["heavy_quantile"] is None
    kw = autotune.single_kwargs(best, None)
    assert kw["theta"] == float("inf")


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    t = autotune.Autotuner(path)
    t.cache["k"] = {"params": dict(autotune.DEFAULT)}
    t._save()
    assert autotune.Autotuner(path).cache["k"]["params"] == autotune.DEFAULT


def test_confirmation_ranks_by_mean_not_by_a_lucky_timing():
    """A point that timed fast once but is slow on average loses to a point
    that is steadily fast."""
    lucky = {"monitor_rate": 1.0}
    seen = {}

    def cost(p):
        k = tuple(sorted(p.items(), key=lambda kv: kv[0]))
        seen[k] = seen.get(k, 0) + 1
        if dict(p, monitor_rate=2.0) == autotune.DEFAULT and p["monitor_rate"] == 1.0:
            return 1.0 if seen[k] == 1 else 10.0     # one point, fast only the first time
        return 3.0 if p["monitor_rate"] == 4.0 else 5.0

    t = autotune.Autotuner()
    best, bt = t._descend(cost, with_priority=False)
    assert best["monitor_rate"] == 4.0
    assert bt == 3.0
    assert lucky["monitor_rate"] != best["monitor_rate"]


def test_budget_stops_the_descent_and_keeps_the_best_so_far():
    """Once the wall budget is spent no new point is timed; the confirmation
    of the fastest points still runs."""
    import time
    calls = []

    def cost(p):
        calls.append(dict(p))
        time.sleep(0.02)
        return 1.0 if p["monitor_rate"] == 1.0 else 2.0

    t = autotune.Autotuner(budget_s=0.05)
    best, _ = t._descend(cost, with_priority=True)
    distinct = len({tuple(sorted(c.items(), key=lambda kv: kv[0])) for c in calls})
    assert distinct <= 5
    assert best["monitor_rate"] in (1.0, 2.0)


def test_sampled_tuning_redoes_the_scale_parameters_on_the_whole_list(monkeypatch):
    """With a sample, the capacity keeps the sample's choice, and occupancy
    (with the monitor and the other contention parameters) is descended again
    on the whole list, where the sample's best occupancy is not the whole
    list's."""
    from paper_2508_16376_amd import workloads as W
    d = W.gen_templates(5, n_nodes=300, name="t")
    faults = W.gen_faults(5, d, 400)
    sample = np.arange(0, 400, 4)
    sizes = []

    def fake_time(dd, g, fl, ps, p, drop=True):
        sizes.append(fl.size)
        t = 10.0 if p["monitor_rate"] == 0.0 else 20.0
        t += 0.5 if p["light_cap"] == 4 else 1.0
        best_wpc = 8 if fl.size == sample.size else 16
        return t + (0.0 if p["waves_per_cu"] == best_wpc else 2.0)

    monkeypatch.setattr(autotune, "_time_single", fake_time)
    t = autotune.Autotuner()
    best = t.tune_single(d, None, None, faults, priority=None, T=10, sample=sample)
    assert best["monitor_rate"] == 0.0 and best["light_cap"] == 4
    assert best["waves_per_cu"] == 16
    assert sample.size in sizes and faults.size in sizes
    # The whole list only times the scale parameters: the capacity and the
    # queue options stay at the sample's choice in every point timed there.
    assert sizes.index(faults.size) > 0 and all(s == faults.size for s in sizes[sizes.index(faults.size):])


def test_no_drop_tuning_descends_only_the_named_parameters(monkeypatch):
    """A descent restricted to some parameters, for the no-dropping
    convention, starts from the given point, times every candidate without
    dropping and changes nothing else."""
    from paper_2508_16376_amd import workloads as W
    d = W.gen_templates(6, n_nodes=300, name="t")
    faults = W.gen_faults(6, d, 300)
    seen = []

    def fake_time(dd, g, fl, ps, p, drop=True):
        seen.append((dict(p), drop))
        return (0.0 if p["light_cap"] == 8 else 1.0) + (0.0 if p["monitor_rate"] == 0.0 else 0.5)

    monkeypatch.setattr(autotune, "_time_single", fake_time)
    start = dict(autotune.DEFAULT, light_cap=4, monitor_rate=4.0, waves_per_cu=16, head_lanes=64)
    best = autotune.Autotuner().tune_single(d, None, None, faults, T=10, drop=False, start=start,
                                            names=("light_cap", "monitor_rate", "unified"))
    assert best["light_cap"] == 8 and best["monitor_rate"] == 0.0
    assert all(not dr for _, dr in seen)
    for p, _ in seen:
        assert {k: v for k, v in p.items() if k not in ("light_cap", "monitor_rate", "unified")} == \
            {k: v for k, v in start.items() if k not in ("light_cap", "monitor_rate", "unified")}


def test_unified_is_tried_with_every_workspace_sharing():
    """The unified schedule pays only with workspaces shared by four
    wavefronts: a one-at-a-time descent from one workspace per wavefront
    would never take it, the joint move does."""
    def cost(p):
        if p["unified"] == 1:
            return 1.0 if p["struct_share"] == 4 else 9.0
        return 5.0 + (0.0 if p["struct_share"] == 1 else 0.5)

    start = dict(autotune.DEFAULT, unified=0, struct_share=1)
    best, bt = autotune.Autotuner()._descend(cost, with_priority=False, start=start,
                                             names=("unified", "struct_share"))
    assert best["unified"] == 1 and best["struct_share"] == 4 and bt == 1.0


def test_whole_list_values_replace_the_space():
    """Candidate values given for the whole list replace SPACE's."""
    timed = []

    def cost(p):
        timed.append(p["monitor_rate"])
        return p["monitor_rate"]

    start = dict(autotune.DEFAULT, monitor_rate=4.0)
    autotune.Autotuner()._descend(cost, with_priority=False, start=start, names=("monitor_rate",),
                                  values=autotune.WHOLE_LIST_VALUES)
    assert set(timed) <= set(autotune.WHOLE_LIST_VALUES["monitor_rate"])


def test_named_descent_follows_the_given_order():
    """A restricted descent visits its parameters in the order given."""
    first_seen = []

    def cost(p):
        for k in ("heavy_wg", "light_cap", "unified", "monitor_rate"):
            if p[k] != start[k] and k not in first_seen:
                first_seen.append(k)
        return 1.0

    start = dict(autotune.DEFAULT)
    autotune.Autotuner()._descend(cost, with_priority=False, start=start,
                                  names=("light_cap", "heavy_wg", "unified", "monitor_rate"))
    assert first_seen == ["light_cap", "heavy_wg", "unified", "monitor_rate"]
