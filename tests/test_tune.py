"""Search logic of the autotuner (no GPU): coordinate descent over launch
knobs with measured times, time-limited trials and a counts check."""
import math

import pytest

from paper_2004_02369_amd import tune

SPACE = {"a": [1, 2, 3, 4, 5], "b": [10, 20, 30], "c": [0, 1]}


def _measure_from(cost, counts=(7, 9), calls=None):
    def measure(knobs, limit_ms):
        if calls is not None:
            calls.append((dict(knobs), limit_ms))
        ms = cost(knobs)
        if limit_ms and ms > limit_ms:
            return None, math.inf
        return list(counts), ms
    return measure


def test_search_finds_separable_optimum():
    cost = lambda k: 100 + (k["a"] - 4) ** 2 * 10 + abs(k["b"] - 20) + 5 * k["c"]
    best, ms, trials = tune.search(_measure_from(cost), SPACE, start={"a": 1, "b": 10, "c": 1})
    assert best == {"a": 4, "b": 20, "c": 0} and ms == 100
    assert trials[0] == ({"a": 1, "b": 10, "c": 1}, cost({"a": 1, "b": 10, "c": 1}))
    # no configuration is measured twice
    keys = [tuple(sorted(k.items())) for k, _ in trials]
    assert len(keys) == len(set(keys))


def test_search_cuts_slow_trials_with_a_time_limit():
    calls = []
    cost = lambda k: 1000.0 if k["a"] == 5 else 50.0 + k["a"]
    best, ms, trials = tune.search(_measure_from(cost, calls=calls), SPACE, start={"a": 3, "b": 10, "c": 0})
    assert calls[0][1] == 0                      # the starting point once without a limit,
    assert all(lim > 0 for _, lim in calls[1:])  # then like every trial, under one
    slow = [t for k, t in trials if k["a"] == 5]
    assert slow and all(math.isinf(t) for t in slow)
    assert best["a"] == 1 and ms == 51.0


def test_search_rejects_inconsistent_counts():
    def measure(knobs, limit_ms):
        return ([1, 2] if knobs["a"] != 2 else [1, 3]), 10.0 - knobs["a"]
    with pytest.raises(tune.InconsistentCounts):
        tune.search(measure, SPACE, start={"a": 1, "b": 10, "c": 0})


def test_search_respects_budget():
    best, ms, trials = tune.search(_measure_from(lambda k: 5.0), SPACE, start={"a": 1, "b": 10, "c": 0},
                                   budget_s=0.0)
    assert len(trials) == 1 and best == {"a": 1, "b": 10, "c": 0}


def test_default_space_is_valid_launch_knobs():
    from paper_2004_02369_amd import pg
    assert set(tune.SPACE) <= set(pg.RUN_KNOBS) and set(tune.DEFAULT) == set(tune.SPACE)
    assert 0 in tune.SPACE["hub_min_degree"] and -1 in tune.SPACE["hub_min_degree"]
    assert tune.SPACE["flags"] == [0, pg.PG_RUN_NO_TASK_BATCH, pg.PG_RUN_LIGHT_KERNEL]
