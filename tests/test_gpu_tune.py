"""GPU tests of the tuned launch knobs: every setting of the per-degree
intersection variant (bitmap or binary search), claim chunk and task
batching gives the oracle's counts; the autotuner's choice does too, and its
cache returns the same choice."""
import os
import sys

import pytest

from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import patterns as pt

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pg():
    import torch
    assert torch.cuda.is_available()
    from paper_2004_02369_amd import pg as _pg
    _pg.lib()
    return _pg


SPECS = pt.all_vertex_induced(4) + [pt.clique(5), pt.P7_TRIANGLE_NO_K4, pt.PA_TWO_COMMON_FRIENDS,
                                    pt.all_vertex_induced(5)[15], pt.all_vertex_induced(5)[-3]]


@pytest.fixture(scope="module")
def case(orc):
    g = gg.chung_lu(3000, 20000, 2.1, 200.0, seed=31)
    og = orc.Graph.from_tuple(g)
    return g, [orc.count(og, s) for s in SPECS]


@pytest.mark.parametrize("load_min", [1, 0, 200, -1])
def test_knob_settings_match_oracle(pg, case, load_min):
    g, want = case
    G = pg.load_graph(*g, device=0, hub_min_degree=load_min)
    if load_min == -1:
        assert G.hub_count == 0
    elif load_min == 1:
        assert G.hub_count == sum(1 for d in _degrees(g) if d >= 1) and G.hub_min_degree == 1
    plans = [pg.plan_pattern(s) for s in SPECS]
    settings = [{}, {"hub_min_degree": -1}, {"hub_min_degree": 2}, {"hub_min_degree": 37},
                {"hub_min_degree": 10 ** 6}, {"chunk": 1}, {"chunk": 7}, {"chunk": 500},
                {"flags": pg.PG_RUN_NO_TASK_BATCH, "chunk": 3, "hub_min_degree": 50},
                {"grid_waves": 37, "chunk": 2}, {"batch_max_avg": 1}, {"batch_max_avg": 40, "chunk": 5},
                {"batch_max_avg": 3, "hub_min_degree": 20, "chunk": 16}]
    for knobs in settings:
        say(f"load hub_min_degree={load_min} knobs={knobs}")
        assert pg.count(G, plans, **knobs) == want, knobs


def _degrees(g):
    import numpy as np
    n, s, d = g
    u, v = np.minimum(s, d), np.maximum(s, d)
    keys = np.unique(u.astype(np.int64) * n + v)
    keys = keys[keys // n != keys % n]
    return np.bincount(np.concatenate([keys // n, keys % n]), minlength=n)


def test_autotune_choice_and_cache(pg, case, tmp_path):
    from paper_2004_02369_amd import tune
    g, want = case
    G = pg.load_graph(*g, device=0)
    plans = [pg.plan_pattern(s) for s in SPECS]
    path = str(tmp_path / "tune.json")
    say("autotune on chung_lu 3000/20000")
    res = tune.autotune(G, plans, reps=1, rounds=1, budget_s=30, cache_path=path)
    assert not res["cached"] and os.path.exists(path)
    assert res["ms"] <= res["default_ms"]
    assert pg.count(G, plans, **res["knobs"]) == want
    again = tune.autotune(G, plans, cache_path=path)
    assert again["cached"] and again["knobs"] == res["knobs"]
    # another plan set is another cache entry
    other = tune.autotune(G, plans[:2], reps=1, rounds=1, budget_s=10, cache_path=path)
    assert not other["cached"]
