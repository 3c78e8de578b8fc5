"""Autotuner of the launch knobs for one resident graph and one plan set.

The knobs (pg_run_config):

* ``hub_min_degree`` -- the intersection variant per degree bucket: rows
  of at least this degree are probed through their dense bitmap (one
  load), shorter rows by binary search over the sorted row;
* ``chunk`` -- the largest claim of root tasks; the guided claim grows from 1
  at the costliest tasks to this at the cheapest, so it sets the chunk per
  cost (degree) bucket;
* ``batch_max_avg`` -- a level whose children only count is expanded for up
  to 64 parents in one flattened pass while the parents average at most this
  many candidates, parent by parent otherwise (decided per batch);
* ``flags`` -- PG_RUN_NO_TASK_BATCH turns the flattened pass off everywhere;
  PG_RUN_LIGHT_KERNEL runs a long count launch on the four-wave build of the
  kernel instead of the five-wave one.

The search is coordinate descent over measured kernel times (best of a few
launches), each trial under a device time limit of a few times the best so
far, so bad settings cost little.  Every trial must return the same counts.
Results are cached per graph fingerprint and plan set.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

SPACE = {
    "hub_min_degree": [0, 32, 64, 128, 256, 1024, -1],
    "chunk": [4, 8, 16, 32, 64, 128, 256, 512, 1024],
    "batch_max_avg": [0, 8, 16, 32, 64, 128, 512, 2048],
    "flags": [0, 4, 8],  # 4 = PG_RUN_NO_TASK_BATCH, 8 = PG_RUN_LIGHT_KERNEL
}
DEFAULT = {"hub_min_degree": 0, "chunk": 0, "batch_max_avg": 0, "flags": 0}


class InconsistentCounts(RuntimeError):
    pass


def search(measure, space=None, start=None, rounds: int = 2, budget_s: float = 60.0, log=None):
    """Coordinate descent.  measure(knobs, limit_ms) -> (counts, ms), with
    ms = inf when the trial hit its limit.  Returns (best knobs, best ms,
    trials [(knobs, ms)])."""
    space = space or SPACE
    cur = dict(start or DEFAULT)
    t0 = time.perf_counter()
    # the starting point: once without a limit (its time sets the trials'
    # limits), then twice under a limit like every trial's, best of those
    # two: a launch that watches a time limit checks the device clock as it
    # goes, which costs a few percent, so only limited runs compare fairly
    ref, first = measure(cur, 0)
    if not math.isfinite(first):
        raise RuntimeError("the starting configuration did not finish")
    best = math.inf
    for _ in range(2):
        c, ms = measure(cur, max(20, int(3 * first)))
        if math.isfinite(ms) and c != ref:
            raise InconsistentCounts(f"{cur} gave {c}, expected {ref}")
        best = min(best, ms)
    if not math.isfinite(best):
        best = first
    trials = [(dict(cur), best)]
    seen = {json.dumps(cur, sort_keys=True)}
    for _ in range(rounds):
        improved = False
        for knob, values in space.items():
            for v in values:
                cand = dict(cur, **{knob: v})
                key = json.dumps(cand, sort_keys=True)
                if key in seen:
                    continue
                if time.perf_counter() - t0 > budget_s:
                    return cur, best, trials
                seen.add(key)
                counts, ms = measure(cand, max(20, int(3 * best)))
                trials.append((cand, ms))
                if log:
                    log(f"{cand} -> {ms:.2f} ms")
                if math.isfinite(ms):
                    if counts != ref:
                        raise InconsistentCounts(f"{cand} gave {counts}, expected {ref}")
                    if ms < best:
                        best, cur, improved = ms, cand, True
        if not improved:
            break
    return cur, best, trials


def fingerprint(G) -> str:
    import numpy as np
    from . import pg
    rp = np.zeros(G.n + 1, dtype=np.int64)
    pg._check(pg.lib().pg_graph_csr(G._h, rp.ctypes.data, None))
    h = hashlib.sha256()
    h.update(np.array([G.n, G.m, G.d_max, G.hub_count], dtype=np.int64).tobytes())
    h.update(rp.tobytes())
    return h.hexdigest()[:24]


def plan_key(plans) -> str:
    items = [p.spec if p.anchor is None else [p.spec, p.anchor] for p in plans]
    return hashlib.sha256(json.dumps(items, sort_keys=True, default=list).encode()).hexdigest()[:24]


# tuning records shipped with the package (written by autotune(cache_path=...))
RECORDS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def lookup(G, plans, path: str):
    """The cached result for this graph and plan set in `path`, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cache = json.load(f)
    res = cache.get(f"{fingerprint(G)}:{plan_key(plans)}")
    return None if res is None else dict(res, cached=True)


def default_cache_path() -> str:
    return os.environ.get("PG_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2004_02369_amd", "tune.json"))


def autotune(G, plans, reps: int = 2, rounds: int = 2, budget_s: float = 60.0, cache_path: str | None = None,
             log=None, force: bool = False):
    """Tune the launch knobs of `plans` on graph G.  Returns a dict with the
    best knobs, their time, the default's time and every trial.  With
    cache_path, a cached result for the same graph and plans is returned
    without measuring (unless force), and a new one is stored."""
    from . import pg
    plans = list(plans)
    key = f"{fingerprint(G)}:{plan_key(plans)}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache and not force:
            return dict(cache[key], cached=True)

    def measure(knobs, limit_ms):
        best, counts = math.inf, None
        for _ in range(reps):
            try:
                c, st = pg.count_ex(G, plans, time_limit_ms=limit_ms, **knobs)
            except pg.PGError as e:
                if e.status == pg.PG_ETIMEDOUT:
                    return None, math.inf
                raise
            counts, best = c, min(best, st["kernel_ms"])
        return counts, best

    knobs, ms, trials = search(measure, rounds=rounds, budget_s=budget_s, log=log)
    default_ms = trials[0][1]
    res = {"knobs": knobs, "ms": ms, "default_ms": default_ms,
           "trials": [[k, t if math.isfinite(t) else None] for k, t in trials],
           "graph": {"n": G.n, "m": G.m, "d_max": G.d_max, "hub_count": G.hub_count}}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
        cache[key] = res
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return dict(res, cached=False)
