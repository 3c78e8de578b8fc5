"""GPU tests of the asynchronous job entry points (pg_job_workspace_size,
pg_submit, pg_job_poll, pg_job_finish), the launch time limit and the
serving loop: every query gives the same answer alone and in a mix."""
import json
import os
import sys
import time

import pytest

from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import patterns as pt
from paper_2004_02369_amd import serve

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pg():
    import torch
    assert torch.cuda.is_available()
    from paper_2004_02369_amd import pg as _pg
    _pg.lib()
    return _pg


@pytest.fixture(scope="module")
def g_mid(pg):
    return pg.load_graph(*gg.workload("chunglu_20k_100k"), device=0)


def _workspace(nbytes):
    import torch
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    shift = (-raw.data_ptr()) % 256
    return raw[shift:shift + nbytes]


def test_jobs_match_synchronous_counts_three_streams(pg, g_mid):
    import torch
    say("three concurrent count jobs on chunglu_20k_100k")
    specs = pt.all_vertex_induced(4)
    plans = [pg.plan_pattern(s) for s in specs]
    want = pg.count(g_mid, plans)
    batches = [plans, plans[:2], [pg.plan_pattern(pt.clique(3)), pg.plan_pattern(pt.star(3))]]
    wants = [want, want[:2], pg.count(g_mid, batches[2])]
    grid = max(1, g_mid.resident_waves[0] // 3)
    streams = serve.slot_streams("cuda:0", len(batches))
    jobs = []
    for b, s in zip(batches, streams):
        nb = pg.job_workspace_size(g_mid, b, grid_waves=grid)
        jobs.append(pg.submit(g_mid, b, _workspace(nb), s, grid_waves=grid))
    t0 = time.perf_counter()
    while not all(j.done() for j in jobs):
        assert time.perf_counter() - t0 < 60
        time.sleep(1e-3)
    for j, w in zip(jobs, wants):
        got, st = j.finish()
        assert got == w
        assert st["grid_waves"] == grid and st["kernel_ms"] > 0
    with pytest.raises(pg.PGError):
        jobs[0].finish()


def test_exists_jobs(pg, g_mid):
    import torch
    s = serve.slot_streams("cuda:0", 1)[0]
    for k in (3, 4, 5, 6, 8, 10, 12, 14):
        say(f"exists job K{k}")
        p = pg.plan_pattern(pt.clique(k))
        nb = pg.job_workspace_size(g_mid, [p], pg.PG_JOB_EXISTS)
        j = pg.submit(g_mid, [p], _workspace(nb), s, mode=pg.PG_JOB_EXISTS)
        got, _ = j.finish()
        assert got == pg.exists(g_mid, p)
    # K_k with k above the largest clique: a full search that finds nothing
    G = pg.load_graph(*gg.complete(9), device=0)
    for k, want in ((9, True), (10, False)):
        p = pg.plan_pattern(pt.clique(k))
        nb = pg.job_workspace_size(G, [p], pg.PG_JOB_EXISTS)
        got, _ = pg.submit(G, [p], _workspace(nb), s, mode=pg.PG_JOB_EXISTS).finish()
        assert got is want


def test_job_argument_errors(pg, g_mid):
    import torch
    s = serve.slot_streams("cuda:0", 1)[0]
    p = pg.plan_pattern(pt.clique(4))
    nb = pg.job_workspace_size(g_mid, [p])
    ws = _workspace(nb + 512)
    with pytest.raises(pg.PGError) as e:
        pg.submit(g_mid, [p], ws[:nb - 1], s)
    assert e.value.status == pg.PG_ENOMEM
    with pytest.raises(pg.PGError) as e:
        pg.submit(g_mid, [p], ws[4:4 + nb], s)
    assert e.value.status == pg.PG_EINVAL
    with pytest.raises(pg.PGError) as e:
        pg.job_workspace_size(g_mid, [p, p], pg.PG_JOB_EXISTS)
    assert e.value.status == pg.PG_EINVAL
    with pytest.raises(pg.PGError):
        pg.job_workspace_size(g_mid, [p], mode=7)
    with pytest.raises(pg.PGError):
        pg.count_ex(g_mid, [p], time_limit_ms=-1)


def test_time_limit_stops_and_a_loose_limit_changes_nothing(pg):
    import torch
    with open(os.path.join(HERE, "golden", "expected.json")) as f:
        w = json.load(f)["workloads"]["chunglu_100k_1m"]
    from oracle import canonical_of_edges
    say("time limit on chunglu_100k_1m, 6 induced 4-motifs")
    G = pg.load_graph(*gg.workload("chunglu_100k_1m"), device=0)
    specs = pt.all_vertex_induced(4)
    plans = [pg.plan_pattern(s) for s in specs]
    want = [w["induced4"][str(canonical_of_edges(4, s["edges"]))]["count"] for s in specs]
    full, st_full = pg.count_ex(G, plans)
    assert full == want
    with pytest.raises(pg.PGError) as e:
        pg.count_ex(G, plans, time_limit_ms=5)
    assert e.value.status == pg.PG_ETIMEDOUT
    got, _ = pg.count_ex(G, plans, time_limit_ms=600000)
    assert got == want
    # the same through a job: partial run ends early and reports the limit
    s = serve.slot_streams("cuda:0", 1)[0]
    nb = pg.job_workspace_size(G, plans)
    j = pg.submit(G, plans, _workspace(nb), s, time_limit_ms=5)
    with pytest.raises(pg.PGError) as e:
        j.finish()
    assert e.value.status == pg.PG_ETIMEDOUT
    j = pg.submit(G, plans, _workspace(nb), s, time_limit_ms=600000)
    got, st = j.finish()
    assert got == want


def test_short_job_finishes_beside_a_long_one(pg):
    """A short launch on another slot stream completes, and is seen as done,
    while a long one still runs: the slots really overlap."""
    say("short job beside a long one on chunglu_100k_1m")
    G = pg.load_graph(*gg.workload("chunglu_100k_1m"), device=0)
    grid = max(1, G.resident_waves[0] // serve.default_slots())
    long_plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
    short_plans = [pg.plan_pattern(pt.clique(3))]
    s_long, s_short = serve.slot_streams("cuda:0", 2)
    w_long = _workspace(pg.job_workspace_size(G, long_plans, grid_waves=grid))
    w_short = _workspace(pg.job_workspace_size(G, short_plans, grid_waves=grid))
    want_short = pg.count(G, short_plans)
    import torch
    torch.cuda.synchronize()
    j_long = pg.submit(G, long_plans, w_long, s_long, grid_waves=grid)
    t0 = time.perf_counter()
    j_short = pg.submit(G, short_plans, w_short, s_short, grid_waves=grid)
    while not j_short.done():
        assert time.perf_counter() - t0 < 60
        time.sleep(1e-4)
    t_short = time.perf_counter() - t0
    got, _ = j_short.finish()
    t_fin = time.perf_counter() - t0
    long_running = not j_long.done()
    j_long.finish()
    say(f"short job seen done after {1e3 * t_short:.1f} ms, finished at {1e3 * t_fin:.1f} ms; long still running: "
        f"{long_running}")
    assert got == want_short
    assert long_running


def test_serving_alone_equals_in_mix(pg, g_mid):
    queries = serve.catalogue(pg, pt)
    say(f"serving mix: {len(queries)} catalogue entries on chunglu_20k_100k")
    # answers from the synchronous entry points
    sync = {}
    for q in queries:
        sync[q.name] = pg.exists(g_mid, q.plans[0]) if q.kind == "exists" else pg.count(g_mid, q.plans)
    def biggest(slots):
        probe = serve.Server(g_mid, 1 << 20, slots=slots)
        return max(probe.size_of(q.plans, q.kind) for q in queries)

    alone = serve.standalone(g_mid, queries, biggest(1), limit_ms=60000)
    for q in queries:
        res, _, err = alone[q.name]
        assert err is None, (q.name, err)
        assert res == sync[q.name], q.name
    # a pool of about two launches: admission has to wait for memory
    pool = 2 * biggest(3) + 4096
    srv = serve.Server(g_mid, pool, slots=3, time_limit_ms=120000,
                       policy=serve.policy_from(queries, alone, 3, light_ms=20.0))
    times, picks = serve.poisson_arrivals(3000.0, 300, len(queries), seed=11)
    reqs, t0 = serve.run_open_loop(srv, queries, times, picks)
    assert len(reqs) == 300 and srv.idle()
    for r in reqs:
        assert r.error is None, (r.query.name, r.error)
        assert r.result == alone[r.query.name][0], r.query.name
    assert srv.merged_requests > 0          # continuous batching happened
    assert any(srv.policy.heavy(r) for r in reqs) and not all(srv.policy.heavy(r) for r in reqs)
    assert srv.pool.used == 0 and sorted(srv.free_slots) == [0, 1, 2]
    # a launch runs on a slot's grid, or (heavy only) on the wide grid of
    # the slots it holds; at most one heavy launch at a time
    wide = [rec for rec in srv.log if rec["grid"] != srv.grid]
    assert all(rec["heavy"] and rec["grid"] == srv.grid * srv.heavy_width for rec in wide)
    summ = serve.summarize(reqs, t0)
    say(f"mix: p50 {summ['p50_ms']:.2f} ms, p99 {summ['p99_ms']:.2f} ms, "
        f"{summ['completed_qps']:.0f} QPS, {srv.launches} launches ({len(wide)} wide)")


def _iso_key(spec):
    """The typed pattern up to relabelling: the smallest (true edges,
    anti-edges) listing over all orders of the vertices (an induced spec's
    implied anti-edges included)."""
    import itertools
    k = spec["k"]
    E = {tuple(sorted(e)) for e in spec["edges"]}
    A = {tuple(sorted(e)) for e in spec.get("anti") or []}
    if spec.get("induced"):
        A |= {(a, b) for a, b in itertools.combinations(range(k), 2) if (a, b) not in E}
    assert not spec.get("av") and not spec.get("labels")
    if len(E) == k * (k - 1) // 2:  # a clique is its own canonical form
        return (k, tuple(sorted(E)), ())
    assert k <= 6
    best = None
    for p in itertools.permutations(range(k)):
        key = (tuple(sorted(tuple(sorted((p[a], p[b]))) for a, b in E)),
               tuple(sorted(tuple(sorted((p[a], p[b]))) for a, b in A)))
        if best is None or key < best:
            best = key
    return (k,) + best


def test_served_results_equal_oracle(pg, orc):
    """Every catalogue query, served alone and in a Poisson mix, gives the
    oracle's answer (counts by valid maps / |Aut_t|, closed forms and the
    existence search, written by tests/golden/make_golden.py)."""
    with open(os.path.join(HERE, "golden", "expected.json")) as f:
        w = json.load(f)["workloads"]["serve_cl5k"]
    gold = {_iso_key(a["spec"]): a["answer"] for a in w["answers"]}
    prm = w["params"]
    say("served results vs oracle on chung_lu 5000/25000")
    G = pg.load_graph(*gg.chung_lu(prm["n"], prm["m"], prm["gamma"], prm["w_max"], seed=prm["seed"]), device=0)
    assert G.m == w["m"]
    queries = serve.catalogue(pg, pt)
    want = {}
    for q in queries:
        assert len(q.specs) == 1
        key = _iso_key(q.specs[0])
        assert key in gold, f"no oracle answer for {q.name}"
        want[q.name] = gold[key] if q.kind == "exists" else [gold[key]]
    assert any(v is True for v in want.values()) and any(v is False for v in want.values())
    def biggest(slots):
        probe = serve.Server(G, 1 << 20, slots=slots)
        return max(probe.size_of(q.plans, q.kind) for q in queries)

    alone = serve.standalone(G, queries, biggest(1), limit_ms=60000)
    for q in queries:
        res, _, err = alone[q.name]
        assert err is None, (q.name, err)
        assert res == want[q.name], (q.name, res, want[q.name])
    for window_ms in (0.0, 0.5):
        # window_ms > 0: heavy launches run as root-task windows, light
        # requests start between them
        say(f"served mix, window_ms {window_ms}")
        srv = serve.Server(G, 2 * biggest(3) + 4096, slots=3, time_limit_ms=120000,
                           policy=serve.policy_from(queries, alone, 3, light_ms=2.0), window_ms=window_ms)
        times, picks = serve.poisson_arrivals(2000.0, 400, len(queries), seed=12)
        reqs, t0 = serve.run_open_loop(srv, queries, times, picks)
        assert len(reqs) == 400 and srv.idle()
        for r in reqs:
            assert r.error is None, (r.query.name, r.error)
            assert r.result == want[r.query.name], r.query.name
        assert srv.merged_requests > 0
        assert (srv.windows_run > 0) == (window_ms > 0)
        assert srv.pool.used == 0 and sorted(srv.free_slots) == [0, 1, 2]
