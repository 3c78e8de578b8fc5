"""Measurements beyond the headline benchmark, each printing JSON lines.

    python -m paper_2004_02369_amd.measure enum      # enumeration into HBM: rows/s, GB/s
    python -m paper_2004_02369_amd.measure motifs5 --workload rmat12_64k
                                                     # 21 induced 5-motifs + K5, batched vs one launch each
    python -m paper_2004_02369_amd.measure small     # launch-bound case: ER 2k/20k, batched vs singles
    python -m paper_2004_02369_amd.measure inversion # induced census via non-induced counts + inversion
    python -m paper_2004_02369_amd.measure c1        # triangle, wedge, K4 on ER 2k/20k, one pattern per launch
    python -m paper_2004_02369_amd.measure c3        # 21 induced 5-motifs + K5 on R-MAT scale 20 (16M edges):
                                                     # each alone under a time limit, the finishing ones batched
    python -m paper_2004_02369_amd.measure c5        # the serving catalogue's count queries on R-MAT scale 22
                                                     # (64M edges): each alone (time, merge-model bytes), then batched
    python -m paper_2004_02369_amd.measure rows      # achievable HBM read bandwidth, and row-pair intersections
                                                     # on the R-MAT scale 22 rows by variant and row length
    python -m paper_2004_02369_amd.measure hubs      # the benchmark batch on R-MAT scale 22 with more or fewer
                                                     # rows held as bitmaps (hub bitmap budget sweep)
    python -m paper_2004_02369_amd.measure tune      # tune the benchmark batch's launch knobs, store the record
    python -m paper_2004_02369_amd.measure balance   # first / last wavefront finish times (load imbalance)
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _say(*a):
    print("[measure]", *a, file=sys.stderr, flush=True)


def enum(args, pg, gg, pt):
    """Matches written to a device buffer (k int32 ids per row) by one
    pg_enumerate launch; the buffer is sized from a first counting pass."""
    G = pg.load_graph(*gg.workload(args.workload), device=0)
    for spec in (pt.clique(3), pt.clique(4), pt.chain(3)):
        plan = pg.plan_pattern(spec)
        rows, total = pg.enumerate_matches(G, plan)  # warm-up, sizes the buffer
        import torch
        buf = torch.empty((max(1, total), plan.k), dtype=torch.int32, device="cuda:0")
        import ctypes
        tot = ctypes.c_uint64()
        best = float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pg._check(pg.lib().pg_enumerate(G._h, plan._h, ctypes.c_void_p(buf.data_ptr()), total,
                                            ctypes.byref(tot), None))
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        assert tot.value == total
        print(json.dumps({"measure": "enumerate", "workload": args.workload, "pattern": spec["edges"],
                          "rows": total, "seconds": best, "rows_per_s": total / best,
                          "output_gb_per_s": total * plan.k * 4 / best / 1e9}), flush=True)


def motifs5(args, pg, gg, pt):
    """The 22-plan batch (21 induced 5-motifs + K5) in one launch, then each
    plan in a launch of its own."""
    G = pg.load_graph(*gg.workload(args.workload), device=0)
    specs = pt.all_vertex_induced(5) + [pt.clique(5)]
    plans = [pg.plan_pattern(s) for s in specs]
    knobs = {"chunk": args.chunk} if args.chunk else {}
    t0 = time.perf_counter()
    counts, st = pg.count_ex(G, plans, time_limit_ms=args.limit_ms, **knobs)
    batched = time.perf_counter() - t0
    _say(f"batched {batched:.2f} s")
    single = []
    for p in plans:
        t0 = time.perf_counter()
        pg.count_ex(G, [p], time_limit_ms=args.limit_ms, **knobs)
        single.append(time.perf_counter() - t0)
    print(json.dumps({"measure": "motifs5", "workload": args.workload, "n": G.n, "m": G.m, "d_max": G.d_max,
                      "knobs": knobs,
                      "batched_s": batched, "kernel_ms": st["kernel_ms"], "single_s": single,
                      "single_sum_s": sum(single), "speedup": sum(single) / batched,
                      "k5_equals_induced_k5": counts[-1] == counts[-2], "counts": counts}), flush=True)


def inversion(args, pg, gg, pt):
    """Induced motif census by the inversion route (edge-induced counts in
    one launch, then exact inversion on the host) against the direct
    pattern-aware route."""
    from . import motifs
    for wl, k in ((args.workload or "chunglu_100k_1m", 4), ("rmat12_64k", 5)):
        G = pg.load_graph(*gg.workload(wl), device=0)
        direct_plans = [pg.plan_pattern({"k": k, "edges": list(s), "induced": True}) for s in motifs.shapes(k)]
        t0 = time.perf_counter()
        direct = pg.count(G, direct_plans, time_limit_ms=args.limit_ms)
        t_direct = time.perf_counter() - t0
        best = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            inv = motifs.induced_counts(G, k, pg)
            best = min(best, time.perf_counter() - t0)
        print(json.dumps({"measure": "inversion", "workload": wl, "k": k, "direct_s": t_direct,
                          "inversion_s": best, "speedup": t_direct / best, "equal": inv == direct}), flush=True)


def c1(args, pg, gg, pt):
    """Triangle, wedge and 4-clique counts on ER 2k/20k, one pattern per
    launch: kernel time (best of several launches), host-side latency of
    the synchronous call, and matches/s."""
    G = pg.load_graph(*gg.workload("er_2k_20k"), device=0)
    import torch
    s = torch.cuda.current_stream(0)
    for name, spec in (("triangle", pt.clique(3)), ("wedge", pt.star(3)), ("K4", pt.clique(4))):
        plan = pg.plan_pattern(spec)
        best_k, best_t, count = float("inf"), float("inf"), None
        for _ in range(30):
            t0 = time.perf_counter()
            c, st = pg.count_ex(G, [plan], stream=s)
            best_t = min(best_t, time.perf_counter() - t0)
            best_k = min(best_k, st["kernel_ms"])
            count = c[0]
        print(json.dumps({"measure": "c1", "workload": "er_2k_20k", "pattern": name, "count": count,
                          "kernel_ms": best_k, "call_ms": best_t * 1e3,
                          "matches_per_s": count / (best_k / 1e3)}), flush=True)


def c3(args, pg, gg, pt):
    """The 22-plan family (21 induced 5-motifs + K5) at full size: each plan
    alone under a device time limit: the exact count when it finishes, else
    the share of root tasks reached, a linear projection of the full time
    and the partial count.  Then the finishing plans batched against their
    single launches, and the tuner on them.  K5 must equal the induced K5."""
    from . import tune
    t0 = time.perf_counter()
    G = pg.load_graph(*gg.workload(args.workload), device=0)
    _say(f"{args.workload}: n={G.n} m={G.m} d_max={G.d_max} ready in {time.perf_counter() - t0:.1f} s")
    specs = pt.all_vertex_induced(5) + [pt.clique(5)]
    plans = [pg.plan_pattern(s) for s in specs]
    lo_plan, hi_plan = (int(x) for x in args.plans.split("-"))
    knobs = {"chunk": args.chunk} if args.chunk else {}
    singles = []
    for i, p in enumerate(plans):
        rec = {"plan": i, "edges": specs[i]["edges"], "core": p.info()["core"], "ms": None, "count": None}
        if not (lo_plan <= i <= hi_plan):
            continue
        try:
            c, st = pg.count_ex(G, [p], time_limit_ms=args.limit_ms, **knobs)
            rec.update(ms=st["kernel_ms"], count=c[0], root_tasks=st["root_tasks"])
        except pg.PGError as e:
            if e.status != pg.PG_ETIMEDOUT:
                raise
            # stopped at the limit: the share of root tasks reached, a linear
            # projection of the full time from it (tasks come roughly
            # costliest first by d(u) + d(v), but a plan's cost per task need
            # not follow that order, so this is an estimate, not a bound), and
            # the partial count (a lower bound)
            st = e.stats
            frac = st["tasks_started"] / max(1, st["root_tasks"])
            rec.update(stopped="ETIMEDOUT", kernel_ms_at_stop=st["kernel_ms"], root_tasks=st["root_tasks"],
                       tasks_started=st["tasks_started"], fraction_started=frac,
                       projected_ms=st["kernel_ms"] / frac if frac > 0 else None, count_lower_bound=e.counts[0])
        singles.append(rec)
        _say(f"plan {i} {specs[i]['edges']}: " + json.dumps({k: v for k, v in rec.items() if k not in ("edges",)}))
    singles = [r for r in singles if "root_tasks" in r]
    done = [r for r in singles if r["ms"] is not None]
    batch = [plans[r["plan"]] for r in done]
    out = {"measure": "c3", "workload": args.workload, "n": G.n, "m": G.m, "d_max": G.d_max,
           "limit_ms": args.limit_ms, "knobs": knobs, "singles": singles, "finished": len(done)}
    if done:
        c, st = pg.count_ex(G, batch, **knobs)
        assert c == [r["count"] for r in done], "batched counts differ from the single launches"
        out["batched_ms"] = st["kernel_ms"]
        out["singles_sum_ms"] = sum(r["ms"] for r in done)
        out["batched_speedup"] = out["singles_sum_ms"] / st["kernel_ms"]
        _say(f"batch of {len(done)}: {st['kernel_ms']:.1f} ms vs {out['singles_sum_ms']:.1f} ms one launch each")
        if args.tune_budget > 0:
            tuned = tune.autotune(G, batch, budget_s=args.tune_budget, log=_say)
            out["tuned"] = {"knobs": tuned["knobs"], "ms": tuned["ms"], "default_ms": tuned["default_ms"],
                            "trials": len(tuned["trials"])}
    byplan = {r["plan"]: r for r in singles}
    k5, ik5 = byplan.get(len(specs) - 1), byplan.get(len(specs) - 2)
    if k5 and ik5 and k5["count"] is not None and ik5["count"] is not None:
        assert k5["count"] == ik5["count"], "K5 differs from the induced K5"
        out["k5_equals_induced_k5"] = True
    print(json.dumps(out), flush=True)


def c5(args, pg, gg, pt):
    """Every count query of the serving catalogue on the serving graph, alone
    under a device time limit: kernel time, count and merge-model bytes
    (a separate counting run); then the finishing ones in one launch."""
    from . import serve
    t0 = time.perf_counter()
    G = pg.load_graph(*gg.workload(args.workload), device=0)
    _say(f"{args.workload}: n={G.n} m={G.m} d_max={G.d_max} ready in {time.perf_counter() - t0:.1f} s")
    seen, rows = {}, []
    for name, kind, specs in serve.catalogue_specs(pt):
        if kind != "count":
            continue
        key = serve.pattern_key(specs[0])
        if key in seen:
            continue
        plan = pg.plan_pattern(specs[0])
        seen[key] = plan
        rec = {"name": name, "edges": specs[0]["edges"], "induced": bool(specs[0].get("induced")),
               "anti": specs[0].get("anti")}
        try:
            c, st = pg.count_ex(G, [plan], time_limit_ms=args.limit_ms)
            rec.update(ms=st["kernel_ms"], count=c[0], grid=st["grid_waves"])
            c2, st2 = pg.count_ex(G, [plan], flags=pg.PG_RUN_COUNT_BYTES, time_limit_ms=4 * args.limit_ms)
            assert c2 == c
            rec["logical_bytes"] = st2["logical_bytes"]
        except pg.PGError as e:
            if e.status not in (pg.PG_ETIMEDOUT, pg.PG_EOVERFLOW):
                raise
            rec.update(ms=None, count=None, error=pg._STATUS.get(e.status))
        rec["plan"] = plan
        rows.append(rec)
        _say(f"{name}: {rec.get('ms')} ms, count {rec.get('count')}, bytes {rec.get('logical_bytes')}")
    done = [r for r in rows if r["ms"] is not None]
    out = {"measure": "c5", "workload": args.workload, "n": G.n, "m": G.m, "d_max": G.d_max,
           "limit_ms": args.limit_ms, "queries": [{k: v for k, v in r.items() if k != "plan"} for r in rows]}
    if done:
        c, st = pg.count_ex(G, [r["plan"] for r in done])
        assert c == [r["count"] for r in done], "batched counts differ from the single launches"
        out["batched_ms"] = st["kernel_ms"]
        out["singles_sum_ms"] = sum(r["ms"] for r in done)
        out["batched_speedup"] = out["singles_sum_ms"] / st["kernel_ms"]
    print(json.dumps(out), flush=True)


def rows(args, pg, gg, pt):
    """Achievable HBM read bandwidth (a 4 GiB streaming read), then
    |N(u) & N(v)| over row pairs of random edges of the serving graph, by
    intersection variant and by length bucket, with the caches flushed
    before every launch.  Work per pair is the merge model's 4 (|A| + |B|)
    bytes; all variants must return the same counts."""
    import numpy as np
    import torch
    from . import rowbench as rb
    dev = torch.device("cuda:0")
    buf = torch.ones(1 << 30, dtype=torch.int32, device=dev)  # 4 GiB
    ms, _ = rb.stream_read(buf, reps=5)
    peak = 4.0 * buf.numel() / (ms * 1e-3) / 1e9
    out = {"measure": "rows", "workload": args.workload, "stream_read_gb_per_s": peak,
           "stream_read_bytes": 4 * buf.numel()}
    _say(f"streaming read: {peak:.0f} GB/s")
    flush_buf = buf[: 1 << 28]  # 1 GiB, larger than L2 and the last-level cache
    G = pg.load_graph(*gg.workload(args.workload), device=0)
    rp_h, col_h = G.csr()
    rp = torch.from_numpy(rp_h).to(dev)
    col = torch.from_numpy(col_h).to(dev)
    rng = np.random.Generator(np.random.PCG64(args.seed))
    slots = rng.integers(0, len(col_h), args.pairs)
    u = (np.searchsorted(rp_h, slots, side="right") - 1).astype(np.int32)
    v = col_h[slots].astype(np.int32)
    deg = np.diff(rp_h)
    size = deg[u] + deg[v]
    edges = [0, 64, 512, 4096, 32768, 1 << 40]
    out["buckets"] = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = np.nonzero((size >= lo) & (size < hi))[0]
        if len(sel) == 0:
            continue
        pu = torch.from_numpy(u[sel]).to(dev)
        pv = torch.from_numpy(v[sel]).to(dev)
        nbytes = 4 * int(size[sel].sum())
        rec = {"len_lo": lo, "len_hi": hi if hi < (1 << 40) else None, "pairs": len(sel), "merge_bytes": nbytes}
        ref = None
        for name, var in rb.VARIANTS.items():
            o = torch.zeros(len(sel), dtype=torch.int32, device=dev)
            best = float("inf")
            for _ in range(3):
                rb.flush(flush_buf)
                best = min(best, rb.intersect(var, rp, col, pu, pv, o))
            got = o.cpu().numpy()
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), f"variant {name} differs"
            rec[name] = {"ms": best, "gb_per_s": nbytes / (best * 1e-3) / 1e9,
                         "frac_of_stream": nbytes / (best * 1e-3) / 1e9 / peak}
        _say(f"[{lo}, {hi}): {len(sel)} pairs " + ", ".join(f"{k} {rec[k]['gb_per_s']:.0f} GB/s" for k in rb.VARIANTS))
        out["buckets"].append(rec)
    print(json.dumps(out), flush=True)


def hubs(args, pg, gg, pt):
    """The benchmark's batch (serving count queries) on the serving graph
    loaded with several hub-bitmap budgets: rows held as bitmaps, HBM held,
    batch and per-pattern kernel time.  Counts must not change."""
    from . import serve
    edges = gg.workload(args.workload)
    names = ["triangle", "wedge", "induced_wedge", "clique4", "book3", "cricket"]
    ref = None
    for mib in [int(x) for x in args.budgets.split(",")]:
        t = time.perf_counter()
        G = pg.load_graph(*edges, device=0, hub_budget_mib=mib)
        load_s = time.perf_counter() - t
        q = {x.name: x for x in serve.catalogue(pg, pt)}
        plans = [q[n].plans[0] for n in names]
        c, _ = pg.count_ex(G, plans)
        ms = min(pg.count_ex(G, plans)[1]["kernel_ms"] for _ in range(2))
        if ref is None:
            ref = c
        assert c == ref, "counts changed with the bitmap budget"
        single = {n: pg.count_ex(G, [p])[1]["kernel_ms"] for n, p in zip(names, plans)}
        rec = {"measure": "hubs", "workload": args.workload, "budget_mib": mib, "hub_rows": G.hub_count,
               "hub_min_degree": G.hub_min_degree, "device_bytes": G.device_bytes, "load_s": load_s,
               "batch_kernel_ms": ms, "single_kernel_ms": single}
        _say(json.dumps(rec))
        print(json.dumps(rec), flush=True)
        del G


def tune_batch(args, pg, gg, pt):
    """Tune the launch knobs of the serving batch on the serving graph, of
    K5 and the induced K5 (the 5-vertex plans that finish) on R-MAT scale
    20, or of the six induced 4-motifs on another workload, and store the
    record in the package's tuning records (tuned.json)."""
    from . import serve, tune
    G = pg.load_graph(*gg.workload(args.workload), device=0)
    if args.workload == "rmat22_64m":
        q = {x.name: x for x in serve.catalogue(pg, pt)}
        plans = [q[n].plans[0] for n in serve.SERVING_BATCH]
    elif args.workload == "rmat20_16m":
        plans = [pg.plan_pattern(pt.all_vertex_induced(5)[-1]), pg.plan_pattern(pt.clique(5))]
    else:
        plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
    res = tune.autotune(G, plans, budget_s=args.tune_budget, cache_path=tune.RECORDS, force=True, log=_say)
    print(json.dumps({"measure": "tune", "workload": args.workload, "knobs": res["knobs"], "ms": res["ms"],
                      "default_ms": res["default_ms"], "trials": len(res["trials"])}), flush=True)


def balance(args, pg, gg, pt):
    """Load balance of the persistent grid: when the first and the last
    wavefront ran out of root tasks (device clock, PG_RUN_WAVE_TIMES), for
    the six induced 4-motifs on Chung-Lu 100K / 1M and the serving batch on
    R-MAT scale 22, with the knobs the benchmark uses."""
    from . import serve, tune
    for wl in ("chunglu_100k_1m", "rmat22_64m"):
        G = pg.load_graph(*gg.workload(wl), device=0)
        if wl == "rmat22_64m":
            q = {x.name: x for x in serve.catalogue(pg, pt)}
            plans = [q[n].plans[0] for n in serve.SERVING_BATCH]
        else:
            plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
        rec = tune.lookup(G, plans, tune.RECORDS)
        knobs = {k: v for k, v in (rec["knobs"] if rec else {}).items() if v}
        knobs["flags"] = knobs.get("flags", 0) | pg.PG_RUN_WAVE_TIMES
        pg.count_ex(G, plans, **knobs)
        runs = []
        for _ in range(3):
            _, st = pg.count_ex(G, plans, **knobs)
            runs.append({"kernel_ms": st["kernel_ms"], "first_done_ms": st["wave_done_first_ms"],
                         "last_done_ms": st["wave_done_last_ms"],
                         "spread_ms": st["wave_done_last_ms"] - st["wave_done_first_ms"]})
        print(json.dumps({"measure": "balance", "workload": wl, "grid_waves": st["grid_waves"], "knobs": knobs,
                          "runs": runs}), flush=True)
        del G


def small(args, pg, gg, pt):
    """Launch-bound regime: the six induced 4-motifs on ER 2k/20k, one
    batched launch against six launches, best of several repetitions."""
    G = pg.load_graph(*gg.workload("er_2k_20k"), device=0)
    plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
    import torch
    s = torch.cuda.current_stream(0)

    def best_of(fn, reps=20):
        b = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            b = min(b, time.perf_counter() - t0)
        return b
    batched = best_of(lambda: pg.count(G, plans, stream=s))
    singles = best_of(lambda: [pg.count(G, [p], stream=s) for p in plans])
    print(json.dumps({"measure": "small_batch", "workload": "er_2k_20k", "batched_ms": batched * 1e3,
                      "singles_ms": singles * 1e3, "speedup": singles / batched}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["enum", "motifs5", "small", "inversion", "c1", "c3", "c5", "rows", "hubs", "tune", "balance"])
    ap.add_argument("--pairs", type=int, default=2_000_000)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--budgets", default="1024,4096,16384,32768")
    ap.add_argument("--plans", default="0-21", help="c3: the plans to run (a-b, of the 22)")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--limit-ms", type=int, default=600000)
    ap.add_argument("--tune-budget", type=float, default=60.0)
    ap.add_argument("--chunk", type=int, default=0, help="motifs5, c3: largest claim of root tasks (0 = library default)")
    args = ap.parse_args(argv)
    import torch
    from . import graphgen as gg
    from . import patterns as pt
    from . import pg
    assert torch.cuda.is_available(), "measurements need a GPU"
    if args.what == "enum":
        args.workload = args.workload or "chunglu_100k_1m"
        enum(args, pg, gg, pt)
    elif args.what == "motifs5":
        args.workload = args.workload or "rmat12_64k"
        motifs5(args, pg, gg, pt)
    elif args.what == "inversion":
        inversion(args, pg, gg, pt)
    elif args.what == "c1":
        c1(args, pg, gg, pt)
    elif args.what == "c3":
        args.workload = args.workload or "rmat20_16m"
        c3(args, pg, gg, pt)
    elif args.what == "balance":
        balance(args, pg, gg, pt)
    elif args.what == "tune":
        args.workload = args.workload or "rmat22_64m"
        tune_batch(args, pg, gg, pt)
    elif args.what == "hubs":
        args.workload = args.workload or "rmat22_64m"
        hubs(args, pg, gg, pt)
    elif args.what == "rows":
        args.workload = args.workload or "rmat22_64m"
        rows(args, pg, gg, pt)
    elif args.what == "c5":
        args.workload = args.workload or "rmat22_64m"
        c5(args, pg, gg, pt)
    else:
        small(args, pg, gg, pt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
