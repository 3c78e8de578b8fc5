"""Benchmark: exact counts of the six connected vertex-induced 4-vertex
motifs in one batched launch on a Chung-Lu power-law graph (n = 100,000,
1,000,000 unique undirected edges, exponent 2.1, max weight 5,000), graph
resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one pg_count call over the batch (plan compile cached, launch,
device reduction, counts back to the host), with the launch knobs the
autotuner picks for this graph and plan set before the timed region.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "chunglu_100k_1m"
HBM_PEAK_GBPS = 8000.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("engine.hip", "engine.hpp", "pg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2004_02369_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"match_kernel_{WORKLOAD}_traffic.txt")
    t = {}
    try:
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", " ", "-")):
                    k, v = line.split(":", 1)
                    t[k.strip()] = v.strip()
    except OSError:
        return None
    if t.get("kernel_hash") != kernel_hash:
        return None
    try:
        return float(t["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(g, specs, budget_s=10.0):
    """The oracle's generic matcher on a bounded sample of start vertices of
    the same graph: matches/s = (valid maps / |Aut|) / time, over the six
    induced motifs.  Start vertices are taken in a seeded random order, one
    at a time, until the time budget is spent."""
    import numpy as np
    import oracle
    og = oracle.Graph.from_tuple(g)
    threads = oracle.default_threads()
    rng = np.random.Generator(np.random.PCG64(99))
    n = og.n
    sample = rng.permutation(n).astype(np.int32)
    spent, matches, used = 0.0, 0.0, 0
    while spent < budget_s and used < n:
        roots = sample[used:used + 1]
        t0 = time.perf_counter()
        for s in specs:
            matches += oracle.valid_maps_from(og, s, roots, threads) / oracle.aut(s)
        spent += time.perf_counter() - t0
        used += len(roots)
    return {"value": matches / spent, "unit": "matches/s", "cores": threads, "kind": "oracle",
            "sample": f"generic matcher over {used} of {n} random start vertices (pattern vertex 0), "
                      f"6 induced 4-motifs, {spent:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-pattern", action="store_true", help="skip the one-launch-per-pattern comparison")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for HBM counters) and exit")
    ap.add_argument("--knobs", default=None, metavar="JSON",
                    help="launch knobs to time (skips the autotuner), e.g. '{\"chunk\": 16}'")
    ap.add_argument("--no-tune", action="store_true", help="time the library defaults")
    ap.add_argument("--tune-budget", type=float, default=40.0, help="autotuner time budget, s")
    ap.add_argument("--retune", action="store_true", help="ignore the committed tuning record")
    ap.add_argument("--tune-out", default="", help="write the tuning result to this cache file")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by root tasks with one final all-reduce; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}))
        return
    from paper_2004_02369_amd import graphgen as gg
    from paper_2004_02369_amd import patterns as pt
    from paper_2004_02369_amd import pg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    w = gg.WORKLOADS[WORKLOAD]
    g = gg.workload(WORKLOAD)
    G = pg.load_graph(*g, device=0)
    specs = pt.all_vertex_induced(4)
    plans = [pg.plan_pattern(s) for s in specs]
    plan_ms = sum(p.info()["plan_ms"] for p in plans)

    # launch knobs: the autotuner's choice for this graph and plan set
    # (untimed), unless given or disabled
    tuning = None
    if args.knobs:
        knobs = json.loads(args.knobs)
    elif args.no_tune:
        knobs = {}
    else:
        # the tuning record committed with the package for this graph and
        # plan set, if its fingerprint matches; else tune now
        from paper_2004_02369_amd import tune
        t_tune = time.perf_counter()
        res = None if args.retune else tune.lookup(G, plans, tune.RECORDS)
        if res is None:
            res = tune.autotune(G, plans, budget_s=args.tune_budget,
                                cache_path=args.tune_out or None, force=args.retune)
        knobs = res["knobs"]
        tuning = {"record": bool(res.get("cached")), "default_kernel_ms": res["default_ms"],
                  "tuned_kernel_ms": res["ms"], "trials": len(res["trials"]),
                  "tune_s": time.perf_counter() - t_tune}
    knobs = {k: v for k, v in knobs.items() if v}

    # merge-model bytes of one launch (counted in a separate, untimed run)
    flags = knobs.get("flags", 0)
    counts_b, st_b = pg.count_ex(G, plans, stream=stream, **dict(knobs, flags=flags | pg.PG_RUN_COUNT_BYTES))
    logical_bytes = st_b["logical_bytes"]

    for _ in range(args.warmup):
        pg.count_ex(G, plans, stream=stream, **knobs)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts, st = pg.count_ex(G, plans, stream=stream, **knobs)
        kernel_ms.append(st["kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert counts == counts_b, "counts differ between runs"
    total = sum(counts)
    ms_per_step = 1e3 * elapsed / args.steps
    avg_kernel_ms = statistics.mean(kernel_ms)

    # batched vs one launch per pattern (same plans, same graph)
    # (each pattern alone, with the better of the default knobs and the batch's)
    single_ms = []
    if not args.no_per_pattern:
        for p in plans:
            best = float("inf")
            for kn in ({}, knobs):
                pg.count_ex(G, [p], stream=stream, **kn)
                t1 = time.perf_counter()
                pg.count_ex(G, [p], stream=stream, **kn)
                best = min(best, 1e3 * (time.perf_counter() - t1))
            single_ms.append(best)

    # context: the same census by the inversion route (not the paper's
    # method; the headline value above is the pattern-aware route)
    from paper_2004_02369_amd import motifs
    inv_ms = float("inf")
    inv_counts = None
    if not args.no_per_pattern:
        for _ in range(2):
            t1 = time.perf_counter()
            inv = motifs.induced_counts(G, 4, pg, stream=stream)
            inv_ms = min(inv_ms, 1e3 * (time.perf_counter() - t1))
        order = [motifs.shapes(4).index(motifs._canon(4, s["edges"])) for s in specs]
        inv_counts = [inv[i] for i in order]

    khash = kernel_source_hash()
    traffic = measured_traffic(khash)
    achieved = logical_bytes / (avg_kernel_ms * 1e-3) / 1e9
    out = {
        "metric": "pattern matches/sec (6 vertex-induced 4-motifs, batched)",
        "value": total / (ms_per_step * 1e-3),
        "unit": "matches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32 ids, u64 counts",
        "data": "synthetic",
        "config": {"workload": f"Chung-Lu n={w['n']}, m={G.m} unique edges, gamma={w['gamma']}, "
                               f"w_max={w['w_max']}, seed={w['seed']}; 6 induced 4-motifs in one launch",
                   "n": G.n, "m": G.m, "d_max": G.d_max, "patterns": 6, "parallelism": "1 GPU"},
        "knobs": knobs,
        "tuning": tuning,
        "counts": counts,
        "kernel_ms": avg_kernel_ms,
        "plan_ms": plan_ms,
        "per_pattern_ms": single_ms or None,
        "per_pattern_ms_sum": sum(single_ms) if single_ms else None,
        "batched_speedup": sum(single_ms) / ms_per_step if single_ms else None,
        "inversion_route": {"ms": inv_ms, "counts_equal": inv_counts == counts} if inv_counts else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": logical_bytes, "kernel": "pg::match_kernel",
                     "kernel_hash": khash},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, specs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
