"""Benchmark: exact counts of a batch of pattern queries in one launch on the
serving graph, an R-MAT graph of 2^22 vertices and 2^26 unique undirected
edges (a=0.57, b=c=0.19) resident in HBM, the largest workload that fits
one GPU.  The batch is the serving catalogue's count queries that finish
alone on this graph: triangle, wedge, induced (open) wedge, 4-clique (also
the induced 4-clique), book of three triangles, and the cricket (triangle
with two pendants on one vertex).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one pg_count_ex call over the batch (plans compiled once, one
launch, device reduction, counts back to the host).  Beside the timed
steps the line reports: each pattern alone (batched vs one launch per
pattern), p50/p99 latency of a short seeded Poisson stream of mixed
queries served with continuous batching, the six induced 4-motifs on the
Chung-Lu 100K / 1M graph, the merge-model roofline with the streaming-read
bandwidth measured on the same GPU, and the CPU oracle on a bounded sample.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "rmat22_64m"
C2_WORKLOAD = "chunglu_100k_1m"
HBM_PEAK_GBPS = 8000.0
# the batch: names in the serving catalogue (paper_2004_02369_amd.serve)
from paper_2004_02369_amd.serve import SERVING_BATCH as BATCH  # noqa: E402
SERVE_EXTRA = ["clique6_exists", "clique8_exists", "clique10_exists", "clique12_exists", "clique14_exists"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("engine.hip", "engine.hpp", "pg_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2004_02369_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel_hash, knobs):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source with the same launch knobs;
    else None."""
    path = os.path.join(ROOT, "profiles", f"match_kernel_{workload}_traffic.txt")
    t = {}
    try:
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", " ", "-")):
                    k, v = line.split(":", 1)
                    t[k.strip()] = v.strip()
    except OSError:
        return None
    if t.get("kernel_hash") != kernel_hash or t.get("knobs") != json.dumps(knobs, sort_keys=True):
        return None
    try:
        return float(t["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(g, specs, names, budget_s=3.0):
    """The oracle's generic matcher (valid maps / |Aut_t|, no symmetry
    breaking, no set arithmetic) on a bounded sample of the same graph:
    start vertices (pattern vertex 0) in a seeded random order, in blocks of
    256 handed to all host threads at once, until the time budget is spent;
    matches/s = sum over patterns of (valid maps from the sample / |Aut_t|)
    over the time.  Three passes over the same blocks give the median; a
    one-thread pass over the first 64 start vertices follows."""
    import numpy as np
    import oracle
    t = time.perf_counter()
    og = oracle.Graph.from_tuple(g)
    build_s = time.perf_counter() - t
    threads = oracle.default_threads()
    rng = np.random.Generator(np.random.PCG64(99))
    order = rng.permutation(og.n).astype(np.int32)
    auts = [oracle.aut(s) for s in specs]

    def run(roots, nthreads):
        t0 = time.perf_counter()
        m = sum(oracle.valid_maps_from(og, s, roots, nthreads) / a for s, a in zip(specs, auts))
        return m, time.perf_counter() - t0

    blocks, spent = [], 0.0
    while spent < budget_s and 256 * len(blocks) < og.n:
        blocks.append(order[256 * len(blocks):256 * (len(blocks) + 1)])
        spent += run(blocks[-1], threads)[1]
    passes = []
    for _ in range(3):
        res = [run(b, threads) for b in blocks]
        passes.append((sum(m for m, _ in res), sum(dt for _, dt in res)))
    rates = sorted(m / dt for m, dt in passes)
    m1, dt1 = run(blocks[0][:64], 1)
    used = sum(len(b) for b in blocks)
    return {"value": rates[1], "unit": "matches/s", "cores": threads, "kind": "oracle",
            "sample": f"generic matcher, patterns {', '.join(names)} of the batch (the others grow as "
                      f"degree^3 or more per start vertex), {used} of {og.n} seeded random start vertices in "
                      f"blocks of 256; median of 3 passes of {statistics.median(dt for _, dt in passes):.1f} s",
            "one_core": {"value": m1 / dt1, "cores": 1, "sample": f"the first 64 start vertices, {dt1:.1f} s"},
            "cpu_model": cpu_model(), "oracle_graph_build_s": build_s}


def achievable_bandwidth():
    """Streaming read of a 4 GiB buffer (librowbench rb_stream_read)."""
    import torch
    from paper_2004_02369_amd import rowbench
    buf = torch.ones(1 << 30, dtype=torch.int32, device="cuda:0")
    ms, _ = rowbench.stream_read(buf, reps=5)
    del buf
    torch.cuda.empty_cache()
    return 4.0 * (1 << 30) / (ms * 1e-3) / 1e9


def serve_window(pg, G, queries, single_ms, qps, n_requests, seed):
    """A seeded Poisson stream of mixed catalogue queries through the serving
    loop (continuous batching, memory admission, early-exit existence):
    p50/p99 latency from arrival to result, completed QPS, and every served
    count equal to the batched launch's."""
    from paper_2004_02369_amd import serve
    slots = serve.default_slots()
    pol = serve.Policy(light_ms=100.0)
    for q in queries:
        if q.kind == "count":
            pol.est[id(q.plans[0])] = single_ms[q.name] * slots
    pool = 40 << 30
    srv = serve.Server(G, pool, slots=slots, time_limit_ms=120000, policy=pol)
    times, picks = serve.poisson_arrivals(qps, n_requests, len(queries), seed)
    reqs, t0 = serve.run_open_loop(srv, queries, times, picks)
    summ = serve.summarize(reqs, t0)
    return reqs, {"qps_offered": qps, "requests": n_requests, "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"],
                  "completed_qps": summ["completed_qps"], "launches": srv.launches,
                  "merged_requests": srv.merged_requests, "slots": slots, "pool_bytes": pool}


def c2_figures(pg, gg, pt, stream, steps):
    """The six vertex-induced 4-motifs on Chung-Lu 100K / 1M in one launch
    (tuned knobs from the committed record), against one launch each."""
    from paper_2004_02369_amd import tune
    G = pg.load_graph(*gg.workload(C2_WORKLOAD), device=0)
    plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
    rec = tune.lookup(G, plans, tune.RECORDS)
    knobs = {k: v for k, v in (rec["knobs"] if rec else {}).items() if v}
    _, stb = pg.count_ex(G, plans, stream=stream, **dict(knobs, flags=knobs.get("flags", 0) | pg.PG_RUN_COUNT_BYTES))
    for _ in range(2):
        pg.count_ex(G, plans, stream=stream, **knobs)
    ms = []
    for _ in range(steps):
        counts, st = pg.count_ex(G, plans, stream=stream, **knobs)
        ms.append(st["kernel_ms"])
    single = []
    for p in plans:
        pg.count_ex(G, [p], stream=stream, **knobs)
        single.append(min(pg.count_ex(G, [p], stream=stream, **knobs)[1]["kernel_ms"] for _ in range(2)))
    kms = statistics.median(ms)
    return {"workload": f"Chung-Lu n=100000, m={G.m}, gamma=2.1, w_max=5000; 6 induced 4-motifs in one launch",
            "kernel_ms": kms, "matches_per_s": sum(counts) / (kms * 1e-3), "counts": counts,
            "merge_model_bytes": stb["logical_bytes"],
            "merge_model_frac_of_8tbs": stb["logical_bytes"] / (kms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "per_pattern_kernel_ms": single, "batched_speedup": sum(single) / kms, "knobs": knobs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed steps and the roofline")
    ap.add_argument("--serve-qps", type=float, default=100.0)
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--knobs", default=None, metavar="JSON", help="launch knobs to time, e.g. '{\"chunk\": 16}'")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for HBM counters) and exit")
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
    from paper_2004_02369_amd import serve

    def say(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    w = gg.WORKLOADS[WORKLOAD]
    t = time.perf_counter()
    g = gg.workload(WORKLOAD)
    say(f"generated {WORKLOAD} in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    G = pg.load_graph(*g, device=0)
    say(f"ingested n={G.n} m={G.m} d_max={G.d_max} in {time.perf_counter() - t:.1f} s")
    queries = {q.name: q for q in serve.catalogue(pg, pt)}
    plans = [queries[n].plans[0] for n in BATCH]
    plan_ms = sum(p.info()["plan_ms"] for p in plans)
    # launch knobs: the committed tuning record for this graph and batch
    # (paper_2004_02369_amd/tuned.json, written by `measure tune`), unless given
    tuning = None
    if args.knobs:
        knobs = json.loads(args.knobs)
    else:
        from paper_2004_02369_amd import tune
        rec = tune.lookup(G, plans, tune.RECORDS)
        knobs = {k: v for k, v in (rec["knobs"] if rec else {}).items() if v}
        if rec:
            tuning = {"record": True, "default_kernel_ms": rec["default_ms"], "tuned_kernel_ms": rec["ms"],
                      "trials": len(rec["trials"])}

    # merge-model bytes of one launch (a separate, untimed counting run)
    counts_b, st_b = pg.count_ex(G, plans, stream=stream, **dict(knobs, flags=knobs.get("flags", 0) | pg.PG_RUN_COUNT_BYTES))
    logical_bytes = st_b["logical_bytes"]
    say(f"merge-model bytes per launch {logical_bytes:.4g}")

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
    say(f"{args.steps} steps in {elapsed:.2f} s, kernel {statistics.mean(kernel_ms):.1f} ms")
    ms_per_step = 1e3 * elapsed / args.steps
    avg_kernel_ms = statistics.mean(kernel_ms)
    total = sum(counts)

    out = {
        "metric": "pattern matches/sec (batch of serving count queries, one launch)",
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
        "config": {"workload": f"R-MAT scale {w['scale']} (a=0.57, b=c=0.19), n={G.n}, m={G.m} unique undirected "
                               f"edges, seed={w['seed']}; {len(BATCH)} count queries in one launch: "
                               + ", ".join(BATCH),
                   "n": G.n, "m": G.m, "d_max": G.d_max, "patterns": len(BATCH), "parallelism": "1 GPU"},
        "knobs": knobs,
        "tuning": tuning,
        "counts": dict(zip(BATCH, counts)),
        "kernel_ms": avg_kernel_ms,
        "plan_ms": plan_ms,
    }

    khash = kernel_source_hash()
    traffic = measured_traffic(WORKLOAD, khash, knobs)
    achieved = logical_bytes / (avg_kernel_ms * 1e-3) / 1e9
    achievable = achievable_bandwidth()
    say(f"streaming read {achievable:.0f} GB/s")
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                       "algorithmic_bytes_per_launch": logical_bytes,
                       "algorithmic_bytes": "merge model: 4 (|A| + |B|) per executed set operation",
                       "achievable_read_gbs": achievable, "frac_of_achievable": achieved / achievable,
                       "measured_frac_of_achievable": (traffic / (avg_kernel_ms * 1e-3) / 1e9 / achievable
                                                       if traffic else None),
                       "kernel": "pg::match_kernel", "kernel_hash": khash}

    if not args.no_extras:
        # each pattern alone, the same plans, best of two
        single = {}
        for name, p in zip(BATCH, plans):
            pg.count_ex(G, [p], stream=stream, **knobs)
            single[name] = min(pg.count_ex(G, [p], stream=stream, **knobs)[1]["kernel_ms"] for _ in range(2))
        out["per_pattern_kernel_ms"] = single
        out["batched_speedup"] = sum(single.values()) / avg_kernel_ms
        say(f"one launch per pattern: {sum(single.values()):.1f} ms")
        # served: a short Poisson window of the batch's queries and clique existence
        sq = [queries[n] for n in BATCH + SERVE_EXTRA]
        reqs, win = serve_window(pg, G, sq, single, args.serve_qps, args.serve_requests, seed=7)
        want = dict(zip(BATCH, counts))
        win["mismatches"] = sum(1 for r in reqs if r.query.kind == "count" and r.result != [want[r.query.name]])
        win["errors"] = sum(1 for r in reqs if r.error is not None)
        out["serving"] = win
        say(f"serving p50 {win['p50_ms']:.1f} ms p99 {win['p99_ms']:.1f} ms")
        del G
        torch.cuda.empty_cache()
        out["c2"] = c2_figures(pg, gg, pt, stream, steps=5)
        say(f"C2 six motifs {out['c2']['kernel_ms']:.1f} ms")
    if not args.no_cpu_baseline:
        names = ["triangle", "wedge", "induced_wedge"]
        out["cpu_baseline"] = cpu_baseline(g, [queries[n].specs[0] for n in names], names)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
