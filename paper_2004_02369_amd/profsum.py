"""Summaries of the rocprofv3 passes of paper_2004_02369_amd/profile.sh.

    python -m paper_2004_02369_amd.profsum --workload rmat22_64m --raw gpurun_out --out profiles

Reads the raw CSV output of the passes (kernel trace, FETCH_SIZE, WRITE_SIZE,
SQ and TA/TCP counters, copy calibration) and writes, for the benchmark's
matching kernel:

* match_kernel_<workload>_kernel_trace.md -- per-kernel calls and durations;
* match_kernel_<workload>_traffic.txt -- HBM-side bytes per launch (the
  FETCH_SIZE / WRITE_SIZE counters scaled by what they read for a plain copy
  of known size); bench.py reads its kernel_hash and hbm_bytes_per_launch;
* match_kernel_<workload>_pmc.md -- issue, LDS and texture-unit counters.

The benchmark's launches under profile.sh are one bytes-counting run and two
timed steps; counters are averaged over the timed ones (the last
TIMED_STEPS dispatches of match_kernel).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import sys

KERNEL = "pg::match_kernel("
CLOCK_GHZ = 2.4
SIMDS = 1024
CUS = 256
BENCH = "python3 bench.py --steps 2 --warmup 0 --no-cpu-baseline --no-extras"
TIMED_STEPS = 2


def kernel_hash(root: str) -> str:
    h = hashlib.sha256()
    for f in ("engine.hip", "engine.hpp", "pg_internal.hpp"):
        with open(os.path.join(root, "paper_2004_02369_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters(path: str, kernel: str):
    """{dispatch id: {counter: value}} for dispatches of `kernel`, in order."""
    out = collections.OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            if not r["Kernel_Name"].startswith(kernel):
                continue
            d = out.setdefault(int(r["Dispatch_Id"]), collections.defaultdict(float))
            d[r["Counter_Name"]] += float(r["Counter_Value"])
    return out


def timed(disp):
    """Counters of the timed dispatches (the last TIMED_STEPS)."""
    vals = list(disp.values())[-TIMED_STEPS:]
    keys = set().union(*vals)
    return {k: sum(v.get(k, 0.0) for v in vals) / len(vals) for k in keys}


def find(raw: str, sub: str, suffix: str):
    d = os.path.join(raw, sub)
    for f in sorted(os.listdir(d)):
        if f.endswith(suffix):
            return os.path.join(d, f)
    raise FileNotFoundError(f"{d}/*{suffix}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat22_64m")
    ap.add_argument("--raw", default="gpurun_out")
    ap.add_argument("--out", default="profiles")
    ap.add_argument("--bench-json", default="", help="bench.py output of a plain run (kernel ms, merge bytes)")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    khash = kernel_hash(root)
    wl = args.workload
    bench = {}
    if args.bench_json:
        with open(args.bench_json) as f:
            bench = json.loads(f.read().strip().splitlines()[-1])
    os.makedirs(args.out, exist_ok=True)

    # kernel trace
    stats = list(csv.DictReader(open(find(args.raw, "prof_kt", "kernel_stats.csv"))))
    trace = [r for r in csv.DictReader(open(find(args.raw, "prof_kt", "kernel_trace.csv")))
             if r["Kernel_Name"].startswith(KERNEL)]
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in trace]
    timed_ms = durs[-TIMED_STEPS:]
    avg_timed = sum(timed_ms) / len(timed_ms)
    lines = [f"# pg::match_kernel on {wl} (the benchmark's batch in one launch): kernel trace", "",
             "Command (run from the repository root):", "",
             f"    bash paper_2004_02369_amd/profile.sh kt", "",
             f"which runs `rocprofv3 --kernel-trace --stats -- {BENCH}`.", "",
             f"kernel_hash (engine sources): {khash}", "",
             "| kernel | calls | average ms | min ms | max ms |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                     f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} |")
    lines += ["", f"match_kernel dispatches in order (ms): {', '.join(f'{d:.1f}' for d in durs)}; the last "
              f"{TIMED_STEPS} are the timed steps (the bytes-counting run, if listed, comes first): "
              f"average {avg_timed:.1f} ms."]
    if bench:
        lines.append(f"bench.py's HIP-event average in a plain run of the same workload: {bench['kernel_ms']:.1f} ms.")
    with open(os.path.join(args.out, f"match_kernel_{wl}_kernel_trace.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    # traffic
    fetch = timed(counters(find(args.raw, "prof_fetch", "counter_collection.csv"), KERNEL))["FETCH_SIZE"]
    write = timed(counters(find(args.raw, "prof_write", "counter_collection.csv"), KERNEL))["WRITE_SIZE"]
    cfetch = sum(v["FETCH_SIZE"] for v in counters(find(args.raw, "prof_cfetch", "counter_collection.csv"),
                                                   "__amd_rocclr_copyBuffer").values())
    cwrite = sum(v["WRITE_SIZE"] for v in counters(find(args.raw, "prof_cwrite", "counter_collection.csv"),
                                                   "__amd_rocclr_copyBuffer").values())
    copy_kib = 512 * 1024
    ff, fw = copy_kib / cfetch, copy_kib / cwrite
    fetch_b, write_b = fetch * 1024 * ff, write * 1024 * fw
    hbm = fetch_b + write_b
    t = [f"# pg::match_kernel on {wl} (the benchmark's batch in one launch): HBM-side traffic", "",
         "Counters from two rocprofv3 PMC passes, one counter each, scaled by what the",
         "same counter reads for a plain 512 MiB device-to-device copy (torch copy_,",
         "dispatched as __amd_rocclr_copyBuffer).", "",
         "Commands (run from the repository root):",
         "  bash paper_2004_02369_amd/profile.sh fetch write cfetch cwrite",
         f"  (rocprofv3 --pmc FETCH_SIZE / --pmc WRITE_SIZE -- {BENCH}, and the same around",
         "   python3 bench.py --calibrate-copy 512)", "",
         f"Copy calibration (512 MiB = {copy_kib} KiB read and written):",
         f"  copy FETCH_SIZE KiB: {cfetch:.3f} -> fetch factor {ff:.4f}",
         f"  copy WRITE_SIZE KiB: {cwrite:.3f} -> write factor {fw:.4f}", "",
         "match_kernel per timed dispatch:",
         f"  FETCH_SIZE KiB: {fetch:.1f}", f"  WRITE_SIZE KiB: {write:.1f}", "",
         "Scaled per launch:", f"  fetch bytes: {fetch_b:.4e}", f"  write bytes: {write_b:.4e}",
         f"  at the traced average of {avg_timed:.1f} ms: {hbm / (avg_timed * 1e-3) / 1e9:.0f} GB/s"]
    if bench:
        t += ["", f"Algorithmic (merge-model) bytes per launch: {bench['roofline']['algorithmic_bytes_per_launch']:.4e}",
              f"Streaming-read bandwidth measured in the same bench run: "
              f"{bench['roofline']['achievable_read_gbs']:.0f} GB/s"]
    t += ["", f"kernel_hash: {khash}"]
    if bench:
        t.append(f"knobs: {json.dumps(bench.get('knobs', {}), sort_keys=True)}")
    t.append(f"hbm_bytes_per_launch: {hbm:.6e}")
    with open(os.path.join(args.out, f"match_kernel_{wl}_traffic.txt"), "w") as f:
        f.write("\n".join(t) + "\n")

    # issue counters
    sq = timed(counters(find(args.raw, "prof_sq", "counter_collection.csv"), KERNEL))
    ta = timed(counters(find(args.raw, "prof_ta", "counter_collection.csv"), KERNEL))
    cycles = avg_timed * 1e-3 * CLOCK_GHZ * 1e9
    rows = [
        ("SQ_WAVES", sq.get("SQ_WAVES"), "persistent grid"),
        ("SQ_INSTS_VALU", sq.get("SQ_INSTS_VALU"),
         f"VALU issue {100 * sq.get('SQ_INSTS_VALU', 0) / (cycles * SIMDS):.1f}% of 1 per SIMD per cycle"),
        ("SQ_INSTS_VMEM_RD", sq.get("SQ_INSTS_VMEM_RD"),
         f"{sq.get('SQ_INSTS_VMEM_RD', 0) / (avg_timed * 1e-3):.3g} vector loads/s"),
        ("SQ_INSTS_LDS", sq.get("SQ_INSTS_LDS"), ""),
        ("SQ_LDS_BANK_CONFLICT", sq.get("SQ_LDS_BANK_CONFLICT"),
         f"{100 * sq.get('SQ_LDS_BANK_CONFLICT', 0) / (cycles * CUS):.1f}% of CU cycles stalled on LDS bank conflicts"),
        ("SQ_WAIT_INST_ANY", sq.get("SQ_WAIT_INST_ANY"),
         f"{100 * sq.get('SQ_WAIT_INST_ANY', 0) / max(1, sq.get('SQ_WAVE_CYCLES', 1)):.1f}% of wave cycles"),
        ("SQ_WAVE_CYCLES", sq.get("SQ_WAVE_CYCLES"), ""),
        ("SQ_BUSY_CYCLES", sq.get("SQ_BUSY_CYCLES"), ""),
        ("TA_BUSY_avr", ta.get("TA_BUSY_avr"), f"{100 * ta.get('TA_BUSY_avr', 0) / cycles:.1f}% of the kernel's cycles"),
        ("TA_BUSY_max", ta.get("TA_BUSY_max"), f"{100 * ta.get('TA_BUSY_max', 0) / cycles:.1f}%"),
        ("TCP_TCC_READ_REQ_sum", ta.get("TCP_TCC_READ_REQ_sum"),
         f"{ta.get('TCP_TCC_READ_REQ_sum', 0) / (avg_timed * 1e-3):.3g} L1-to-L2 read requests/s"),
    ]
    p = [f"# pg::match_kernel on {wl} (the benchmark's batch in one launch): issue counters", "",
         "Commands (run from the repository root):", "",
         "    bash paper_2004_02369_amd/profile.sh sq ta", "",
         "(rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT",
         " SQ_WAIT_INST_ANY SQ_WAVE_CYCLES SQ_BUSY_CYCLES, then --pmc TA_BUSY_avr TA_BUSY_max",
         f" TCP_TCC_READ_REQ_sum, around {BENCH})", "",
         f"kernel_hash (engine sources): {khash}.  Values per timed dispatch; kernel {avg_timed:.1f} ms "
         f"(trace average), clock {CLOCK_GHZ} GHz, {SIMDS} SIMDs, {CUS} CUs.", "",
         "| counter | per launch | derived |", "|---|---|---|"]
    for name, v, d in rows:
        p.append(f"| {name} | {v:.4g} | {d} |" if v is not None else f"| {name} | n/a | |")
    with open(os.path.join(args.out, f"match_kernel_{wl}_pmc.md"), "w") as f:
        f.write("\n".join(p) + "\n")
    print(json.dumps({"kernel_hash": khash, "avg_timed_ms": avg_timed, "hbm_bytes_per_launch": hbm}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
