"""Frequent subgraph mining with MNI support (Sec. 2, Sec. 3.2, Sec. 5.5).

The loop follows the paper's FSM program: match the candidate patterns,
keep those whose support reaches the threshold, extend the frequent ones by
one edge, repeat.  Support is the minimum node image (MNI): the smallest,
over the pattern's vertices, number of distinct data vertices that vertex is
mapped to by some match (anti-monotone: a pattern's support never exceeds a
sub-pattern's).

Label discovery: a new vertex's label is not known in advance.  The
candidates give it every label of the graph's alphabet whose labelled edge
to its attachment vertex is frequent (anti-monotonicity rules out the
rest), and each labelled candidate is matched as its own pattern.

Support on the GPU: a pattern's domain sizes come from anchored plans (one
per automorphism orbit of the labelled pattern), batched up to 64 per
launch (``pg.domain_sizes``).  Everything in this module is host logic.

    python -m paper_2004_02369_amd.fsm --workload chunglu_1m_10m_l16 --support 10000 --edges 3
"""
from __future__ import annotations

import argparse
import itertools
import json
import sys
import time
from dataclasses import dataclass


@dataclass(frozen=True)
class LPattern:
    """A connected labelled pattern: k vertices, edges as sorted pairs,
    one label per vertex.  Instances built by `canonical` are canonical."""
    k: int
    edges: tuple
    labels: tuple

    def spec(self) -> dict:
        return {"k": self.k, "edges": [tuple(e) for e in self.edges], "labels": list(self.labels)}


def _relabel(p: LPattern, perm) -> tuple:
    edges = tuple(sorted(tuple(sorted((perm[a], perm[b]))) for a, b in p.edges))
    labels = [0] * p.k
    for i in range(p.k):
        labels[perm[i]] = p.labels[i]
    return labels, edges


def canonical(k: int, edges, labels) -> LPattern:
    """The smallest (labels, edges) over all relabellings of the vertices."""
    p = LPattern(k, tuple(sorted(tuple(sorted(e)) for e in edges)), tuple(labels))
    best = None
    for perm in itertools.permutations(range(k)):
        key = _relabel(p, perm)
        if best is None or key < best:
            best = key
    labels_c, edges_c = best
    return LPattern(k, edges_c, tuple(labels_c))


def automorphisms(p: LPattern):
    E = set(p.edges)
    out = []
    for perm in itertools.permutations(range(p.k)):
        if any(p.labels[i] != p.labels[perm[i]] for i in range(p.k)):
            continue
        if all(tuple(sorted((perm[a], perm[b]))) in E for a, b in p.edges):
            out.append(perm)
    return out


def orbit_representatives(p: LPattern) -> list[int]:
    """One vertex per orbit of the labelled pattern's automorphism group
    (automorphic vertices have equal domains)."""
    auts = automorphisms(p)
    seen, reps = set(), []
    for u in range(p.k):
        if u in seen:
            continue
        reps.append(u)
        seen |= {perm[u] for perm in auts}
    return reps


def _connected(k: int, edges) -> bool:
    adj = {i: set() for i in range(k)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen, todo = {0}, [0]
    while todo:
        x = todo.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                todo.append(y)
    return len(seen) == k


def single_edges(alphabet) -> list[LPattern]:
    return sorted({canonical(2, [(0, 1)], (a, b)) for a, b in itertools.combinations_with_replacement(alphabet, 2)},
                  key=lambda p: (p.labels, p.edges))


def extend_by_edge(frequent, alphabet, frequent_edges=None) -> list[LPattern]:
    """All distinct connected patterns with one more edge: between two
    existing non-adjacent vertices, or to a new vertex labelled from the
    alphabet.  With frequent_edges (canonical single edges), a new vertex
    only takes labels whose edge to its attachment is frequent."""
    out = set()
    for p in frequent:
        E = set(p.edges)
        for a, b in itertools.combinations(range(p.k), 2):
            if (a, b) not in E:
                out.add(canonical(p.k, E | {(a, b)}, p.labels))
        for a in range(p.k):
            for lab in alphabet:
                if frequent_edges is not None and canonical(2, [(0, 1)], (p.labels[a], lab)) not in frequent_edges:
                    continue
                out.add(canonical(p.k + 1, E | {(a, p.k)}, p.labels + (lab,)))
    return sorted(out, key=lambda q: (q.k, q.labels, q.edges))


def sub_patterns(p: LPattern) -> list[LPattern]:
    """Connected patterns with one edge fewer (a vertex left isolated is
    dropped)."""
    out = set()
    for e in p.edges:
        rest = [f for f in p.edges if f != e]
        used = sorted({v for f in rest for v in f})
        if len(used) == p.k and _connected(p.k, rest):
            out.add(canonical(p.k, rest, p.labels))
        elif len(used) == p.k - 1:
            idx = {v: i for i, v in enumerate(used)}
            ren = [(idx[a], idx[b]) for a, b in rest]
            if ren and _connected(p.k - 1, ren):
                out.add(canonical(p.k - 1, ren, [p.labels[v] for v in used]))
    return sorted(out, key=lambda q: (q.k, q.labels, q.edges))


def mine(support_fn, alphabet, threshold: int, max_edges: int, log=None):
    """The FSM loop.  support_fn(list of LPattern) -> list of MNI supports.
    Returns {n_edges: {pattern: support}} of the frequent patterns, and
    per-level statistics."""
    alphabet = sorted(set(int(a) for a in alphabet))
    frequent_by_level, stats = {}, []
    cands = single_edges(alphabet)
    freq_edges = None
    for n_edges in range(1, max_edges + 1):
        if n_edges > 1:
            prev = set(frequent_by_level[n_edges - 1])
            cands = extend_by_edge(sorted(prev, key=lambda q: (q.k, q.labels, q.edges)), alphabet, freq_edges)
            # anti-monotone pruning: every sub-pattern must be frequent
            cands = [c for c in cands if all(s in prev for s in sub_patterns(c) if len(s.edges) == n_edges - 1)]
        t0 = time.perf_counter()
        sup = support_fn(cands) if cands else []
        dt = time.perf_counter() - t0
        freq = {c: s for c, s in zip(cands, sup) if s >= threshold}
        frequent_by_level[n_edges] = freq
        if n_edges == 1:
            freq_edges = set(freq)
        stats.append({"edges": n_edges, "candidates": len(cands), "frequent": len(freq), "seconds": dt})
        if log:
            log(f"{n_edges} edge(s): {len(cands)} candidates, {len(freq)} frequent, {dt:.2f} s")
        if not freq:
            break
    return frequent_by_level, stats


class OutOfTime(RuntimeError):
    pass


def gpu_support(G, pg, batch: int = 64, log=None, deadline: float | None = None, **knobs):
    """support_fn running on libpg: one anchored plan per orbit
    representative, batched across patterns, `batch` plans per launch.
    deadline (time.perf_counter() value): raise OutOfTime when passed."""
    stats = {"launches": 0, "plans": 0, "kernel_s": 0.0}

    def support(cands):
        jobs = []  # (pattern index, plan)
        order = []
        for i, p in enumerate(cands):
            for u in orbit_representatives(p):
                order.append((p.labels[u], sorted(p.labels), p.k, i, u))
        # plans whose roots carry the same labels share trie roots in a launch
        order.sort()
        for _, _, _, i, u in order:
            jobs.append((i, pg.plan_pattern(cands[i].spec(), anchor=u)))
        best = [None] * len(cands)
        t_log = time.perf_counter()
        for s in range(0, len(jobs), batch):
            part = jobs[s:s + batch]
            t0 = time.perf_counter()
            sizes = pg.domain_sizes(G, [pl for _, pl in part], **knobs)
            stats["kernel_s"] += time.perf_counter() - t0
            stats["launches"] += 1
            stats["plans"] += len(part)
            if log and time.perf_counter() - t_log > 15:
                log(f"  {s + len(part)}/{len(jobs)} anchored plans")
                t_log = time.perf_counter()
            if deadline is not None and time.perf_counter() > deadline:
                stats["level_plans_done"], stats["level_plans"] = s + len(part), len(jobs)
                raise OutOfTime(f"{s + len(part)} of {len(jobs)} anchored plans done")
            for (i, _), sz in zip(part, sizes):
                best[i] = sz if best[i] is None else min(best[i], sz)
        for _, pl in jobs:
            pl.free()
        return best

    support.stats = stats
    return support


def main(argv=None):
    ap = argparse.ArgumentParser(description="frequent subgraph mining with MNI support")
    ap.add_argument("--workload", default="chunglu_1m_10m_l16")
    ap.add_argument("--support", type=int, default=10000)
    ap.add_argument("--edges", type=int, default=3)
    ap.add_argument("--budget-s", type=float, default=0.0, help="stop (and report progress) after this long")
    args = ap.parse_args(argv)

    import torch
    from . import graphgen as gg
    from . import pg

    def say(*a):
        print("[fsm]", *a, file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "FSM on the GPU needs a GPU"
    t = time.perf_counter()
    n, src, dst, labels = gg.labelled_workload(args.workload)
    say(f"generated {args.workload} in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    G = pg.load_graph(n, src, dst, labels=labels, device=0)
    say(f"ingested n={G.n} m={G.m} d_max={G.d_max} in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    support = gpu_support(G, pg, log=say, deadline=t + args.budget_s if args.budget_s else None)
    levels = []
    try:
        freq, stats = mine(support, sorted(set(labels.tolist())), args.support, args.edges,
                           log=lambda m: (say(m), levels.append(m)))
        finished = True
    except OutOfTime as e:
        say(f"time budget spent: {e}")
        freq, stats, finished = {}, levels, False
    total = time.perf_counter() - t
    out = {"workload": args.workload, "n": G.n, "m": G.m, "d_max": G.d_max, "support": args.support,
           "max_edges": args.edges, "seconds": total, "finished": finished, "levels": stats, **support.stats,
           "frequent": {str(e): len(f) for e, f in freq.items()}}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
