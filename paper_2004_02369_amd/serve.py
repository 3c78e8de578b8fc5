"""Serving many pattern queries over one resident graph.

Requests arrive over time (count or existence queries).  The loop admits
them while launch slots and workspace memory are free:

* every admitted batch is one asynchronous launch (``pg.submit``) on a stream
  of its own, with a grid of ``resident waves / slots`` wavefronts, so up to
  ``slots`` launches run side by side; a heavy launch (by the cost policy)
  holds ``slots - 1`` slots and their share of the grid, one at a time, so
  one slot always stays for light requests and a heavy launch ends sooner;
* count requests waiting in the queue are merged into one launch
  (continuous batching): their plans share one root frontier (Sec. 5.4),
  identical plans are counted once, up to 64 plans per launch;
* an existence query runs in a launch of its own (shared only with repeats
  of the same query), with its own stop flag, and ends at the first match
  (Sec. 5.3);
* a launch is admitted only when its workspace (control words, program trie,
  per-wavefront scratch) fits in what is left of a fixed device pool; the
  pool is carved first-fit, never grown.

Everything here is host logic; the matching runs in libpg.

    python -m paper_2004_02369_amd.serve --workload rmat22_64m --qps 50,100,200,500
"""
from __future__ import annotations

import argparse
import collections
import itertools
import json
import math
import sys
import time
from dataclasses import dataclass, field

ALIGN = 256
MAX_PLANS = 64


# ------------------------------------------------------------------ pool

class Pool:
    """First-fit allocator of byte ranges in [0, size), ALIGN-aligned."""

    def __init__(self, size: int):
        self.size = size - size % ALIGN
        self.free_list = [(0, self.size)]  # sorted (offset, length)
        self.live = {}

    @property
    def used(self) -> int:
        return sum(self.live.values())

    def largest_free(self) -> int:
        return max((n for _, n in self.free_list), default=0)

    def alloc(self, nbytes: int):
        n = max(ALIGN, -(-nbytes // ALIGN) * ALIGN)
        for i, (off, length) in enumerate(self.free_list):
            if length >= n:
                if length == n:
                    del self.free_list[i]
                else:
                    self.free_list[i] = (off + n, length - n)
                self.live[off] = n
                return off
        return None

    def free(self, off: int):
        n = self.live.pop(off)
        fl = self.free_list
        fl.append((off, n))
        fl.sort()
        merged = []
        for o, ln in fl:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free_list = merged


# --------------------------------------------------------------- requests

@dataclass
class Query:
    """A catalogue entry: a name, "count" or "exists", and its plans (one
    for an existence query)."""
    name: str
    kind: str
    plans: list
    specs: list = field(default_factory=list)

    def __post_init__(self):
        if self.kind not in ("count", "exists"):
            raise ValueError(self.kind)
        if self.kind == "exists" and len(self.plans) != 1:
            raise ValueError("an existence query has one plan")
        if not 1 <= len(self.plans) <= MAX_PLANS:
            raise ValueError("a query has 1..64 plans")


@dataclass
class Request:
    rid: int
    query: Query
    arrival: float
    admitted: float | None = None
    done: float | None = None
    result: object = None
    error: str | None = None
    launch: int = -1


@dataclass
class Batch:
    """Requests admitted together as one launch."""
    requests: list
    plans: list                 # unique plans, launch order
    index: list                 # per request: positions of its plans in `plans`
    kind: str
    nbytes: int
    offset: int = -1
    slot: int = -1
    extra_slots: list = field(default_factory=list)  # further slots a wide (heavy) launch holds
    grid: int = 0
    job: object = None
    t_submit: float = 0.0
    heavy: bool = False
    lid: int = -1
    # a heavy count launch runs as consecutive root-task windows: those still
    # to run, the counts and kernel time of the windows done so far
    windows: list = field(default_factory=list)
    acc: list = None
    kernel_ms: float = 0.0
    waiting: bool = False       # between two windows: holds its workspace and one slot


def _merge(requests):
    plans, pos, index = [], {}, []
    for r in requests:
        ix = []
        for p in r.query.plans:
            if id(p) not in pos:
                pos[id(p)] = len(plans)
                plans.append(p)
            ix.append(pos[id(p)])
        index.append(ix)
    return plans, index


@dataclass
class Policy:
    """Cost model of admission.  est maps id(plan) to the estimated duration
    (ms) of a launch of that plan alone at the server's grid; a plan with no
    estimate costs 0.  A request is heavy when its plans cost more than
    light_ms.  Launches are formed within one class, so light requests never
    wait behind a heavy one in the same launch, and requests with new plans
    join a launch only while its estimated cost stays within
    max(head's cost, merge_cap_ms).  Requests whose plans are already in the
    launch always join: they add no work."""
    light_ms: float = 100.0
    merge_cap_ms: float = 200.0
    est: dict = field(default_factory=dict)

    def cost(self, plans) -> float:
        return sum(self.est.get(id(p), 0.0) for p in plans)

    def heavy(self, req) -> bool:
        return self.cost(req.query.plans) > self.light_ms

    def observe(self, plans, ms: float):
        """Fold a finished launch's duration into the estimates."""
        if len(plans) == 1:
            k = id(plans[0])
            old = self.est.get(k)
            self.est[k] = ms if old is None else 0.5 * (old + ms)
        else:
            for p in plans:
                self.est.setdefault(id(p), ms / len(plans))


class _Failed:
    """Stands in for the job of a windowed launch whose next window could not
    start: done at once, finish() raises the error."""

    def __init__(self, msg):
        self.msg = msg

    def done(self):
        return True

    def finish(self):
        from . import pg
        raise pg.PGError(pg.PG_EDEVICE, self.msg)


def next_batch(queue, size_of, pool: Pool, policy: Policy | None = None, allow_heavy: bool = True):
    """Choose the next launch from the queue.

    The head is the oldest request that may start now (heavy requests are
    skipped while allow_heavy is False).  Count requests of the head's class
    behind it join its launch while the unique plans stay within 64 and the
    policy's cost cap holds (existence requests run alone and keep their
    place).  The launch is cut from the back until its workspace fits.
    size_of(plans, kind, heavy) -> workspace bytes.  Returns (batch, rejected): a
    Batch (its workspace already carved from the pool) or None when nothing
    can start now; and the head if it can never fit (larger than the whole
    pool), else None."""
    policy = policy or Policy()
    head = None
    for r in queue:
        if allow_heavy or not policy.heavy(r):
            head = r
            break
    if head is None:
        return None, None
    heavy = policy.heavy(head)
    chosen = [head]
    if head.query.kind == "exists":
        # the same existence question asked again shares the answer
        chosen += [r for r in queue if r is not head and r.query.kind == "exists"
                   and r.query.plans[0] is head.query.plans[0]]
    else:
        ids = {id(p) for p in head.query.plans}
        cost = policy.cost(_merge(chosen)[0])
        cap = max(cost, policy.merge_cap_ms)
        for r in queue:
            if r is head or r.query.kind != "count" or policy.heavy(r) != heavy:
                continue
            new = {id(p): p for p in r.query.plans if id(p) not in ids}
            if len(ids) + len(new) > MAX_PLANS:
                continue
            add = policy.cost(new.values())
            if new and cost + add > cap:
                continue
            chosen.append(r)
            ids |= set(new)
            cost += add
    while True:
        plans, index = _merge(chosen)
        nbytes = size_of(plans, head.query.kind, heavy)
        if len(chosen) == 1 and nbytes > pool.size:
            return None, head
        off = pool.alloc(nbytes)
        if off is not None:
            return Batch(requests=chosen, plans=plans, index=index, kind=head.query.kind, nbytes=nbytes,
                         offset=off, heavy=heavy), None
        if len(chosen) == 1:
            return None, None
        chosen.pop()


def task_windows(total: int, n: int) -> list[tuple[int, int]]:
    """Cut root tasks [0, total) into at most n consecutive windows that
    partition them.  Tasks come costliest first, so the windows grow
    geometrically (each twice the one before) and their costs are closer to
    equal than equal task counts would give."""
    n = max(1, min(n, total))
    if n == 1 or total <= 1:
        return [(0, total)]
    unit = total / (2 ** n - 1)
    cuts = [0] + [min(total, max(1, round(unit * (2 ** (i + 1) - 1)))) for i in range(n - 1)] + [total]
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b > a:
            out.append((a, b))
    return out


# ----------------------------------------------------------------- server

_STREAMS = {}


def hw_queues() -> int:
    """Hardware queues HIP gives this process per device (its default is 4)."""
    import os
    try:
        return max(1, int(os.environ.get("GPU_MAX_HW_QUEUES", "4")))
    except ValueError:
        return 4


def default_slots() -> int:
    # one queue stays with the default stream; more streams than queues
    # would share queues, and work on a shared queue runs in order
    return max(1, min(4, hw_queues() - 1))


def slot_streams(device: str, n: int):
    """The first n of this process's serving streams on `device`, created
    once and reused (default priority)."""
    import torch
    pool = _STREAMS.setdefault(device, [])
    while len(pool) < n:
        pool.append(torch.cuda.Stream(device=device))
    return pool[:n]


class Server:
    """Admits requests into concurrent launches on one graph (see the module
    docstring).  Drive it with offer() and pump()."""

    def __init__(self, graph, pool_bytes: int, slots: int | None = None, time_limit_ms: int = 0,
                 policy: Policy | None = None, window_ms: float = 0.0):
        import torch
        from . import pg
        self.pg = pg
        self.g = graph
        slots = slots or default_slots()
        self.slots = slots
        self.grid = max(1, graph.resident_waves[0] // slots)
        self.time_limit_ms = time_limit_ms
        self.policy = policy or Policy()
        # one heavy launch at a time holds all slots but one (and their share
        # of the grid); the last slot stays for light ones
        self.heavy_width = max(1, slots - 1)
        dev = f"cuda:{graph.device}"
        pool_bytes = -(-pool_bytes // ALIGN) * ALIGN
        self.streams = slot_streams(dev, slots)
        raw = torch.empty(pool_bytes + ALIGN, dtype=torch.uint8, device=dev)
        shift = (-raw.data_ptr()) % ALIGN
        self._raw = raw
        self.mem = raw[shift:shift + pool_bytes]
        self.pool = Pool(pool_bytes)
        torch.cuda.synchronize(dev)
        self.free_slots = list(range(slots))
        self.queue = collections.deque()
        self.inflight = []
        self.finished = []
        self._sizes = {}
        self.launches = 0
        self.merged_requests = 0
        self.log = []  # one record per finished launch
        # heavy count launches are cut into root-task windows of about this
        # many ms each (by the policy's estimate); between two windows the
        # launch gives back its extra slots, so light requests start there
        self.window_ms = window_ms
        self.windows_run = 0

    def launch_shape(self, plans, kind, heavy=False):
        """(workspace bytes, grid) of a launch: a heavy one is wide unless its
        wide workspace could never fit the pool."""
        key = (tuple(id(p) for p in plans), kind, heavy)
        r = self._sizes.get(key)
        if r is None:
            mode = self.pg.PG_JOB_EXISTS if kind == "exists" else self.pg.PG_JOB_COUNT
            grid = self.grid * (self.heavy_width if heavy else 1)
            b = self.pg.job_workspace_size(self.g, plans, mode, grid_waves=grid)
            if grid != self.grid and b > self.pool.size:
                grid = self.grid
                b = self.pg.job_workspace_size(self.g, plans, mode, grid_waves=grid)
            r = self._sizes[key] = (b, grid)
        return r

    def size_of(self, plans, kind, heavy=False):
        return self.launch_shape(plans, kind, heavy)[0]

    def offer(self, req: Request):
        self.queue.append(req)

    def idle(self) -> bool:
        return not self.queue and not self.inflight

    def pump(self) -> int:
        """Retire finished launches, then admit what fits.  Returns the
        number of requests retired or admitted (0 = nothing to do now)."""
        pg = self.pg
        progress = 0
        for b in list(self.inflight):
            if b.job is not None and b.job.done():
                progress += self._advance(b) if b.windows else self._retire(b)
        while self.free_slots and self.queue:
            heavy_busy = any(x.heavy for x in self.inflight)
            allow_heavy = not heavy_busy and len(self.free_slots) >= self.heavy_width
            if not heavy_busy and not allow_heavy and self.policy.heavy(self.queue[0]):
                # the oldest request is heavy and waits for its slots: light
                # launches keep to the slots a heavy launch leaves free
                n_light = sum(1 for x in self.inflight if not x.heavy)
                if n_light >= self.slots - self.heavy_width:
                    break
            b, rejected = next_batch(self.queue, self.size_of, self.pool, self.policy, allow_heavy=allow_heavy)
            if rejected is not None:
                self.queue.remove(rejected)
                rejected.error = "workspace larger than the pool"
                rejected.done = time.perf_counter()
                self.finished.append(rejected)
                progress += 1
                continue
            if b is None:
                break
            for r in b.requests:
                self.queue.remove(r)
            b.slot = self.free_slots.pop()
            _, b.grid = self.launch_shape(b.plans, b.kind, b.heavy)
            if b.heavy:
                for _ in range(min(len(self.free_slots), b.grid // self.grid - 1)):
                    b.extra_slots.append(self.free_slots.pop())
            ws = self.mem[b.offset:b.offset + b.nbytes]
            mode = pg.PG_JOB_EXISTS if b.kind == "exists" else pg.PG_JOB_COUNT
            b.t_submit = time.perf_counter()
            win = {}
            if b.heavy and b.kind == "count" and self.window_ms > 0:
                n = int(math.ceil(self.policy.cost(b.plans) / max(1, len(b.extra_slots) + 1) / self.window_ms))
                if n > 1:
                    b.windows = task_windows(pg.launch_tasks(self.g, b.plans), min(n, 16))
                    b.acc = [0] * len(b.plans)
                    a, e = b.windows.pop(0)
                    win = {"task_begin": a, "task_end": e}
            try:
                b.job = pg.submit(self.g, b.plans, ws, self.streams[b.slot], mode=mode, grid_waves=b.grid,
                                  time_limit_ms=self.time_limit_ms, **win)
            except pg.PGError as e:
                self._release(b)
                for r in b.requests:
                    r.error, r.done = str(e), time.perf_counter()
                    self.finished.append(r)
                progress += len(b.requests)
                continue
            for r in b.requests:
                r.admitted = b.t_submit
                r.launch = self.launches
            b.lid = self.launches
            self.inflight.append(b)
            self.launches += 1
            self.merged_requests += len(b.requests) - 1
            progress += len(b.requests)
        progress += self._resume()
        return progress

    def _advance(self, b) -> int:
        """A windowed launch finished one window: fold its counts in and give
        back the extra slots until the next window starts (_resume)."""
        try:
            res, st = b.job.finish()
        except self.pg.PGError as e:
            b.windows = []
            b.acc = None
            b.job = _Failed(str(e))
            return self._retire(b)
        b.acc = [x + y for x, y in zip(b.acc, res)]
        b.kernel_ms += st["kernel_ms"]
        self.windows_run += 1
        b.job = None
        b.waiting = True
        self.free_slots.extend(b.extra_slots)
        b.extra_slots = []
        return 1

    def _resume(self) -> int:
        """Start the next window of every waiting windowed launch, on its own
        slot plus the free slots up to its width (fewer while light launches
        hold them)."""
        started = 0
        for b in self.inflight:
            if not b.waiting:
                continue
            while self.free_slots and len(b.extra_slots) < self.heavy_width - 1:
                b.extra_slots.append(self.free_slots.pop())
            grid = self.grid * (1 + len(b.extra_slots))
            a, e = b.windows.pop(0)
            ws = self.mem[b.offset:b.offset + b.nbytes]
            try:
                b.job = self.pg.submit(self.g, b.plans, ws, self.streams[b.slot], mode=self.pg.PG_JOB_COUNT,
                                       grid_waves=min(grid, b.grid), time_limit_ms=self.time_limit_ms,
                                       task_begin=a, task_end=e)
            except self.pg.PGError as err:
                b.windows = []
                b.job = _Failed(str(err))
            b.waiting = False
            started += 1
        return started

    def _release(self, b):
        self.pool.free(b.offset)
        self.free_slots.append(b.slot)
        self.free_slots.extend(b.extra_slots)
        b.extra_slots = []

    def _retire(self, b) -> int:
        err, st = None, {}
        try:
            res, st = b.job.finish()
            if b.acc is not None:
                res = [x + y for x, y in zip(b.acc, res)]
                st = dict(st, kernel_ms=b.kernel_ms + st["kernel_ms"])
            self.policy.observe(b.plans, st["kernel_ms"])
        except self.pg.PGError as e:
            err, res = str(e), None
        t = time.perf_counter()
        self.log.append({"launch": b.lid, "slot": b.slot, "grid": b.grid, "kind": b.kind, "heavy": b.heavy,
                         "queries": sorted({r.query.name for r in b.requests}), "requests": len(b.requests),
                         "t_submit": b.t_submit, "t_done": t, "kernel_ms": st.get("kernel_ms"), "error": err})
        self.inflight.remove(b)
        self._release(b)
        for r, ix in zip(b.requests, b.index):
            r.done = t
            if err is not None:
                r.error = err
            elif b.kind == "exists":
                r.result = res
            else:
                r.result = [res[i] for i in ix]
            self.finished.append(r)
        return len(b.requests)

    def drain(self, poll_s: float = 1e-4):
        while not self.idle():
            if not self.pump():
                time.sleep(poll_s)


# -------------------------------------------------------------- workloads

def catalogue_specs(pt):
    """The query catalogue as plain specs: (name, kind, pattern specs).
    Counts of 3-5 vertices, k-clique existence with early exit (Sec. 3.2.2),
    and patterns with anti-edges (Sec. 3.1.1)."""
    ent = [("triangle", "count", [pt.clique(3)]), ("wedge", "count", [pt.star(3)]),
           ("induced_wedge", "count", [pt.star(3, induced=True)])]
    for i, s in enumerate(pt.all_vertex_induced(4)):
        ent.append((f"induced4_{i}", "count", [s]))
    ent += [("clique4", "count", [pt.clique(4)]), ("clique5", "count", [pt.clique(5)])]
    ent += [(f"clique{k}_exists", "exists", [pt.clique(k)]) for k in (6, 8, 10, 12, 14)]
    ent += [("induced_diamond", "count", [pt.P8_INDUCED_DIAMOND]),
            ("two_common_friends", "count", [pt.PA_TWO_COMMON_FRIENDS])]
    trees5 = [s for s in pt.all_edge_induced(4) if s["k"] == 5]
    ent += [(f"tree5_{i}", "count", [s]) for i, s in enumerate(trees5)]
    # 5-vertex patterns whose core is one edge: every other vertex is
    # counted from the sizes of that edge's rows
    ent += [(name, "count", [spec]) for name, spec in pt.EDGE_CORE_5.items()]
    return ent


# The catalogue's count queries that finish alone on the serving graph (R-MAT
# 2^22 vertices, 2^26 edges) and fit in 64 bits: the benchmark's batch.
SERVING_BATCH = ["triangle", "wedge", "induced_wedge", "clique4", "book3", "cricket"]


def catalogue(pg, pt):
    """The query catalogue: (name, kind, plans), one plan per typed pattern:
    entries that ask the same question (K4 and the induced K4) share a plan,
    so their requests merge in a launch."""
    plans = {}

    def plan(spec):
        key = pattern_key(spec)
        if key not in plans:
            plans[key] = pg.plan_pattern(spec)
        return plans[key]
    return [Query(name, kind, [plan(s) for s in specs], list(specs)) for name, kind, specs in catalogue_specs(pt)]


def pattern_key(spec) -> str:
    """The typed pattern a spec describes, written out: vertex count, true
    edges, anti-edges (an induced spec's implied ones included), anti-vertex
    neighbourhoods and labels.  Equal keys mean equal patterns."""
    k = int(spec["k"])
    edges = sorted(tuple(sorted(e)) for e in spec.get("edges", []))
    anti = {tuple(sorted(e)) for e in spec.get("anti") or []}
    if spec.get("induced"):
        es = set(edges)
        anti |= {(a, b) for a in range(k) for b in range(a + 1, k) if (a, b) not in es}
    body = {"k": k, "edges": edges, "anti": sorted(anti), "av": [sorted(a) for a in spec.get("av") or []],
            "labels": list(spec.get("labels") or []), "av_labels": list(spec.get("av_labels") or [])}
    return json.dumps(body, sort_keys=True)


def poisson_arrivals(lam: float, n: int, n_queries: int, seed: int):
    """Seeded open-loop arrivals: (times in s from the start, catalogue indices)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / lam, n))
    pick = rng.integers(0, n_queries, n)
    return t, pick


def run_open_loop(server: Server, queries, times, picks, progress=None):
    """Offer request i at times[i] (seconds after the start) and serve until
    all are finished.  Latency is measured from the scheduled arrival."""
    n = len(times)
    t0 = time.perf_counter()
    reqs, i = [], 0
    start = len(server.finished)
    next_report, last_done, last_print = 200, 0, t0
    while i < n or not server.idle():
        now = time.perf_counter() - t0
        while i < n and times[i] <= now:
            r = Request(i, queries[picks[i]], t0 + times[i])
            server.offer(r)
            reqs.append(r)
            i += 1
        moved = server.pump()
        done = len(server.finished) - start
        if progress and done > last_done and (done >= next_report or time.perf_counter() - last_print > 20):
            progress(done, n)
            next_report = done + 200
            last_print = time.perf_counter()
        last_done = done
        if not moved:
            wait = 1e-4 if i >= n else min(1e-4, max(0.0, times[i] - (time.perf_counter() - t0)))
            time.sleep(wait)
    return reqs, t0


def summarize(reqs, t0):
    ok = [r for r in reqs if r.error is None]
    lat = sorted(1e3 * (r.done - r.arrival) for r in ok)

    def pct(p):
        if not lat:
            return None
        return lat[min(len(lat) - 1, max(0, math.ceil(p / 100 * len(lat)) - 1))]

    end = max((r.done for r in reqs), default=t0)
    span = max(1e-9, end - t0)
    matches = sum(sum(r.result) for r in ok if r.query.kind == "count")
    per_query = {}
    for name in sorted({r.query.name for r in ok}):
        ls = sorted(1e3 * (r.done - r.arrival) for r in ok if r.query.name == name)
        per_query[name] = {"n": len(ls), "p50_ms": ls[(len(ls) - 1) // 2],
                           "p99_ms": ls[min(len(ls) - 1, max(0, math.ceil(0.99 * len(ls)) - 1))]}
    return {"requests": len(reqs), "completed": len(ok), "errors": len(reqs) - len(ok),
            "p50_ms": pct(50), "p99_ms": pct(99), "mean_ms": sum(lat) / len(lat) if lat else None,
            "completed_qps": len(ok) / span, "matches_per_s": matches / span, "span_s": span,
            "per_query": per_query}


def standalone(graph, queries, pool_bytes: int, limit_ms: int, progress=None):
    """Each query alone on the whole GPU (one slot), with a time limit.
    Returns {name: (result or None, latency ms, error)}."""
    out = {}
    srv = Server(graph, pool_bytes, slots=1, time_limit_ms=limit_ms)
    for q in queries:
        r = Request(0, q, time.perf_counter())
        srv.offer(r)
        srv.drain()
        out[q.name] = (r.result, 1e3 * (r.done - r.arrival), r.error)
        if progress:
            progress(q.name, *out[q.name])
    return out


def policy_from(queries, alone, slots: int, **kw) -> Policy:
    """Estimates from standalone latencies: a launch at 1/slots of the grid
    is taken to last slots times as long."""
    pol = Policy(**kw)
    for q in queries:
        res, ms, err = alone[q.name]
        if len(q.plans) == 1 and err is None:
            pol.est[id(q.plans[0])] = ms * slots
    return pol


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="rmat22_64m")
    ap.add_argument("--qps", default="50,100,200,500")
    ap.add_argument("--queries", type=int, default=2000)
    ap.add_argument("--slots", type=int, default=0, help="concurrent launches (0 = hardware queues - 1)")
    ap.add_argument("--pool-mib", type=int, default=4096)
    ap.add_argument("--limit-ms", type=int, default=10000, help="standalone latency cut-off")
    ap.add_argument("--mix-limit-ms", type=int, default=120000, help="time limit of one launch in the mix")
    ap.add_argument("--light-ms", type=float, default=100.0, help="heavy/light cut (ms at a slot's grid)")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--window-ms", type=float, default=0.0,
                    help="cut heavy launches into root-task windows of about this many ms (0 = whole launches)")
    ap.add_argument("--trace", default="", help="write per-launch and per-request records to TRACE.<qps>.json")
    args = ap.parse_args(argv)

    import torch
    from . import graphgen as gg
    from . import patterns as pt
    from . import pg

    def say(*a):
        print("[serve]", *a, file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "serving needs a GPU"
    t = time.perf_counter()
    edges = gg.workload(args.workload)
    say(f"generated {args.workload} in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    G = pg.load_graph(*edges, device=0)
    del edges
    say(f"ingested n={G.n} m={G.m} d_max={G.d_max} in {time.perf_counter() - t:.1f} s")
    queries = catalogue(pg, pt)
    pool = args.pool_mib << 20
    alone = standalone(G, queries, pool, args.limit_ms,
                       progress=lambda name, res, ms, err: say(f"alone {name}: {ms:.1f} ms "
                                                               f"{'error ' + err if err else res}"))
    keep = [q for q in queries if alone[q.name][2] is None]
    excluded = [q.name for q in queries if q not in keep]
    slots = args.slots or default_slots()
    head = {"workload": args.workload, "n": G.n, "m": G.m, "d_max": G.d_max, "slots": slots,
            "pool_bytes": pool, "limit_ms": args.limit_ms,
            "alone_ms": {k: v[1] for k, v in alone.items()}, "excluded": excluded}
    print(json.dumps({"catalogue": head}), flush=True)
    for lam in [float(x) for x in args.qps.split(",")]:
        srv = Server(G, pool, slots=slots, time_limit_ms=args.mix_limit_ms,
                     policy=policy_from(keep, alone, slots, light_ms=args.light_ms), window_ms=args.window_ms)
        times, picks = poisson_arrivals(lam, args.queries, len(keep), args.seed)
        say(f"lambda {lam:g}: {args.queries} queries over {times[-1]:.1f} s")
        reqs, t0 = run_open_loop(srv, keep, times, picks,
                                 progress=lambda d, n: say(f"  {d}/{n} done"))
        summ = summarize(reqs, t0)
        mism = sum(1 for r in reqs if r.error is None and r.result != alone[r.query.name][0])
        summ.update({"qps_offered": lam, "launches": srv.launches, "merged_requests": srv.merged_requests,
                     "mismatches_vs_alone": mism, "window_ms": args.window_ms, "windows_run": srv.windows_run})
        per = collections.defaultdict(list)
        for r in reqs:
            if r.error is None:
                per[r.query.name].append(1e3 * (r.done - r.arrival))
        summ["p50_ms_by_query"] = {k: sorted(v)[len(v) // 2] for k, v in sorted(per.items())}
        print(json.dumps(summ), flush=True)
        if args.trace:
            with open(f"{args.trace}.{lam:g}.json", "w") as f:
                json.dump({"t0": t0, "launches": srv.log,
                           "requests": [{"name": r.query.name, "arrival": r.arrival, "admitted": r.admitted,
                                         "done": r.done, "launch": r.launch, "error": r.error} for r in reqs]}, f)
        del srv
    return 0


if __name__ == "__main__":
    sys.exit(main())
