"""Python binding of libpg (ctypes).  Argument marshalling only: every step
of matching runs in the library (host plan compiler + HIP kernels).  The
binding raises if the built library is missing; there is no fallback.

Pattern specs are plain dicts::

    {"k": 4, "edges": [(0, 1), ...], "anti": [(u, v), ...],
     "av": [[u, ...], ...],            # regular neighbours of each anti-vertex
     "labels": [...] | None, "av_labels": [...] | None, "induced": bool}
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pg.h")

PG_OK, PG_STOPPED = 0, 1
PG_EINVAL, PG_ENOMEM, PG_EDEVICE, PG_EOVERFLOW, PG_EUNSUPPORTED, PG_ETIMEDOUT = -1, -2, -3, -4, -5, -6
PG_EDGE, PG_ANTI_EDGE = 0, 1
PG_PLAN_AUTO, PG_PLAN_LINEAR_EXT, PG_PLAN_PARTIAL_ORDER = 0, 1, 2
PG_RUN_COUNT_BYTES, PG_RUN_NO_MODE_B, PG_RUN_NO_TASK_BATCH, PG_RUN_LIGHT_KERNEL, PG_RUN_NO_SHARE = 1, 2, 4, 8, 16
PG_RUN_WAVE_TIMES = 32
PG_JOB_COUNT, PG_JOB_EXISTS = 0, 1

_STATUS = {PG_EINVAL: "EINVAL", PG_ENOMEM: "ENOMEM", PG_EDEVICE: "EDEVICE", PG_EOVERFLOW: "EOVERFLOW",
           PG_EUNSUPPORTED: "EUNSUPPORTED", PG_ETIMEDOUT: "ETIMEDOUT"}


class PGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class pg_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("hub_min_degree", ctypes.c_int32), ("hub_budget_mib", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class pg_graph_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d_max", ctypes.c_int32), ("m", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("labelled", ctypes.c_int32), ("device", ctypes.c_int32),
                ("perm", ctypes.POINTER(ctypes.c_int32)), ("resident_waves", ctypes.c_int32 * 2),
                ("hub_count", ctypes.c_int32), ("hub_min_degree", ctypes.c_int32)]


class pg_edge(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int32), ("v", ctypes.c_int32), ("type", ctypes.c_int32)]


class pg_pattern_desc(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n_anti_vertices", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("induced", ctypes.c_int32), ("edges", ctypes.POINTER(pg_edge)),
                ("labels", ctypes.POINTER(ctypes.c_int16))]


class pg_plan_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("anchored", ctypes.c_int32), ("anchor", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class pg_plan_info_t(ctypes.Structure):
    _fields_ = [("aut", ctypes.c_uint64), ("k", ctypes.c_int32), ("core_size", ctypes.c_int32),
                ("core_mask", ctypes.c_uint32), ("n_matching_orders", ctypes.c_int32),
                ("n_programs", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("n_order", ctypes.c_int32),
                ("order", ctypes.c_int32 * 240), ("n_orbit_steps", ctypes.c_int32),
                ("orbit_size", ctypes.c_int32 * 16), ("orbit_vertex", ctypes.c_int32 * 16),
                ("mode_used", ctypes.c_int32), ("plan_ms", ctypes.c_double), ("anchor", ctypes.c_int32)]


class pg_run_config(ctypes.Structure):
    _fields_ = [("grid_waves", ctypes.c_int32), ("chunk", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("time_limit_ms", ctypes.c_int32), ("hub_min_degree", ctypes.c_int32),
                ("batch_max_avg", ctypes.c_int32), ("task_begin", ctypes.c_int32), ("task_end", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class pg_run_stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("logical_bytes", ctypes.c_uint64), ("root_tasks", ctypes.c_uint64),
                ("grid_waves", ctypes.c_int32), ("chunk", ctypes.c_int32), ("tasks_started", ctypes.c_uint64),
                ("wave_done_first_ms", ctypes.c_double), ("wave_done_last_ms", ctypes.c_double)]


MATCH_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p)

EXPORTS = ["pg_load_graph", "pg_graph_info", "pg_graph_csr", "pg_free_graph", "pg_plan_pattern",
           "pg_plan_pattern_ex", "pg_plan_info", "pg_free_plan", "pg_plan_programs", "pg_count", "pg_count_ex",
           "pg_count_noalloc", "pg_exists", "pg_enumerate", "pg_match", "pg_match_ex", "pg_root_tasks", "pg_launch_tasks", "pg_enumerate_range",
           "pg_domain_sizes", "pg_job_workspace_size", "pg_submit", "pg_job_poll", "pg_job_finish",
           "pg_last_error"]

_lib = None


def lib():
    """Load libpg.so (built by __graft_entry__.build() / build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    L.pg_load_graph.argtypes = [i32, i64, vp, vp, vp, ctypes.POINTER(pg_options), ctypes.POINTER(vp)]
    L.pg_graph_info.argtypes = [vp, ctypes.POINTER(pg_graph_info_t)]
    L.pg_graph_csr.argtypes = [vp, vp, vp]
    L.pg_free_graph.argtypes = [vp]
    L.pg_free_graph.restype = None
    L.pg_plan_pattern.argtypes = [ctypes.POINTER(pg_pattern_desc), ctypes.POINTER(vp)]
    L.pg_plan_pattern_ex.argtypes = [ctypes.POINTER(pg_pattern_desc), ctypes.POINTER(pg_plan_options),
                                     ctypes.POINTER(vp)]
    L.pg_plan_info.argtypes = [vp, ctypes.POINTER(pg_plan_info_t)]
    L.pg_free_plan.argtypes = [vp]
    L.pg_free_plan.restype = None
    L.pg_plan_programs.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64)]
    L.pg_count.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(u64), vp]
    L.pg_count_noalloc.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(u64), ctypes.POINTER(pg_run_config), vp]
    L.pg_count_ex.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(u64), ctypes.POINTER(pg_run_config),
                              ctypes.POINTER(pg_run_stats), vp]
    L.pg_exists.argtypes = [vp, vp, ctypes.POINTER(i32), vp]
    L.pg_enumerate.argtypes = [vp, vp, vp, u64, ctypes.POINTER(u64), vp]
    L.pg_match.argtypes = [vp, vp, MATCH_CB, vp, ctypes.POINTER(u64)]
    L.pg_match_ex.argtypes = [vp, vp, MATCH_CB, vp, ctypes.POINTER(u64), u64]
    L.pg_root_tasks.argtypes = [vp, vp, ctypes.POINTER(i64)]
    L.pg_launch_tasks.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(i64)]
    L.pg_enumerate_range.argtypes = [vp, vp, i64, i64, vp, u64, ctypes.POINTER(u64), vp]
    L.pg_domain_sizes.argtypes = [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(u64), ctypes.POINTER(pg_run_config), vp]
    L.pg_job_workspace_size.argtypes = [vp, ctypes.POINTER(vp), i32, i32, ctypes.POINTER(pg_run_config),
                                        ctypes.POINTER(u64)]
    L.pg_submit.argtypes = [vp, ctypes.POINTER(vp), i32, i32, ctypes.POINTER(pg_run_config), vp, u64, vp,
                            ctypes.POINTER(vp)]
    L.pg_job_poll.argtypes = [vp, ctypes.POINTER(i32)]
    L.pg_job_finish.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(pg_run_stats)]
    L.pg_last_error.argtypes = []
    L.pg_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("pg_free_graph", "pg_free_plan", "pg_last_error"):
            getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


def _check(st):
    if st < 0:
        raise PGError(st, lib().pg_last_error().decode())
    return st


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # a torch.cuda.Stream


# ------------------------------------------------------------------ graph

class Graph:
    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)
        info = pg_graph_info_t()
        _check(lib().pg_graph_info(self._h, ctypes.byref(info)))
        self.n, self.m, self.d_max = info.n, info.m, info.d_max
        self.device_bytes = info.device_bytes
        self.device = info.device
        self.perm = np.ctypeslib.as_array(info.perm, shape=(info.n,)).copy()
        self.resident_waves = (int(info.resident_waves[0]), int(info.resident_waves[1]))
        self.hub_count, self.hub_min_degree = int(info.hub_count), int(info.hub_min_degree)

    def csr(self):
        rp = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(max(1, 2 * self.m), dtype=np.int32)
        _check(lib().pg_graph_csr(self._h, rp.ctypes.data, col.ctypes.data))
        return rp, col[: 2 * self.m]

    def free(self):
        if self._h:
            lib().pg_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def load_graph(n, src, dst, labels=None, device: int = -1, hub_min_degree: int = 0, hub_budget_mib: int = 0) -> Graph:
    """Ingest and upload.  hub_min_degree: rows of at least this degree also
    get a dense bitmap (0 = library default, -1 = none)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int16)
    opt = pg_options(device=device, hub_min_degree=hub_min_degree, hub_budget_mib=hub_budget_mib)
    h = ctypes.c_void_p()
    _check(lib().pg_load_graph(int(n), len(src), src.ctypes.data, dst.ctypes.data,
                               None if lab is None else lab.ctypes.data, ctypes.byref(opt), ctypes.byref(h)))
    return Graph(h.value)


# ------------------------------------------------------------------ plans

def pattern_desc(spec):
    k = int(spec["k"])
    av = [list(x) for x in (spec.get("av") or [])]
    edges = [(int(u), int(v), PG_EDGE) for u, v in spec.get("edges", [])]
    edges += [(int(u), int(v), PG_ANTI_EDGE) for u, v in (spec.get("anti") or [])]
    for a, nb in enumerate(av):
        edges += [(k + a, int(u), PG_ANTI_EDGE) for u in nb]
    earr = (pg_edge * max(1, len(edges)))(*[pg_edge(u, v, t) for u, v, t in edges])
    labels = spec.get("labels")
    avl = spec.get("av_labels")
    lab = None
    if labels is not None or avl is not None:
        vals = list(labels) if labels is not None else [-1] * k
        vals += list(avl) if avl is not None else [-1] * len(av)
        lab = (ctypes.c_int16 * len(vals))(*vals)
    d = pg_pattern_desc(k=k, n_anti_vertices=len(av), n_edges=len(edges), induced=1 if spec.get("induced") else 0,
                        edges=earr, labels=lab)
    return d, (earr, lab)


class Plan:
    def __init__(self, handle, spec):
        self._h = ctypes.c_void_p(handle)
        self.spec = spec
        self.k = int(spec["k"])
        self.anchor = None

    def info(self) -> dict:
        i = pg_plan_info_t()
        _check(lib().pg_plan_info(self._h, ctypes.byref(i)))
        return {
            "aut": i.aut, "k": i.k, "core_size": i.core_size,
            "core": [u for u in range(i.k) if i.core_mask >> u & 1],
            "n_matching_orders": i.n_matching_orders, "n_programs": i.n_programs, "n_levels": i.n_levels,
            "order": [(i.order[2 * j], i.order[2 * j + 1]) for j in range(i.n_order)],
            "orbit_size": list(i.orbit_size[: i.n_orbit_steps]),
            "orbit_vertex": list(i.orbit_vertex[: i.n_orbit_steps]),
            "mode_used": i.mode_used, "plan_ms": i.plan_ms, "anchor": i.anchor,
        }

    def programs(self, enum_mode: bool = False) -> list[dict]:
        """The level programs the GPU runs (decoded pg_plan_programs)."""
        n = ctypes.c_int64()
        lib().pg_plan_programs(self._h, int(enum_mode), None, 0, ctypes.byref(n))
        buf = np.zeros(int(n.value), dtype=np.int32)
        _check(lib().pg_plan_programs(self._h, int(enum_mode), buf.ctypes.data, len(buf), ctypes.byref(n)))
        it = iter(buf.tolist())
        progs = []
        for _ in range(next(it)):
            nl = next(it)
            lo, hi = next(it) & 0xFFFFFFFF, next(it) & 0xFFFFFFFF
            def level():
                keys = ["isect", "diff", "lo", "hi", "excl", "t_isect", "t_diff"]
                L = {k: next(it) & 0xFFFFFFFF for k in keys}
                L.update(base=next(it), label=next(it), group=next(it), pv=next(it))
                avs = []
                for _ in range(next(it)):
                    nbr, lab = next(it) & 0xFFFFFFFF, next(it)
                    avs.append({"nbr": nbr, "label": lab, "xmask": [next(it) & 0xFFFFFFFF for _ in range(16)]})
                L["avs"] = avs
                return L
            levels = [level() for _ in range(nl)]
            factors = [level() for _ in range(next(it))]
            progs.append({"mult": lo | hi << 32, "levels": levels, "factors": factors})
        return progs

    def free(self):
        if self._h:
            lib().pg_free_plan(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def plan_pattern(spec, mode: int = PG_PLAN_AUTO, anchor: int | None = None) -> Plan:
    """Compile a pattern spec.  anchor: plan for the domain of that regular
    vertex (domain_sizes)."""
    d, keep = pattern_desc(spec)
    opt = pg_plan_options(mode=mode, anchored=0 if anchor is None else 1, anchor=0 if anchor is None else anchor)
    h = ctypes.c_void_p()
    _check(lib().pg_plan_pattern_ex(ctypes.byref(d), ctypes.byref(opt), ctypes.byref(h)))
    del keep
    p = Plan(h.value, spec)
    p.anchor = anchor
    return p


# --------------------------------------------------------------- counting

RUN_KNOBS = ("grid_waves", "chunk", "flags", "time_limit_ms", "hub_min_degree", "batch_max_avg", "task_begin",
             "task_end")


def run_config(**kw) -> pg_run_config:
    """pg_run_config from keyword knobs (RUN_KNOBS); 0 = library default."""
    bad = set(kw) - set(RUN_KNOBS)
    if bad:
        raise TypeError(f"unknown launch knobs {sorted(bad)}")
    return pg_run_config(**{k: int(v) for k, v in kw.items()})


def count_ex(graph: Graph, plans, stream=None, **knobs):
    """Counts and stats of one launch.  knobs: the fields of pg_run_config
    (RUN_KNOBS: grid, claim chunk, flags, time limit, bitmap degree
    threshold, leaf-batching limit, root-task window).  A run that reaches
    its time limit raises PGError with status PG_ETIMEDOUT (its partial
    counts and stats ride on the exception as .counts and .stats)."""
    plans = list(plans)
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    out = (ctypes.c_uint64 * len(plans))()
    cfg = run_config(**knobs)
    st = pg_run_stats()
    rc = lib().pg_count_ex(graph._h, arr, len(plans), out, ctypes.byref(cfg), ctypes.byref(st), _stream_ptr(stream))
    if rc < 0:
        err = PGError(rc, lib().pg_last_error().decode())
        # a run stopped by its time limit: the counts so far (lower bounds)
        # and how far it got
        err.counts = [int(x) for x in out]
        err.stats = _stats(st)
        raise err
    return [int(x) for x in out], _stats(st)


def count_noalloc(graph: Graph, plans, stream=None, **knobs):
    """pg_count_noalloc: counts with no device allocation (a fixed device
    array of the library holds the launch's memory)."""
    plans = list(plans)
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    out = (ctypes.c_uint64 * len(plans))()
    cfg = run_config(**knobs)
    _check(lib().pg_count_noalloc(graph._h, arr, len(plans), out, ctypes.byref(cfg), _stream_ptr(stream)))
    return [int(x) for x in out]


def _stats(st):
    return {"kernel_ms": st.kernel_ms, "total_ms": st.total_ms, "logical_bytes": st.logical_bytes,
            "root_tasks": st.root_tasks, "grid_waves": st.grid_waves, "chunk": st.chunk,
            "tasks_started": st.tasks_started, "wave_done_first_ms": st.wave_done_first_ms,
            "wave_done_last_ms": st.wave_done_last_ms}


def count(graph: Graph, plans, stream=None, **kw):
    single = isinstance(plans, Plan)
    res, _ = count_ex(graph, [plans] if single else plans, stream, **kw)
    return res[0] if single else res


def domain_sizes(graph: Graph, plans, stream=None, **knobs) -> list[int]:
    """|dom(anchor)| of each anchored plan (MNI domains), in one launch."""
    plans = list(plans)
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    sizes = (ctypes.c_uint64 * len(plans))()
    cfg = run_config(**knobs)
    _check(lib().pg_domain_sizes(graph._h, arr, len(plans), sizes, ctypes.byref(cfg), _stream_ptr(stream)))
    return [int(x) for x in sizes]


def exists(graph: Graph, plan: Plan, stream=None) -> bool:
    f = ctypes.c_int32()
    _check(lib().pg_exists(graph._h, plan._h, ctypes.byref(f), _stream_ptr(stream)))
    return bool(f.value)


def enumerate_matches(graph: Graph, plan: Plan, cap: int | None = None, stream=None):
    """All matches as an (n, k) int32 numpy array of original ids (device
    buffer from torch, copied back).  cap=None sizes it from a first pass."""
    import torch
    tot = ctypes.c_uint64()
    if cap is None:
        _check(lib().pg_enumerate(graph._h, plan._h, None, 0, ctypes.byref(tot), _stream_ptr(stream)))
        cap = int(tot.value)
    buf = torch.empty((max(1, cap), plan.k), dtype=torch.int32, device=f"cuda:{graph.device}")
    torch.cuda.synchronize(graph.device)
    _check(lib().pg_enumerate(graph._h, plan._h, ctypes.c_void_p(buf.data_ptr()), cap, ctypes.byref(tot),
                              _stream_ptr(stream)))
    n = min(cap, int(tot.value))
    return buf[:n].cpu().numpy(), int(tot.value)


def root_tasks(graph: Graph, plan: Plan) -> int:
    n = ctypes.c_int64()
    _check(lib().pg_root_tasks(graph._h, plan._h, ctypes.byref(n)))
    return int(n.value)


def launch_tasks(graph: Graph, plans) -> int:
    """Root tasks of one counting launch of these plans (pg_launch_tasks)."""
    plans = list(plans)
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    n = ctypes.c_int64()
    _check(lib().pg_launch_tasks(graph._h, arr, len(plans), ctypes.byref(n)))
    return int(n.value)


def enumerate_range(graph: Graph, plan: Plan, task_begin: int, task_end: int, cap: int, stream=None):
    """Matches found from root tasks [task_begin, task_end): (rows, total);
    rows holds min(cap, total) of them."""
    import torch
    tot = ctypes.c_uint64()
    buf = torch.empty((max(1, cap), plan.k), dtype=torch.int32, device=f"cuda:{graph.device}")
    torch.cuda.synchronize(graph.device)
    _check(lib().pg_enumerate_range(graph._h, plan._h, int(task_begin), int(task_end),
                                    ctypes.c_void_p(buf.data_ptr()), cap, ctypes.byref(tot), _stream_ptr(stream)))
    n = min(cap, int(tot.value))
    return buf[:n].cpu().numpy(), int(tot.value)


def match(graph: Graph, plan: Plan, fn, buffer_rows: int = 0) -> tuple[int, bool]:
    """Calls fn(ids: tuple) per match; a truthy return stops.  Returns
    (callbacks made, stopped).  buffer_rows: device buffer (0 = default)."""
    def cb(ids, k, user):
        return 1 if fn(tuple(ids[i] for i in range(k))) else 0
    c = MATCH_CB(cb)
    n = ctypes.c_uint64()
    st = _check(lib().pg_match_ex(graph._h, plan._h, c, None, ctypes.byref(n), int(buffer_rows)))
    return int(n.value), st == PG_STOPPED


# ------------------------------------------------------- asynchronous jobs

def job_workspace_size(graph: Graph, plans, mode=PG_JOB_COUNT, **knobs) -> int:
    plans = list(plans)
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    cfg = run_config(**knobs)
    b = ctypes.c_uint64()
    _check(lib().pg_job_workspace_size(graph._h, arr, len(plans), mode, ctypes.byref(cfg), ctypes.byref(b)))
    return int(b.value)


class Job:
    """One launch in flight (pg_submit).  Keeps its plans and workspace alive
    until finish()."""

    def __init__(self, handle, plans, workspace, mode):
        self._h = ctypes.c_void_p(handle)
        self.plans = plans
        self.workspace = workspace
        self.mode = mode

    def done(self) -> bool:
        d = ctypes.c_int32()
        _check(lib().pg_job_poll(self._h, ctypes.byref(d)))
        return bool(d.value)

    def finish(self):
        """Counts (list) or, for an existence job, a bool; plus stats."""
        if self._h is None:
            raise PGError(PG_EINVAL, "job already finished")
        out = (ctypes.c_uint64 * len(self.plans))()
        st = pg_run_stats()
        h, self._h = self._h, None
        _check(lib().pg_job_finish(h, out, ctypes.byref(st)))
        self.workspace = None
        res = [int(x) for x in out]
        return (bool(res[0]) if self.mode == PG_JOB_EXISTS else res), _stats(st)


def submit(graph: Graph, plans, workspace, stream, mode=PG_JOB_COUNT, **knobs) -> Job:
    """Enqueue one launch on `stream` (a torch.cuda.Stream or raw handle).
    `workspace` is a device uint8 torch tensor of at least
    job_workspace_size() bytes with a 256-byte aligned data pointer."""
    plans = list(plans)
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    cfg = run_config(**knobs)
    h = ctypes.c_void_p()
    _check(lib().pg_submit(graph._h, arr, len(plans), mode, ctypes.byref(cfg),
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                           _stream_ptr(stream), ctypes.byref(h)))
    return Job(h.value, plans, workspace, mode)
