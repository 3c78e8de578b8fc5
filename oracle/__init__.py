"""CPU oracle for pattern-aware subgraph counting.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It
shares no code with the HIP library and never imports it.

Routes (each cites the passage it follows):

* :func:`count` -- the count as a definition: valid maps / |Aut_t|
  (problem statement Sec. 2.1; anti-edges Sec. 3.1.1; anti-vertices Sec. 3.1.2;
  vertex-induced via anti-edges, Theorem in Sec. 3.1.3).  Plain C, threaded over
  the first pattern vertex (``oracle.c``).
* :func:`motif_census` -- ESU enumeration of connected k-vertex sets
  classified by their induced subgraph (motif counting, Sec. 2.1).
* :func:`induced4_closed_form` -- non-induced 4-vertex counts from textbook
  closed forms, turned into vertex-induced counts by inverting the
  "spanning copies of P inside Q" matrix, whose coefficients are computed
  here by brute force over edge subsets.
* :mod:`oracle.brute` -- exhaustive checks on tiny graphs (all injective
  maps / all k-subsets); the oracle of the oracle.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SANITIZE=1 builds and loads liboracle_san.so instead, with
# AddressSanitizer and UndefinedBehaviorSanitizer (the process must then have
# libasan preloaded; tests/test_sanitizers.py runs the oracle's tests so).
_SAN = os.environ.get("ORACLE_SANITIZE", "") == "1"
_SO = os.path.join(_HERE, "liboracle_san.so" if _SAN else "liboracle.so")
_FLAGS = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined"] if _SAN else ["-O2"])


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, no GPU code)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_FLAGS, "-Wall", "-shared", "-fPIC", "-pthread", src, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


class _Pattern(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32), ("n_av", ctypes.c_int32),
        ("edge", ctypes.c_uint32 * 16), ("anti", ctypes.c_uint32 * 16),
        ("av", ctypes.c_uint32 * 4), ("label", ctypes.c_int16 * 16),
        ("av_label", ctypes.c_int16 * 4),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        vp, i32, i64, u64p = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)
        lib.orc_graph_build.restype = vp
        lib.orc_graph_build.argtypes = [i32, i64, vp, vp, vp]
        lib.orc_graph_free.argtypes = [vp]
        lib.orc_graph_m.restype = i64
        lib.orc_graph_m.argtypes = [vp]
        lib.orc_graph_degrees.argtypes = [vp, vp]
        lib.orc_graph_csr.argtypes = [vp, vp, vp]
        lib.orc_aut.restype = ctypes.c_uint64
        lib.orc_aut.argtypes = [ctypes.POINTER(_Pattern)]
        lib.orc_count.restype = ctypes.c_int
        lib.orc_count.argtypes = [vp, ctypes.POINTER(_Pattern), ctypes.c_int, u64p, u64p, u64p]
        lib.orc_valid_maps.restype = ctypes.c_int
        lib.orc_valid_maps.argtypes = [vp, ctypes.POINTER(_Pattern), ctypes.c_int, u64p, u64p]
        lib.orc_valid_maps_roots.restype = ctypes.c_int
        lib.orc_valid_maps_roots.argtypes = [vp, ctypes.POINTER(_Pattern), ctypes.c_int, vp, i64, u64p, u64p]
        lib.orc_esu_census.restype = ctypes.c_int
        lib.orc_esu_census.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp]
        lib.orc_noninduced4.restype = ctypes.c_int
        lib.orc_noninduced4.argtypes = [vp, ctypes.c_int, vp, vp]
        lib.orc_triangles_per_vertex.argtypes = [vp, vp]
        lib.orc_edge_triangles.argtypes = [vp, ctypes.c_int, vp]
        lib.orc_exists.restype = ctypes.c_int
        lib.orc_exists.argtypes = [vp, ctypes.POINTER(_Pattern), ctypes.c_int]
        lib.orc_domains.restype = ctypes.c_int
        lib.orc_domains.argtypes = [vp, ctypes.POINTER(_Pattern), ctypes.c_int, vp, vp]
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


class Graph:
    """The oracle's own canonical adjacency (loops dropped, duplicates
    collapsed, symmetrised, rows sorted)."""

    def __init__(self, n, src, dst, labels=None):
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        self._keep = (src, dst)
        lab = None
        if labels is not None:
            lab = np.ascontiguousarray(labels, dtype=np.int16)
            self._keep = (src, dst, lab)
        self.n = int(n)
        self.labels = lab
        self._h = _L().orc_graph_build(self.n, len(src), src.ctypes.data, dst.ctypes.data,
                                       lab.ctypes.data if lab is not None else None)
        self.m = int(_L().orc_graph_m(self._h))

    @classmethod
    def from_tuple(cls, g, labels=None):
        n, u, v = g
        return cls(n, u, v, labels)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_graph_free(self._h)
            self._h = None

    def degrees(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int64)
        _L().orc_graph_degrees(self._h, out.ctypes.data)
        return out

    def csr(self):
        off = np.zeros(self.n + 1, dtype=np.int64)
        _L().orc_graph_degrees(self._h, off[1:].ctypes.data)
        off = np.cumsum(off)
        adj = np.zeros(max(1, int(off[-1])), dtype=np.int32)
        off2 = np.zeros(self.n + 1, dtype=np.int64)
        _L().orc_graph_csr(self._h, off2.ctypes.data, adj.ctypes.data)
        return off2, adj[: int(off2[-1])]

    def triangles_per_vertex(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int64)
        _L().orc_triangles_per_vertex(self._h, out.ctypes.data)
        return out


# ------------------------------------------------------------------ patterns
#
# A pattern spec is plain data:
#   {"k": int, "edges": [(u, v), ...], "anti": [(u, v), ...],
#    "av": [[u, ...], ...],          # regular neighbours of each anti-vertex
#    "labels": [int | -1, ...] | None, "av_labels": [...] | None,
#    "induced": bool}

def _to_struct(spec) -> _Pattern:
    k = int(spec["k"])
    if not 1 <= k <= 16:
        raise ValueError("k out of range")
    p = _Pattern()
    p.k = k
    av = list(spec.get("av", []) or [])
    if len(av) > 4:
        raise ValueError("too many anti-vertices")
    p.n_av = len(av)
    edge = [0] * 16
    anti = [0] * 16
    for u, v in spec.get("edges", []):
        edge[u] |= 1 << v
        edge[v] |= 1 << u
    for u, v in spec.get("anti", []) or []:
        anti[u] |= 1 << v
        anti[v] |= 1 << u
    if spec.get("induced"):
        for u in range(k):
            for v in range(k):
                if u != v and not (edge[u] >> v & 1):
                    anti[u] |= 1 << v
    for i in range(16):
        p.edge[i] = edge[i]
        p.anti[i] = anti[i]
    for a, nb in enumerate(av):
        msk = 0
        for u in nb:
            msk |= 1 << u
        p.av[a] = msk
    labels = spec.get("labels")
    for i in range(16):
        p.label[i] = -1 if labels is None or i >= k else int(labels[i])
    avl = spec.get("av_labels")
    for a in range(4):
        p.av_label[a] = -1 if avl is None or a >= len(av) else int(avl[a])
    return p


def aut(spec) -> int:
    a = int(_L().orc_aut(ctypes.byref(_to_struct(spec))))
    if a == 0:
        raise ValueError("automorphism search out of range for this pattern")
    return a


def valid_maps(g: Graph, spec, threads: int | None = None) -> int:
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    rc = _L().orc_valid_maps(g._h, ctypes.byref(_to_struct(spec)), threads or default_threads(),
                             ctypes.byref(lo), ctypes.byref(hi))
    if rc:
        raise ValueError("pattern is not connected by true edges")
    return (hi.value << 64) | lo.value


def valid_maps_from(g: Graph, spec, roots, threads: int | None = None) -> int:
    """Valid maps whose pattern vertex 0 is mapped into ``roots``."""
    r = np.ascontiguousarray(roots, dtype=np.int32)
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    rc = _L().orc_valid_maps_roots(g._h, ctypes.byref(_to_struct(spec)), threads or default_threads(),
                                   r.ctypes.data, len(r), ctypes.byref(lo), ctypes.byref(hi))
    if rc:
        raise ValueError("pattern is not connected by true edges")
    return (hi.value << 64) | lo.value


def count(g: Graph, spec, threads: int | None = None) -> int:
    """Number of matches of the pattern: |valid maps| / |Aut_t|."""
    lo, hi, a = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = _L().orc_count(g._h, ctypes.byref(_to_struct(spec)), threads or default_threads(),
                        ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(a))
    if rc == -1:
        raise ValueError("pattern is not connected by true edges")
    if rc == -2:
        raise ValueError("automorphism search out of range for this pattern")
    if rc == -3:
        raise AssertionError("valid-map count not divisible by |Aut|")
    return (hi.value << 64) | lo.value


def exists(g: Graph, spec, threads: int | None = None) -> bool:
    """Whether the pattern has at least one match (Sec. 3.2.2): a search for
    one valid map, stopped at the first found."""
    rc = _L().orc_exists(g._h, ctypes.byref(_to_struct(spec)), threads or default_threads())
    if rc < 0:
        raise ValueError("pattern is not connected by true edges")
    return rc == 1


def domains(g: Graph, spec, threads: int | None = None, members: bool = False):
    """MNI domains (Sec. 2): sizes[u] = |{m(u) : m a valid map}| for each
    regular vertex u; with members=True also a (k, n) 0/1 array."""
    k = int(spec["k"])
    sizes = np.zeros(k, dtype=np.int64)
    mem = np.zeros((k, g.n), dtype=np.uint8) if members else None
    rc = _L().orc_domains(g._h, ctypes.byref(_to_struct(spec)), threads or default_threads(), sizes.ctypes.data,
                          mem.ctypes.data if members else None)
    if rc == -1:
        raise ValueError("pattern is not connected by true edges")
    if rc:
        raise MemoryError("orc_domains")
    return (sizes.tolist(), mem) if members else sizes.tolist()


def mni_support(g: Graph, spec, threads: int | None = None) -> int:
    """Minimum node image support: the smallest domain."""
    return min(domains(g, spec, threads))


# ------------------------------------------------------------ motif classes

def _pair_index(k):
    return {p: i for i, p in enumerate(itertools.combinations(range(k), 2))}


@lru_cache(maxsize=None)
def canon_table(k: int) -> np.ndarray:
    """adjacency bitmask (pairs in lexicographic order) -> the smallest
    bitmask among all relabellings of the k vertices."""
    pidx = _pair_index(k)
    pairs = list(pidx)
    nb = len(pairs)
    perms = list(itertools.permutations(range(k)))
    # where each pair goes under each permutation
    moves = []
    for pm in perms:
        moves.append([pidx[tuple(sorted((pm[a], pm[b])))] for a, b in pairs])
    table = np.zeros(1 << nb, dtype=np.uint16)
    for mask in range(1 << nb):
        bits = [i for i in range(nb) if mask >> i & 1]
        best = mask
        for mv in moves:
            r = 0
            for i in bits:
                r |= 1 << mv[i]
            if r < best:
                best = r
        table[mask] = best
    return table


def _connected(k, mask) -> bool:
    pairs = list(itertools.combinations(range(k), 2))
    adj = {i: set() for i in range(k)}
    for i, (a, b) in enumerate(pairs):
        if mask >> i & 1:
            adj[a].add(b)
            adj[b].add(a)
    seen, stack = {0}, [0]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == k


@lru_cache(maxsize=None)
def motif_classes(k: int):
    """Canonical bitmasks of the connected k-vertex graphs, ascending by
    (edge count, bitmask)."""
    t = canon_table(k)
    reps = sorted({int(t[m]) for m in range(len(t)) if _connected(k, m)},
                  key=lambda r: (bin(r).count("1"), r))
    return reps


def class_edges(k: int, rep: int):
    pairs = list(itertools.combinations(range(k), 2))
    return [pairs[i] for i in range(len(pairs)) if rep >> i & 1]


def motif_census(g: Graph, k: int, threads: int | None = None) -> dict[int, int]:
    """Vertex-induced counts of every connected k-vertex motif, keyed by the
    canonical bitmask (ESU enumeration; every connected k-set visited once)."""
    t = canon_table(k)
    counts = np.zeros(len(t), dtype=np.uint64)
    rc = _L().orc_esu_census(g._h, k, t.ctypes.data, threads or default_threads(), counts.ctypes.data)
    if rc:
        raise ValueError("k out of range")
    return {rep: int(counts[rep]) for rep in motif_classes(k)}


def canonical_of_edges(k: int, edges) -> int:
    pidx = _pair_index(k)
    mask = 0
    for a, b in edges:
        mask |= 1 << pidx[tuple(sorted((a, b)))]
    return int(canon_table(k)[mask])


# ------------------------------------------------------ closed-form route

@lru_cache(maxsize=None)
def spanning_copies(k: int) -> dict[tuple[int, int], int]:
    """c(P, Q): number of edge subsets of the labelled graph Q (a class
    representative) whose spanning subgraph is isomorphic to P.  Brute force
    over all edge subsets of Q."""
    t = canon_table(k)
    reps = motif_classes(k)
    out = {}
    for q in reps:
        qbits = [i for i in range(16) if q >> i & 1]
        for sel in range(1 << len(qbits)):
            sub = 0
            for j, b in enumerate(qbits):
                if sel >> j & 1:
                    sub |= 1 << b
            c = int(t[sub])
            if c in reps:
                out[(c, q)] = out.get((c, q), 0) + 1
    return out


def invert_noninduced(k: int, noninduced: dict[int, int]) -> dict[int, int]:
    """Solve N_P = sum_Q c(P,Q) I_Q for the vertex-induced counts I, densest
    first (the system is triangular: c(P,Q) = 0 unless P has no more edges)."""
    c = spanning_copies(k)
    reps = motif_classes(k)
    induced = {}
    for q in sorted(reps, key=lambda r: -bin(r).count("1")):
        rest = sum(c.get((q, r), 0) * induced[r] for r in induced if r != q)
        val = noninduced[q] - rest
        assert c[(q, q)] == 1 and val >= 0
        induced[q] = val
    return induced


def noninduced4(g: Graph, threads: int | None = None) -> dict[str, int]:
    lo = np.zeros(6, dtype=np.uint64)
    hi = np.zeros(6, dtype=np.uint64)
    _L().orc_noninduced4(g._h, threads or default_threads(), lo.ctypes.data, hi.ctypes.data)
    vals = [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]
    return dict(zip(["triangle", "star", "path", "cycle", "paw", "diamond"], vals))


FOUR_NAMES = {
    "star": [(0, 1), (0, 2), (0, 3)],
    "path": [(0, 1), (1, 2), (2, 3)],
    "cycle": [(0, 1), (1, 2), (2, 3), (3, 0)],
    "paw": [(0, 1), (1, 2), (2, 0), (0, 3)],
    "diamond": [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)],
    "clique": [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
}


def induced4_closed_form(g: Graph, threads: int | None = None) -> dict[str, int]:
    """Vertex-induced counts of the six connected 4-vertex motifs: closed
    forms for the non-induced counts (K4 from the generic matcher), then the
    exact triangular inversion."""
    nc = noninduced4(g, threads)
    nc["clique"] = count(g, {"k": 4, "edges": FOUR_NAMES["clique"]}, threads)
    by_rep = {canonical_of_edges(4, FOUR_NAMES[name]): nc[name] for name in FOUR_NAMES}
    ind = invert_noninduced(4, by_rep)
    return {name: ind[canonical_of_edges(4, FOUR_NAMES[name])] for name in FOUR_NAMES}


def degree_choose_sum(g: Graph, j: int) -> int:
    """sum_v C(d_v, j), exact."""
    d = g.degrees()
    vals, cnt = np.unique(d, return_counts=True)
    return sum(math.comb(int(x), j) * int(c) for x, c in zip(vals, cnt))


def star_row_invariant(k: int, induced_counts: dict[int, int]) -> int:
    """sum_Q c(K_{1,k-1}, Q) I_Q: equals the number of non-induced (k-1)-leaf
    stars, i.e. sum_v C(d_v, k-1)."""
    c = spanning_copies(k)
    star = canonical_of_edges(k, [(0, i) for i in range(1, k)])
    return sum(c.get((star, q), 0) * induced_counts[q] for q in induced_counts)


# ------------------------------------------- 5-vertex non-induced closed forms
#
# Counts of (not necessarily induced) subgraphs of a few 5-vertex shapes,
# each from degrees and per-edge triangle counts.  With the spanning-copy
# coefficients c(P, Q) they give exact linear checks on a vertex-induced
# 5-motif census: N(P) = sum_Q c(P, Q) I(Q) (Sec. 3.1.3 relates the two
# kinds of matches).  Shapes as edge lists:
FIVE_NONINDUCED = {
    "star4": [(0, 1), (0, 2), (0, 3), (0, 4)],
    "fork": [(0, 1), (0, 2), (0, 3), (1, 4)],
    "cricket": [(0, 1), (0, 2), (1, 2), (0, 3), (0, 4)],
    "bull": [(0, 1), (0, 2), (1, 2), (0, 3), (1, 4)],
    "book3": [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 4), (1, 4)],
}


def edge_triangles(g: Graph, threads: int | None = None):
    """(off, adj, t): the oracle's CSR and, per adjacency slot, the number of
    triangles through that edge."""
    off, adj = g.csr()
    t = np.zeros(max(1, len(adj)), dtype=np.int64)
    _L().orc_edge_triangles(g._h, threads or default_threads(), t.ctypes.data)
    return off, adj, t[: len(adj)]


def noninduced5_closed_forms(g: Graph, threads: int | None = None) -> dict[str, int]:
    """Subgraph counts of the FIVE_NONINDUCED shapes, exact (Python ints):

    * star4:   sum_v C(d_v, 4)  (centre and an unordered 4-set of its neighbours)
    * fork:    sum over ordered edges (c, x) of
               (d_x - 1 - t_cx) C(d_c - 1, 2) + t_cx C(d_c - 2, 2)
               (c the degree-3 vertex, x its neighbour of degree 2; x's other
               neighbour w, then two more neighbours of c besides x and w)
    * cricket: sum_v t_v C(d_v - 2, 2)  (the degree-4 vertex, one of its
               triangles, two more of its neighbours)
    * bull:    sum over edges {a, b} of t_ab ((d_a - 2)(d_b - 2) - (t_ab - 1))
               (the triangle's edge that carries both pendants, the third
               triangle vertex, then a pendant on each end; the two pendants
               must differ, and they coincide exactly on another common
               neighbour of a and b)
    * book3:   sum over edges of C(t_ab, 3)  (the spine and three pages)
    """
    off, adj, t = edge_triangles(g, threads)
    n = g.n
    deg = np.diff(off).astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dc = [int(x) for x in deg]
    out = {"star4": 0, "fork": 0, "cricket": 0, "bull": 0, "book3": 0}
    tv = [0] * n
    for v, x, te in zip(src.tolist(), adj.tolist(), t.tolist()):
        tv[v] += te
        dv, dx = dc[v], dc[x]
        # ordered (c = v, x)
        out["fork"] += (dx - 1 - te) * math.comb(dv - 1, 2) + te * math.comb(max(dv - 2, 0), 2)
        if v < x:
            out["bull"] += te * ((dv - 2) * (dx - 2) - (te - 1)) if te else 0
            out["book3"] += math.comb(te, 3)
    for v in range(n):
        out["star4"] += math.comb(dc[v], 4)
        out["cricket"] += (tv[v] // 2) * math.comb(max(dc[v] - 2, 0), 2)
    return out


def noninduced5_rows(induced_counts: dict[int, int]) -> dict[str, int]:
    """sum_Q c(P, Q) I(Q) for each FIVE_NONINDUCED shape P, from a vertex-
    induced 5-motif census keyed by canonical bitmask."""
    c = spanning_copies(5)
    out = {}
    for name, edges in FIVE_NONINDUCED.items():
        p = canonical_of_edges(5, edges)
        out[name] = sum(c.get((p, q), 0) * cnt for q, cnt in induced_counts.items())
    return out