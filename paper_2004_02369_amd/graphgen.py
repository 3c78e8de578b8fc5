"""Seeded synthetic data graphs.

This module only draws inputs: it holds no step of the matching method.
It is the one module that both the HIP path and the CPU oracle consume,
and it only returns plain edge arrays.

Every generator returns ``(n, src, dst)`` with ``src``/``dst`` int32 numpy
arrays of undirected edges.  The large generators (ER, Chung-Lu, R-MAT)
return exactly the requested number of *distinct* undirected edges with
no self-loops, in draw order, with each edge's two endpoints in random
order, and the vertex ids scrambled by a seeded permutation so that the
ingest step really has to re-rank vertices by degree.  Callers that want
to exercise ingest of dirty input (loops, duplicates, both directions)
use :func:`dirty_copy`.

PRNG: numpy ``Generator(PCG64(seed))`` (O'Neill's PCG-64 XSL-RR), which is
deterministic across platforms for a fixed numpy major version.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "erdos_renyi_m", "chung_lu", "rmat", "gnp", "complete", "complete_multipartite",
    "cycle", "path", "star", "petersen", "turan", "disjoint_union", "dirty_copy",
    "relabel", "all_graphs", "hub_plus_er", "WORKLOADS", "workload", "labelled_workload",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _first_unique(keys: np.ndarray, m: int) -> np.ndarray:
    """Indices (in draw order) of the first ``m`` distinct keys, or all if fewer."""
    _, first = np.unique(keys, return_index=True)
    first.sort()
    return first[:m]


def _draw_until(n: int, m: int, seed: int, draw_batch) -> tuple[np.ndarray, np.ndarray]:
    """Draw endpoint pairs with ``draw_batch(rng, size)`` until ``m`` distinct
    undirected non-loop pairs exist; keep the first ``m`` in draw order."""
    if m < 0:
        raise ValueError("m must be >= 0")
    if m > n * (n - 1) // 2:
        raise ValueError(f"m={m} exceeds n(n-1)/2 for n={n}")
    rng = _rng(seed)
    us, vs = [], []
    total_keys = np.empty(0, dtype=np.int64)
    have = 0
    while True:
        need = m - have
        size = max(1024, int(need * 1.25) + 1024)
        u, v = draw_batch(rng, size)
        keep = u != v
        u, v = u[keep].astype(np.int64), v[keep].astype(np.int64)
        us.append(u)
        vs.append(v)
        lo, hi = np.minimum(u, v), np.maximum(u, v)
        total_keys = np.concatenate([total_keys, lo * n + hi])
        idx = _first_unique(total_keys, m)
        have = idx.size
        if have >= m:
            break
    u = np.concatenate(us)[idx]
    v = np.concatenate(vs)[idx]
    return u, v


def _scramble(n: int, u: np.ndarray, v: np.ndarray, seed: int):
    perm = _rng(seed ^ 0x5EED5EED).permutation(n).astype(np.int64)
    return perm[u].astype(np.int32), perm[v].astype(np.int32)


def erdos_renyi_m(n: int, m: int, seed: int = 1):
    """G(n, m): uniform unordered pairs u != v, duplicates rejected, until m unique."""
    def draw(rng, size):
        return rng.integers(0, n, size), rng.integers(0, n, size)
    u, v = _draw_until(n, m, seed, draw)
    u, v = _scramble(n, u, v, seed)
    return n, u, v


def chung_lu_weights(n: int, m: int, gamma: float, w_max: float) -> np.ndarray:
    """w_i = w_max * (1 + i/i0)^(-1/(gamma-1)), i0 solved so that sum(w) = 2m."""
    a = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)

    def total(i0):
        return float(np.sum(w_max * (1.0 + i / i0) ** (-a)))

    lo, hi = 1e-6, float(n) * 1e3
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if total(mid) < 2.0 * m:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return w_max * (1.0 + i / i0) ** (-a)


def chung_lu(n: int, m: int, gamma: float, w_max: float, seed: int = 2):
    """Chung-Lu: endpoints drawn i.i.d. proportional to w; loops and duplicates
    dropped until m unique edges remain."""
    w = chung_lu_weights(n, m, gamma, w_max)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(rng, size):
        a = np.searchsorted(cdf, rng.random(size), side="right")
        b = np.searchsorted(cdf, rng.random(size), side="right")
        return np.minimum(a, n - 1), np.minimum(b, n - 1)
    u, v = _draw_until(n, m, seed, draw)
    u, v = _scramble(n, u, v, seed)
    return n, u, v


def rmat(scale: int, m: int, a=0.57, b=0.19, c=0.19, seed: int = 3):
    """R-MAT (Chakrabarti et al. 2004) without noise: per edge, `scale` quadrant
    choices with probabilities a, b, c, d=1-a-b-c; loops and duplicates are
    dropped until m unique undirected edges remain.  Isolated vertices kept."""
    n = 1 << scale
    cut = np.array([a, a + b, a + b + c])

    def draw(rng, size):
        u = np.zeros(size, dtype=np.int64)
        v = np.zeros(size, dtype=np.int64)
        for _ in range(scale):
            q = np.searchsorted(cut, rng.random(size), side="right")
            u = (u << 1) | (q >= 2)
            v = (v << 1) | ((q == 1) | (q == 3))
        return u, v
    u, v = _draw_until(n, m, seed, draw)
    u, v = _scramble(n, u, v, seed)
    return n, u, v


def gnp(n: int, p: float, seed: int = 4):
    """G(n, p) over unordered pairs (small n only)."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return n, iu[keep].astype(np.int32), ju[keep].astype(np.int32)


def _pairs(n, pairs):
    pairs = list(pairs)
    if not pairs:
        return n, np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.array(pairs, dtype=np.int32)
    return n, a[:, 0].copy(), a[:, 1].copy()


def complete(n: int):
    return _pairs(n, itertools.combinations(range(n), 2))


def complete_multipartite(sizes):
    part = []
    for i, s in enumerate(sizes):
        part += [i] * s
    n = len(part)
    return _pairs(n, [(x, y) for x, y in itertools.combinations(range(n), 2) if part[x] != part[y]])


def turan(n: int, r: int):
    sizes = [n // r + (1 if i < n % r else 0) for i in range(r)]
    return complete_multipartite(sizes)


def cycle(n: int):
    return _pairs(n, [(i, (i + 1) % n) for i in range(n)])


def path(n: int):
    return _pairs(n, [(i, i + 1) for i in range(n - 1)])


def star(n_leaves: int):
    return _pairs(n_leaves + 1, [(0, i) for i in range(1, n_leaves + 1)])


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return _pairs(10, outer + spokes + inner)


def disjoint_union(*graphs):
    off, us, vs = 0, [], []
    for n, u, v in graphs:
        us.append(u.astype(np.int64) + off)
        vs.append(v.astype(np.int64) + off)
        off += n
    return off, np.concatenate(us).astype(np.int32), np.concatenate(vs).astype(np.int32)


def hub_plus_er(n_leaves: int, m_leaves: int, seed: int = 5):
    """One hub adjacent to every other vertex (vertex 0, degree n_leaves)
    plus G(n_leaves, m_leaves) among the leaves (vertices 1..n_leaves)."""
    _, u, v = erdos_renyi_m(n_leaves, m_leaves, seed=seed)
    leaves = np.arange(1, n_leaves + 1, dtype=np.int32)
    src = np.concatenate([np.zeros(n_leaves, np.int32), u + 1])
    dst = np.concatenate([leaves, v + 1])
    return n_leaves + 1, src.astype(np.int32), dst.astype(np.int32)


def relabel(graph, seed: int):
    """Random vertex relabelling (same graph, different ids)."""
    n, u, v = graph
    perm = _rng(seed).permutation(n).astype(np.int32)
    return n, perm[u], perm[v]


def dirty_copy(graph, seed: int):
    """Same undirected simple graph, written dirtily: every edge in both
    directions, some repeated, plus self-loops, shuffled."""
    n, u, v = graph
    rng = _rng(seed)
    uu = np.concatenate([u, v, u[: len(u) // 3]])
    vv = np.concatenate([v, u, v[: len(v) // 3]])
    if n > 0:
        loops = rng.integers(0, n, max(1, n // 7))
        uu = np.concatenate([uu, loops])
        vv = np.concatenate([vv, loops])
    order = rng.permutation(uu.size)
    return n, uu[order].astype(np.int32), vv[order].astype(np.int32)


def all_graphs(n: int):
    """Every labelled simple graph on n vertices (n <= 6: 2^15 graphs)."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield _pairs(n, [pairs[i] for i in range(len(pairs)) if mask >> i & 1])


# Named synthetic workloads: sizes and skew of the paper's evaluation inputs.
WORKLOADS = {
    # uniform random graph, average degree 20
    "er_2k_20k": dict(kind="er", n=2000, m=20000, seed=20001),
    # power law, exponent 2.1, max weight 5000 (stands in for Mico's 100K / 1M)
    "chunglu_100k_1m": dict(kind="cl", n=100_000, m=1_000_000, gamma=2.1, w_max=5000.0, seed=20002),
    # R-MAT a=.57 b=c=.19, edge factor 16 (16M edges stand in for Patents' edge count)
    "rmat20_16m": dict(kind="rmat", scale=20, m=16 * (1 << 20), seed=20003),
    # the serving graph: 4M vertices, 64M edges (CSR larger than the last-level cache)
    "rmat22_64m": dict(kind="rmat", scale=22, m=16 * (1 << 22), seed=20008),
    "rmat16_1m": dict(kind="rmat", scale=16, m=16 * (1 << 16), seed=20004),
    "rmat14_256k": dict(kind="rmat", scale=14, m=16 * (1 << 14), seed=20005),
    "rmat12_64k": dict(kind="rmat", scale=12, m=16 * (1 << 12), seed=20006),
    "chunglu_20k_100k": dict(kind="cl", n=20_000, m=100_000, gamma=2.1, w_max=700.0, seed=20007),
    # labelled (frequent subgraph mining): power law, exponent 2.2, max weight
    # 3.5 * sqrt(2m), 16 labels drawn uniformly with their own seed
    "chunglu_1m_10m_l16": dict(kind="cl", n=1_000_000, m=10_000_000, gamma=2.2, w_max=15652.0, seed=20009,
                               labels=16, label_seed=20010),
    "chunglu_20k_100k_l4": dict(kind="cl", n=20_000, m=100_000, gamma=2.2, w_max=700.0, seed=20011,
                                labels=4, label_seed=20012),
}


def labelled_workload(name: str):
    """(n, src, dst, labels int16) of a labelled workload."""
    w = WORKLOADS[name]
    n, src, dst = workload(name)
    labels = _rng(w["label_seed"]).integers(0, w["labels"], n).astype(np.int16)
    return n, src, dst, labels


def workload(name: str):
    w = WORKLOADS[name]
    if w["kind"] == "er":
        return erdos_renyi_m(w["n"], w["m"], seed=w["seed"])
    if w["kind"] == "cl":
        return chung_lu(w["n"], w["m"], w["gamma"], w["w_max"], seed=w["seed"])
    if w["kind"] == "rmat":
        return rmat(w["scale"], w["m"], seed=w["seed"])
    raise KeyError(name)
