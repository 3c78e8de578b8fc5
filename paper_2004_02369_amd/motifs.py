"""Vertex-induced motif counts by a second exact route: count every
connected k-vertex pattern edge-induced (non-induced subgraph copies, which
pattern-aware matching counts with small cores and more set-size
arithmetic), then solve the triangular system

    N(P) = sum over Q of c(P, Q) * I(Q)

for the induced counts I, where c(P, Q) is the number of spanning
subgraphs of Q isomorphic to P.  This is not the paper's method (it
matches each vertex-induced pattern with anti-edges, Sec. 3.1.3); it is the
inversion route kept beside it for motif censuses.  The GPU counts; the
inversion is exact integer arithmetic on the host.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

from . import patterns as pt


def _canon(k, edges):
    best = None
    for perm in itertools.permutations(range(k)):
        key = tuple(sorted(tuple(sorted((perm[a], perm[b]))) for a, b in edges))
        if best is None or key < best:
            best = key
    return best


@lru_cache(maxsize=None)
def shapes(k: int) -> tuple:
    """The connected k-vertex shapes, as canonical edge tuples, sparsest
    first (the generator's order)."""
    return tuple(_canon(k, s["edges"]) for s in pt.all_vertex_induced(k))


@lru_cache(maxsize=None)
def spanning_copies(k: int) -> tuple:
    """c[i][j]: subsets of the edges of shape j, touching all k vertices and
    connected, isomorphic to shape i (0 unless shape i has no more edges)."""
    sh = shapes(k)
    index = {s: i for i, s in enumerate(sh)}
    c = [[0] * len(sh) for _ in sh]
    for j, q in enumerate(sh):
        for r in range(k - 1, len(q) + 1):
            for sub in itertools.combinations(q, r):
                if len({v for e in sub for v in e}) != k:
                    continue
                key = _canon(k, sub)
                if key in index:
                    c[index[key]][j] += 1
    return tuple(tuple(row) for row in c)


def invert(noninduced, k: int) -> list[int]:
    """Induced counts from the non-induced ones (both in shapes(k) order)."""
    c = spanning_copies(k)
    n = len(c)
    # denser shapes have fewer supergraphs: solve from the densest down
    order = sorted(range(n), key=lambda i: -len(shapes(k)[i]))
    out = [0] * n
    for i in order:
        rest = sum(c[i][j] * out[j] for j in range(n) if j != i and c[i][j])
        assert c[i][i] == 1
        out[i] = int(noninduced[i]) - rest
    return out


def induced_counts(G, k: int, pg, **knobs) -> list[int]:
    """All connected k-vertex vertex-induced motif counts (shapes(k) order)
    by the inversion route: one batched launch of the edge-induced shapes."""
    plans = [pg.plan_pattern({"k": k, "edges": list(s)}) for s in shapes(k)]
    non = pg.count(G, plans, **knobs)
    return invert(non, k)
