"""Pattern constructors (Fig. "Pattern Interface", [S1-S3], [G1-G2], [C1]).

Host-side helpers returning plain pattern specs (dicts, see :mod:`pg`).
generateStar(k) has k vertices (one centre, k-1 leaves), as the paper
uses it (3-star = wedge, Sec. 3.2.2; 4-star in Sec. 6.3).
"""
from __future__ import annotations

import itertools
from functools import lru_cache


def clique(k: int, induced: bool = False) -> dict:
    return {"k": k, "edges": list(itertools.combinations(range(k), 2)), "induced": induced}


def star(k: int, induced: bool = False) -> dict:
    return {"k": k, "edges": [(0, i) for i in range(1, k)], "induced": induced}


def chain(k: int, induced: bool = False) -> dict:
    return {"k": k, "edges": [(i, i + 1) for i in range(k - 1)], "induced": induced}


def _canon(k: int, edges) -> tuple:
    """Smallest sorted edge tuple over all relabellings (k <= 6)."""
    best = None
    for pm in itertools.permutations(range(k)):
        e = tuple(sorted(tuple(sorted((pm[a], pm[b]))) for a, b in edges))
        if best is None or e < best:
            best = e
    return best


def _connected(k: int, edges) -> bool:
    adj = {i: set() for i in range(k)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen, todo = {0}, [0]
    while todo:
        x = todo.pop()
        for y in adj[x] - seen:
            seen.add(y)
            todo.append(y)
    return len(seen) == k


@lru_cache(maxsize=None)
def _vertex_induced_shapes(k: int):
    pairs = list(itertools.combinations(range(k), 2))
    shapes = set()
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        if _connected(k, edges):
            shapes.add(_canon(k, edges))
    return sorted(shapes, key=lambda e: (len(e), e))


def all_vertex_induced(k: int) -> list[dict]:
    """[G2] Every connected k-vertex pattern up to isomorphism, vertex-induced
    (1, 2, 6, 21 for k = 2..5)."""
    return [{"k": k, "edges": list(e), "induced": True} for e in _vertex_induced_shapes(k)]


def all_edge_induced(n_edges: int) -> list[dict]:
    """[G1] Every connected pattern with n_edges edges up to isomorphism."""
    out = set()
    for k in range(2, n_edges + 2):
        pairs = list(itertools.combinations(range(k), 2))
        for sel in itertools.combinations(pairs, n_edges):
            if len({v for e in sel for v in e}) == k and _connected(k, sel):
                out.add((k, _canon(k, sel)))
    return [{"k": k, "edges": list(e)} for k, e in sorted(out, key=lambda t: (t[0], t[1]))]


def extend_by_edge(patterns: list[dict]) -> list[dict]:
    """[C1] All distinct connected patterns obtained by adding one edge
    (between existing vertices or to one new vertex)."""
    out = set()
    for p in patterns:
        k, E = p["k"], {tuple(sorted(e)) for e in p["edges"]}
        for a, b in itertools.combinations(range(k), 2):
            if (a, b) not in E:
                out.add((k, _canon(k, E | {(a, b)})))
        for a in range(k):
            out.add((k + 1, _canon(k + 1, E | {(a, k)})))
    return [{"k": k, "edges": list(e)} for k, e in sorted(out, key=lambda t: (t[0], t[1]))]


# Named patterns of the paper's evaluation whose shapes the text states.
P7_TRIANGLE_NO_K4 = {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "av": [[0, 1, 2]]}   # Sec. 6.5, p7
P8_INDUCED_DIAMOND = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3)], "induced": True}  # p8
PA_TWO_COMMON_FRIENDS = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(1, 3)]}  # Sec. 3.1.1 p_a

# 5-vertex patterns whose every edge touches the edge (0, 1): their core is
# that one edge, and the other three vertices are completed from set sizes
# (the edge's common neighbours and each end's own neighbours).
EDGE_CORE_5 = {
    # triangle 0-1-2 with two pendant vertices on vertex 0
    "cricket": {"k": 5, "edges": [(0, 1), (0, 2), (1, 2), (0, 3), (0, 4)]},
    # triangle 0-1-2 with one pendant on vertex 0 and one on vertex 1
    "bull": {"k": 5, "edges": [(0, 1), (0, 2), (1, 2), (0, 3), (1, 4)]},
    # three triangles sharing the edge 0-1 (the book K_{1,1,3})
    "book3": {"k": 5, "edges": [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 4), (1, 4)]},
}
