"""Exhaustive checks on tiny graphs (n <= ~12): the oracle of the oracle.

TEST INFRASTRUCTURE ONLY.  Pure Python, no shared code with anything else.

* :func:`maps_count` -- every injective map of the regular pattern vertices
  into V(G), tested against the four match conditions (true edges, anti-edges,
  labels, anti-vertices as stated in Sec. 3.1.2), divided by the number of
  permutations of the pattern that preserve its typed structure.
* :func:`induced_subsets_count` -- vertex-induced matches counted the way the
  problem statement defines them (Sec. 2.1): k-vertex subsets whose induced
  subgraph is isomorphic to the pattern, by trying every bijection.
"""
from __future__ import annotations

import itertools


def _adj_sets(n, src, dst):
    adj = [set() for _ in range(n)]
    for a, b in zip(list(map(int, src)), list(map(int, dst))):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def _pattern_sets(spec):
    k = spec["k"]
    E = set()
    for u, v in spec.get("edges", []):
        E.add(frozenset((u, v)))
    A = set()
    for u, v in spec.get("anti", []) or []:
        A.add(frozenset((u, v)))
    if spec.get("induced"):
        for u, v in itertools.combinations(range(k), 2):
            if frozenset((u, v)) not in E:
                A.add(frozenset((u, v)))
    av = [frozenset(x) for x in (spec.get("av") or [])]
    labels = spec.get("labels") or [-1] * k
    avl = spec.get("av_labels") or [-1] * len(av)
    return k, E, A, av, labels, avl


def _typed_aut(spec) -> int:
    k, E, A, av, labels, avl = _pattern_sets(spec)
    av_items = sorted((tuple(sorted(s)), l) for s, l in zip(av, avl))
    c = 0
    for pm in itertools.permutations(range(k)):
        if any(labels[i] != labels[pm[i]] for i in range(k)):
            continue
        ok = True
        for i, j in itertools.combinations(range(k), 2):
            e = frozenset((i, j))
            f = frozenset((pm[i], pm[j]))
            if (e in E) != (f in E) or (e in A) != (f in A):
                ok = False
                break
        if not ok:
            continue
        img = sorted((tuple(sorted(pm[x] for x in s)), l) for s, l in zip(av, avl))
        if img == av_items:
            c += 1
    return c


def is_valid_map(adj, glabels, spec, img) -> bool:
    k, E, A, av, labels, avl = _pattern_sets(spec)
    if len(set(img)) != k:
        return False
    for i in range(k):
        if labels[i] != -1 and (glabels is None or glabels[img[i]] != labels[i]):
            return False
    for e in E:
        a, b = tuple(e)
        if img[b] not in adj[img[a]]:
            return False
    for e in A:
        a, b = tuple(e)
        if img[b] in adj[img[a]]:
            return False
    pn = {u: {v for v in range(k) if frozenset((u, v)) in E} for u in range(k)}
    for s, lab in zip(av, avl):
        common = None
        for u in s:
            part = set(adj[img[u]]) - {img[y] for y in pn[u]}
            common = part if common is None else common & part
        if lab != -1:
            common = {w for w in common if glabels is not None and glabels[w] == lab}
        if common:
            return False
    return True


def maps_count(graph, spec, labels=None) -> int:
    n, src, dst = graph
    adj = _adj_sets(n, src, dst)
    k = spec["k"]
    valid = sum(1 for img in itertools.permutations(range(n), k) if is_valid_map(adj, labels, spec, img))
    a = _typed_aut(spec)
    assert valid % a == 0
    return valid // a


def canonical_maps(graph, spec, labels=None):
    """All valid maps (as tuples indexed by pattern vertex)."""
    n, src, dst = graph
    adj = _adj_sets(n, src, dst)
    return [img for img in itertools.permutations(range(n), spec["k"]) if is_valid_map(adj, labels, spec, img)]


def induced_subsets_count(graph, k, pattern_edges) -> int:
    n, src, dst = graph
    adj = _adj_sets(n, src, dst)
    P = {frozenset(e) for e in pattern_edges}
    c = 0
    for S in itertools.combinations(range(n), k):
        for pm in itertools.permutations(S):
            if all(((pm[b] in adj[pm[a]]) == (frozenset((a, b)) in P))
                   for a, b in itertools.combinations(range(k), 2)):
                c += 1
                break
    return c


def typed_aut(spec) -> int:
    return _typed_aut(spec)


def domains_brute(graph, spec, labels=None) -> list[int]:
    """|{m(u) : m valid}| for every regular vertex u, over every injective map."""
    maps = canonical_maps(graph, spec, labels)
    return [len({m[u] for m in maps}) for u in range(spec["k"])]
