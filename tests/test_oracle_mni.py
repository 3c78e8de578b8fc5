"""Pins of the oracle's MNI domains (Sec. 2: a pattern's support is the
smallest number of distinct data vertices any of its vertices is mapped
to): brute force over every injective map, label-histogram closed forms,
textbook special cases and anti-monotonicity."""
import itertools
import random

import numpy as np
import pytest

from oracle import brute
from paper_2004_02369_amd import graphgen as gg


def _labelled(n, m, nl, seed):
    g = gg.erdos_renyi_m(n, m, seed=seed)
    lab = np.random.default_rng(seed + 1).integers(0, nl, n).astype(np.int16)
    return g, lab


def _adj(g):
    n, s, d = g
    adj = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def _hist(adj, lab, nl):
    h = np.zeros((len(adj), nl), dtype=np.int64)
    for v, nb in enumerate(adj):
        for w in nb:
            h[v, lab[w]] += 1
    return h


RANDOM_SPECS = [
    {"k": 3, "edges": [(0, 1), (1, 2)]},
    {"k": 3, "edges": [(0, 1), (1, 2)], "labels": [0, 1, 0]},
    {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "labels": [1, -1, 1]},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [0, 1, 1, 0]},
    {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [1, 0, 0, 2]},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(1, 3)]},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "induced": True},
    {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "av": [[0, 1, 2]]},
    {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0, 2]], "labels": [-1, 0, -1]},
]


@pytest.mark.parametrize("si", range(len(RANDOM_SPECS)))
def test_domains_match_brute_force(orc, si):
    spec = RANDOM_SPECS[si]
    for seed in range(4):
        g, lab = _labelled(9, 16 + 2 * seed, 3, 100 + seed)
        og = orc.Graph.from_tuple(g, lab)
        assert orc.domains(og, spec) == brute.domains_brute(g, spec, lab), (spec, seed)


def test_labelled_edge_and_wedge_closed_forms(orc):
    nl = 4
    g, lab = _labelled(400, 1500, nl, 7)
    og = orc.Graph.from_tuple(g, lab)
    adj = _adj(g)
    h = _hist(adj, lab, nl)
    for a, b in itertools.combinations_with_replacement(range(nl), 2):
        # one labelled edge: an endpoint labelled a with a neighbour labelled b
        want_a = sum(1 for v in range(400) if lab[v] == a and h[v, b] >= 1)
        want_b = sum(1 for v in range(400) if lab[v] == b and h[v, a] >= 1)
        assert orc.domains(og, {"k": 2, "edges": [(0, 1)], "labels": [a, b]}) == [want_a, want_b]
    for c in range(nl):
        for a, b in itertools.combinations_with_replacement(range(nl), 2):
            spec = {"k": 3, "edges": [(0, 1), (0, 2)], "labels": [c, a, b]}
            need = {x: (a, b).count(x) for x in (a, b)}
            centre = sum(1 for v in range(400) if lab[v] == c and all(h[v, x] >= t for x, t in need.items()))
            # a leaf labelled a: a neighbour w labelled c with another
            # neighbour (not v) labelled b
            leaf_a = sum(1 for v in range(400) if lab[v] == a and any(
                lab[w] == c and h[w, b] - (1 if lab[v] == b else 0) >= 1 for w in adj[v]))
            leaf_b = sum(1 for v in range(400) if lab[v] == b and any(
                lab[w] == c and h[w, a] - (1 if lab[v] == a else 0) >= 1 for w in adj[v]))
            assert orc.domains(og, spec) == [centre, leaf_a, leaf_b], spec


def test_labelled_star_centre_closed_form(orc):
    nl = 3
    g, lab = _labelled(300, 1400, nl, 11)
    og = orc.Graph.from_tuple(g, lab)
    h = _hist(_adj(g), lab, nl)
    for c in range(nl):
        for leaves in itertools.combinations_with_replacement(range(nl), 3):
            spec = {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [c, *leaves]}
            need = {x: leaves.count(x) for x in set(leaves)}
            want = sum(1 for v in range(300) if lab[v] == c and all(h[v, x] >= t for x, t in need.items()))
            assert orc.domains(og, spec)[0] == want


def test_special_cases(orc):
    # every vertex of K_n is in every domain of K_k (k <= n); none for k > n
    og = orc.Graph.from_tuple(gg.complete(6))
    for k in range(2, 7):
        assert orc.domains(og, {"k": k, "edges": list(itertools.combinations(range(k), 2))}) == [6] * k
    assert orc.mni_support(og, {"k": 3, "edges": [(0, 1), (1, 2)], "induced": True}) == 0
    # star K_{1,5}: a 3-star's centre has one image, its leaves five
    og = orc.Graph.from_tuple(gg.star(5))
    assert orc.domains(og, {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)]}) == [1, 5, 5, 5]
    # a path's end vertices: in P_6 every vertex is some 3-path's end, only
    # inner ones are centres
    og = orc.Graph.from_tuple(gg.path(6))
    assert orc.domains(og, {"k": 3, "edges": [(0, 1), (1, 2)]}) == [6, 4, 6]


def test_anti_monotone(orc):
    rng = random.Random(5)
    g, lab = _labelled(150, 700, 2, 21)
    og = orc.Graph.from_tuple(g, lab)
    for _ in range(20):
        base = {"k": 3, "edges": [(0, 1), (1, 2)], "labels": [rng.randrange(2) for _ in range(3)]}
        sup = orc.mni_support(og, base)
        # add an edge between existing vertices, or a new labelled vertex
        closed = dict(base, edges=base["edges"] + [(0, 2)])
        grown = {"k": 4, "edges": base["edges"] + [(rng.randrange(3), 3)],
                 "labels": base["labels"] + [rng.randrange(2)]}
        assert orc.mni_support(og, closed) <= sup
        assert orc.mni_support(og, grown) <= sup
