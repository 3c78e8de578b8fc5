"""Host logic of frequent subgraph mining (no GPU): canonical labelled
patterns, orbits, extension by one edge, and the FSM loop checked against a
direct computation of every labelled pattern's MNI support by the oracle."""
import itertools
import random

import numpy as np
import pytest

from paper_2004_02369_amd import fsm
from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import patterns as pt


def test_canonical_is_relabelling_invariant():
    rng = random.Random(3)
    for _ in range(200):
        k = rng.randint(2, 5)
        edges = {(i, rng.randrange(i)) for i in range(1, k)}
        for _ in range(rng.randint(0, 3)):
            a, b = rng.sample(range(k), 2)
            edges.add((a, b))
        labels = [rng.randrange(3) for _ in range(k)]
        p = fsm.canonical(k, edges, labels)
        perm = list(range(k))
        rng.shuffle(perm)
        q = fsm.canonical(k, [(perm[a], perm[b]) for a, b in edges], [labels[perm.index(i)] for i in range(k)])
        assert p == q


def test_class_counts():
    # labelled single edges over 3 labels: 6; unlabelled 3-edge shapes: 3
    assert len(fsm.single_edges([0, 1, 2])) == 6
    wedge = fsm.extend_by_edge(fsm.single_edges([0]), [0])
    assert len(wedge) == 1 and wedge[0].k == 3
    three = fsm.extend_by_edge(wedge, [0])
    assert sorted((p.k, len(p.edges)) for p in three) == [(3, 3), (4, 3), (4, 3)]
    # the same shapes as the unlabelled generator
    assert len(three) == len([s for s in pt.extend_by_edge([{"k": 3, "edges": [(0, 1), (1, 2)]}])])


def test_orbits():
    star = fsm.canonical(4, [(0, 1), (0, 2), (0, 3)], [5, 1, 1, 2])
    reps = fsm.orbit_representatives(star)
    assert len(reps) == 3  # centre, the two 1-leaves, the 2-leaf
    tri = fsm.canonical(3, [(0, 1), (1, 2), (0, 2)], [0, 0, 0])
    assert len(fsm.orbit_representatives(tri)) == 1
    path = fsm.canonical(4, [(0, 1), (1, 2), (2, 3)], [0, 1, 1, 0])
    assert len(fsm.orbit_representatives(path)) == 2


def test_sub_patterns():
    p4 = fsm.canonical(4, [(0, 1), (1, 2), (2, 3)], [0, 1, 2, 3])
    subs = fsm.sub_patterns(p4)
    assert {(s.k, s.labels) for s in subs} == {(3, fsm.canonical(3, [(0, 1), (1, 2)], [0, 1, 2]).labels),
                                               (3, fsm.canonical(3, [(0, 1), (1, 2)], [1, 2, 3]).labels)}
    tri = fsm.canonical(3, [(0, 1), (1, 2), (0, 2)], [0, 1, 2])
    assert len(fsm.sub_patterns(tri)) == 3


def _all_labelled(max_edges, alphabet):
    """Every connected labelled pattern with 1..max_edges edges, by brute
    force over shapes and labellings."""
    out = set()
    for k in range(2, max_edges + 2):
        pairs = list(itertools.combinations(range(k), 2))
        for ne in range(k - 1, max_edges + 1):
            for sel in itertools.combinations(pairs, ne):
                if len({v for e in sel for v in e}) != k or not fsm._connected(k, sel):
                    continue
                for labels in itertools.product(alphabet, repeat=k):
                    out.add(fsm.canonical(k, sel, labels))
    return out


@pytest.mark.parametrize("threshold", [5, 20, 60])
def test_loop_equals_direct_supports(orc, threshold):
    g = gg.chung_lu(150, 400, 2.2, 20.0, seed=4)
    lab = np.random.default_rng(8).integers(0, 3, 150).astype(np.int16)
    og = orc.Graph.from_tuple(g, lab)

    def support(cands):
        return [orc.mni_support(og, p.spec()) for p in cands]

    freq, stats = fsm.mine(support, [0, 1, 2], threshold, 3)
    got = {p for level in freq.values() for p in level}
    every = _all_labelled(3, [0, 1, 2])
    direct = {p for p in every if orc.mni_support(og, p.spec()) >= threshold}
    assert got == direct
    assert stats[0]["candidates"] == 6
    for level in freq.values():
        for p, s in level.items():
            assert s >= threshold and s == orc.mni_support(og, p.spec())
