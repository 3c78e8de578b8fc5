"""The inversion route (non-induced counts -> induced counts) on the CPU:
its coefficients against direct isomorphism counting and its arithmetic
against the oracle's induced and edge-induced counts."""
import itertools
import math

import pytest

from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import motifs


def test_shape_counts_and_diagonal():
    assert [len(motifs.shapes(k)) for k in (2, 3, 4, 5)] == [1, 2, 6, 21]
    for k in (3, 4, 5):
        c = motifs.spanning_copies(k)
        assert all(c[i][i] == 1 for i in range(len(c)))
        # the path is a spanning subgraph of every connected shape with a
        # Hamiltonian path; the complete graph contains k!/2 paths
        path = motifs.shapes(k).index(motifs._canon(k, [(i, i + 1) for i in range(k - 1)]))
        complete = motifs.shapes(k).index(motifs._canon(k, list(itertools.combinations(range(k), 2))))
        assert c[path][complete] == math.factorial(k) // 2


def test_known_coefficients_k4():
    sh = motifs.shapes(4)
    c = motifs.spanning_copies(4)
    star = sh.index(motifs._canon(4, [(0, 1), (0, 2), (0, 3)]))
    cyc = sh.index(motifs._canon(4, [(0, 1), (1, 2), (2, 3), (3, 0)]))
    k4 = sh.index(motifs._canon(4, list(itertools.combinations(range(4), 2))))
    assert c[star][k4] == 4 and c[cyc][k4] == 3 and c[star][cyc] == 0


@pytest.mark.parametrize("k", [3, 4, 5])
def test_invert_matches_oracle(orc, k):
    for seed in range(3):
        g = gg.gnp(11 if k == 5 else 14, 0.45, seed=70 + seed)
        og = orc.Graph.from_tuple(g)
        non = [orc.count(og, {"k": k, "edges": list(s)}) for s in motifs.shapes(k)]
        ind = [orc.count(og, {"k": k, "edges": list(s), "induced": True}) for s in motifs.shapes(k)]
        assert motifs.invert(non, k) == ind
