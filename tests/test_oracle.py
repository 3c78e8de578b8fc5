"""Pins for the CPU oracle: each test checks it against something other than
itself -- closed forms, textbook automorphism counts, brute force over all
maps or all k-subsets, and the special cases the paper states."""
import itertools
import math

import numpy as np
import pytest

from oracle import brute
from paper_2004_02369_amd import graphgen as gg

CLIQUE = lambda k: {"k": k, "edges": list(itertools.combinations(range(k), 2))}
STAR = lambda k: {"k": k, "edges": [(0, i) for i in range(1, k)]}          # k vertices
PATH = lambda k: {"k": k, "edges": [(i, i + 1) for i in range(k - 1)]}
CYCLE = lambda k: {"k": k, "edges": [(i, (i + 1) % k) for i in range(k)]}
DIAMOND = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3)]}      # chord u2-u4
PAW = {"k": 4, "edges": [(0, 1), (1, 2), (2, 0), (0, 3)]}
# p7: triangle whose three vertices share no further common neighbour
P7 = {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "av": [[0, 1, 2]]}
# p8: vertex-induced chordal square (diamond with its missing chord as anti-edge)
P8 = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3)], "anti": [(0, 2)]}
# p_a: two non-adjacent vertices with two common neighbours (4-cycle + one anti-edge)
PA = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(1, 3)]}
# p_d: the middle of a 3-path has no neighbour besides the two ends
PD = {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[1]]}
# p_c: an edge whose endpoints have no common neighbour
PC = {"k": 2, "edges": [(0, 1)], "av": [[0, 1]]}
# p_e: a 3-path whose two ends have no common neighbour besides the middle
PE = {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "av": [[0, 2]]}


def G(orc, g, labels=None):
    return orc.Graph.from_tuple(g, labels)


# ----------------------------------------------------------------- ingest

def test_canonical_graph_invariants(orc):
    g = gg.erdos_renyi_m(300, 2000, seed=7)
    og = G(orc, g)
    assert og.m == 2000
    d = og.degrees()
    assert d.sum() == 2 * og.m
    off, adj = og.csr()
    for v in range(og.n):
        row = adj[off[v]:off[v + 1]]
        assert np.all(np.diff(row) > 0) and v not in row
    dirty = G(orc, gg.dirty_copy(g, seed=3))
    assert dirty.m == og.m
    off2, adj2 = dirty.csr()
    assert np.array_equal(off, off2) and np.array_equal(adj, adj2)


# ------------------------------------------------------- automorphisms

@pytest.mark.parametrize("spec,expected", [
    (CLIQUE(3), 6), (CLIQUE(4), 24), (CLIQUE(5), 120), (CLIQUE(14), math.factorial(14)),
    (STAR(4), 6), (STAR(5), 24), (PATH(4), 2), (PATH(5), 2), (CYCLE(4), 8), (CYCLE(5), 10),
    (DIAMOND, 4), (PAW, 2), (P7, 6), (P8, 4), (PA, 4), (PD, 2), (PC, 2), (PE, 2),
])
def test_aut_textbook(orc, spec, expected):
    assert orc.aut(spec) == expected
    if spec["k"] <= 7:
        assert brute.typed_aut(spec) == expected


def test_aut_anti_edge_breaks_symmetry(orc):
    # a 4-cycle with one diagonal anti-edge keeps only the symmetries that
    # fix that diagonal as a set (the anti-edge is a structural element)
    assert orc.aut(PA) == 4
    assert orc.aut(CYCLE(4)) == 8


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n,k", [(6, 3), (7, 4), (8, 5), (9, 3), (10, 6)])
def test_cliques_in_complete_graph(orc, n, k):
    assert orc.count(G(orc, gg.complete(n)), CLIQUE(k)) == math.comb(n, k)


def _esym(sizes, k):
    return sum(math.prod(c) for c in itertools.combinations(sizes, k))


@pytest.mark.parametrize("sizes,k", [([2, 3, 4], 3), ([2, 2, 2, 2], 4), ([3, 1, 2, 2, 1], 4), ([4, 4], 3)])
def test_cliques_in_multipartite(orc, sizes, k):
    assert orc.count(G(orc, gg.complete_multipartite(sizes)), CLIQUE(k)) == _esym(sizes, k)


def test_no_triangles_in_bipartite(orc):
    assert orc.count(G(orc, gg.complete_multipartite([6, 7])), CLIQUE(3)) == 0


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_stars_degree_sum(orc, k):
    n, u, v = gg.erdos_renyi_m(200, 900, seed=11)
    d = np.bincount(np.concatenate([u, v]), minlength=n)
    # k >= 3: the centre is unique, so sum_v C(d_v, k-1); k = 2 is one edge
    expected = sum(math.comb(int(x), k - 1) for x in d) if k >= 3 else 900
    assert orc.count(G(orc, (n, u, v)), STAR(k)) == expected


def _dense(g):
    n, u, v = g
    A = np.zeros((n, n), dtype=np.int64)
    A[u, v] = 1
    A[v, u] = 1
    np.fill_diagonal(A, 0)
    return A


@pytest.mark.parametrize("seed", [1, 2])
def test_triangles_trace(orc, seed):
    g = gg.erdos_renyi_m(400, 4000, seed=seed)
    A = _dense(g)
    T = int(np.trace(A @ A @ A)) // 6
    og = G(orc, g)
    assert orc.count(og, CLIQUE(3)) == T
    assert og.triangles_per_vertex().sum() == 3 * T
    assert orc.noninduced4(og)["triangle"] == T


def test_four_cycles_trace_and_complete(orc):
    for n in (5, 6, 8):
        assert orc.count(G(orc, gg.complete(n)), CYCLE(4)) == 3 * math.comb(n, 4)
    g = gg.erdos_renyi_m(150, 1200, seed=5)
    A = _dense(g)
    d = A.sum(1)
    m = int(A.sum()) // 2
    c4 = (int(np.trace(np.linalg.matrix_power(A, 4))) - 2 * int((d * d).sum()) + 2 * m) // 8
    og = G(orc, g)
    assert orc.count(og, CYCLE(4)) == c4
    assert orc.noninduced4(og)["cycle"] == c4


def test_noninduced4_forms_match_matcher(orc):
    og = G(orc, gg.erdos_renyi_m(120, 900, seed=9))
    nc = orc.noninduced4(og)
    for name in ("star", "path", "cycle", "paw", "diamond"):
        assert nc[name] == orc.count(og, {"k": 4, "edges": orc.FOUR_NAMES[name]}), name


# ----------------------------------------------------- brute force (O5)

PATTERNS_SMALL = [CLIQUE(3), STAR(3), STAR(4), PATH(4), CYCLE(4), DIAMOND, PAW, CLIQUE(4), P7, P8,
                  PA, PD, PC, PE,
                  {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "anti": [(0, 2)]},
                  # the counterexample to ignoring anti-edges when breaking symmetry
                  {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(0, 2)]},
                  {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0, 2], [1]]}]


@pytest.mark.parametrize("pi", range(len(PATTERNS_SMALL)))
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_matcher_vs_bruteforce(orc, pi, seed):
    spec = PATTERNS_SMALL[pi]
    g = gg.gnp(8, 0.45 + 0.1 * seed, seed=seed)
    assert orc.count(G(orc, g), spec) == brute.maps_count(g, spec)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_labelled_vs_bruteforce(orc, seed):
    g = gg.gnp(8, 0.6, seed=seed)
    lab = np.random.Generator(np.random.PCG64(seed)).integers(0, 2, 8).astype(np.int16)
    for spec in ({"k": 3, "edges": [(0, 1), (1, 2)], "labels": [0, 1, 0]},
                 {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "labels": [1, 1, 0]},
                 {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0, 2]], "labels": [0, -1, 1], "av_labels": [1]}):
        assert orc.count(G(orc, g, lab), spec) == brute.maps_count(g, spec, labels=lab)


@pytest.mark.parametrize("k", [3, 4])
def test_induced_theorem(orc, k):
    """Vertex-induced count through anti-edges equals the k-subset definition."""
    reps = orc.motif_classes(k)
    for seed in (1, 2):
        g = gg.gnp(8, 0.5, seed=seed)
        og = G(orc, g)
        for rep in reps:
            edges = orc.class_edges(k, rep)
            spec = {"k": k, "edges": edges, "induced": True}
            assert orc.count(og, spec) == brute.induced_subsets_count(g, k, edges)


def test_motif_class_counts(orc):
    # connected graphs on 3, 4, 5 vertices: 2, 6, 21
    assert [len(orc.motif_classes(k)) for k in (3, 4, 5)] == [2, 6, 21]


@pytest.mark.parametrize("k", [3, 4, 5])
def test_esu_census_vs_bruteforce(orc, k):
    g = gg.gnp(9, 0.45, seed=k)
    cen = orc.motif_census(G(orc, g), k)
    for rep, c in cen.items():
        assert c == brute.induced_subsets_count(g, k, orc.class_edges(k, rep))


def test_esu_census_all_graphs_on_5_vertices(orc):
    # every labelled graph on 5 vertices: census of connected 4-sets equals
    # the k-subset definition (checks ESU's each-set-once property exhaustively)
    for i, g in enumerate(gg.all_graphs(5)):
        if i % 37:
            continue
        cen = orc.motif_census(G(orc, g), 4)
        for rep, c in cen.items():
            assert c == brute.induced_subsets_count(g, 4, orc.class_edges(4, rep))


def test_closed_form_route_vs_census(orc):
    og = G(orc, gg.chung_lu(3000, 15000, 2.1, 150.0, seed=5))
    cf = orc.induced4_closed_form(og)
    cen = orc.motif_census(og, 4)
    for name, edges in orc.FOUR_NAMES.items():
        assert cf[name] == cen[orc.canonical_of_edges(4, edges)], name
        assert cf[name] == orc.count(og, {"k": 4, "edges": edges, "induced": True}), name


def test_inversion_matrix_known_rows(orc):
    c = orc.spanning_copies(4)
    rep = {n: orc.canonical_of_edges(4, e) for n, e in orc.FOUR_NAMES.items()}
    # textbook coefficients: spanning copies of P in Q
    assert c[(rep["diamond"], rep["clique"])] == 6
    assert c[(rep["paw"], rep["diamond"])] == 4 and c[(rep["paw"], rep["clique"])] == 12
    assert c[(rep["cycle"], rep["diamond"])] == 1 and c[(rep["cycle"], rep["clique"])] == 3
    assert c[(rep["path"], rep["paw"])] == 2 and c[(rep["path"], rep["cycle"])] == 4
    assert c[(rep["path"], rep["diamond"])] == 6 and c[(rep["path"], rep["clique"])] == 12
    assert c[(rep["star"], rep["paw"])] == 1 and c[(rep["star"], rep["diamond"])] == 2
    assert c[(rep["star"], rep["clique"])] == 4


@pytest.mark.parametrize("k", [4, 5])
def test_star_row_invariant(orc, k):
    og = G(orc, gg.rmat(9, 3000, seed=4))
    cen = orc.motif_census(og, k)
    assert orc.star_row_invariant(k, cen) == orc.degree_choose_sum(og, k - 1)


# ------------------------------------------------- anti-vertex special cases

@pytest.mark.parametrize("n", [4, 5, 7])
def test_p7_zero_in_complete(orc, n):
    assert orc.count(G(orc, gg.complete(n)), P7) == 0


def test_p7_counts_isolated_triangles(orc):
    g = gg.disjoint_union(*[gg.complete(3)] * 5, gg.complete(4))
    # the K4 contributes no triangle that avoids a 4-clique
    assert orc.count(G(orc, g), P7) == 5


def test_pd_degree_two_middle(orc):
    # p_d: middle vertex of degree exactly 2; a cycle C_n has n such paths,
    # a star with >= 3 leaves has none
    assert orc.count(G(orc, gg.cycle(7)), PD) == 7
    assert orc.count(G(orc, gg.star(5)), PD) == 0
    assert orc.count(G(orc, gg.path(6)), PD) == 4


def test_p8_induced_diamond(orc):
    assert orc.count(G(orc, gg.complete(4)), P8) == 0
    n, u, v = gg.complete(4)
    keep = ~((u == 0) & (v == 2))
    assert orc.count(G(orc, (n, u[keep], v[keep])), P8) == 1


def test_valid_maps_brute_force(orc):
    """The oracle's valid-map count (no symmetry breaking) equals the number of
    injective maps that satisfy every match condition, listed exhaustively
    (Sec. 2.1 and Sec. 3.1), on tiny graphs with and without anti-edges and
    anti-vertices."""
    for seed in (3, 4, 5):
        g = gg.gnp(9, 0.5, seed=seed)
        og = G(orc, g)
        for spec in (CLIQUE(3), STAR(4), DIAMOND, PAW, P8, PA, P7, PD, PE):
            assert orc.valid_maps(og, spec) == len(brute.canonical_maps(g, spec)), (seed, spec)


def test_valid_maps_from_partition_and_brute_force(orc):
    """valid_maps_from counts the valid maps whose pattern vertex 0 lands in
    the given roots: over a partition of V it sums to valid_maps, and on a
    tiny graph it equals the brute-force maps with img[0] in the roots."""
    g = gg.chung_lu(300, 1500, 2.1, 40.0, seed=17)
    og = G(orc, g)
    rng = np.random.Generator(np.random.PCG64(5))
    parts = np.array_split(rng.permutation(og.n).astype(np.int32), 7)
    for spec in (CLIQUE(3), PATH(4), P8, P7):
        total = orc.valid_maps(og, spec)
        assert sum(orc.valid_maps_from(og, spec, p) for p in parts) == total, spec
        assert orc.valid_maps_from(og, spec, np.zeros(0, np.int32)) == 0
    t = gg.gnp(9, 0.55, seed=8)
    ot = G(orc, t)
    for spec in (CLIQUE(3), STAR(4), P8, PD):
        maps = brute.canonical_maps(t, spec)
        for roots in ([0], [1, 4, 7], list(range(9))):
            want = sum(1 for m in maps if m[0] in roots)
            assert orc.valid_maps_from(ot, spec, np.array(roots, np.int32)) == want, (spec, roots)

def test_noninduced5_closed_forms(orc):
    """Each 5-vertex closed form equals the generic matcher's count of the
    same (edge-induced) pattern, and the row sum_Q c(P, Q) I(Q) of the ESU
    census, on graphs with hubs, triangles and isolated vertices."""
    graphs = [gg.gnp(11, 0.45, seed=s) for s in (1, 2)] + [
        gg.chung_lu(250, 1200, 2.1, 40.0, seed=23), gg.complete(7),
        gg.disjoint_union(gg.star(9), gg.complete(5), gg.cycle(6))]
    for g in graphs:
        og = G(orc, g)
        cf = orc.noninduced5_closed_forms(og)
        census = orc.motif_census(og, 5)
        rows = orc.noninduced5_rows(census)
        for name, edges in orc.FIVE_NONINDUCED.items():
            direct = orc.count(og, {"k": 5, "edges": edges})
            assert cf[name] == direct == rows[name], (name, cf[name], direct, rows[name])


def test_exists_equals_count_positive(orc):
    """Existence (a search stopped at the first valid map) is count > 0:
    cliques in complete multipartite graphs (K_k exists iff k <= parts),
    and patterns with anti-edges and anti-vertices on random graphs."""
    for parts, k in (([2] * 6, 6), ([2] * 6, 7), ([3] * 4, 4), ([3] * 4, 5)):
        og = G(orc, gg.complete_multipartite(parts))
        assert orc.exists(og, CLIQUE(k)) is (k <= len(parts))
    for seed in (1, 2, 3):
        og = G(orc, gg.gnp(12, 0.3, seed=seed))
        for spec in (CLIQUE(3), CLIQUE(4), P7, P8, PA, PD, STAR(5)):
            assert orc.exists(og, spec) is (orc.count(og, spec) > 0), (seed, spec)
