"""Host-side tests of libpg (no GPU needed): the C ABI loads and exports
every declared symbol, the plan compiler reproduces the paper's worked
example and textbook symmetry counts, and the programs it emits -- run by
a slow literal interpreter -- give the oracle's counts and match sets."""
import itertools
import math
import os
import re

import numpy as np
import pytest

from oracle import brute
from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import patterns as pt
from paper_2004_02369_amd import pg
from tests.plan_interp import interp_count, interp_enumerate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(pg.LIB_PATH):
        from paper_2004_02369_amd import build
        build.build()


def header_functions(prefix="pg_", header=None):
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h") and (header is None or fn == header):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\**\s*(" + prefix + r"\w+)\s*\(", txt, flags=re.M))
    return names


def test_abi_exports_every_declared_symbol():
    names = header_functions()
    assert {"pg_load_graph", "pg_count", "pg_enumerate", "pg_match", "pg_exists", "pg_last_error"} <= names
    L = pg.lib()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(pg.EXPORTS) == names


def test_rowbench_exports_every_declared_symbol():
    from paper_2004_02369_amd import rowbench
    names = header_functions("rb_", "rowbench.h")
    assert {"rb_stream_read", "rb_flush", "rb_intersect", "rb_last_error"} == names == set(rowbench.EXPORTS)
    L = rowbench.lib()
    for n in sorted(names):
        assert hasattr(L, n), n


# ------------------------------------------------------------ worked example

DIAMOND = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3)]}   # u1..u4 = 0..3, chord u2-u4


def test_diamond_plan_matches_paper():
    """Sec. 4.1: partial order u1 < u3, u2 < u4; core {u2, u4}; one matching order."""
    info = pg.plan_pattern(DIAMOND).info()
    assert sorted(info["order"]) == [(0, 2), (1, 3)]
    assert info["core"] == [1, 3]
    assert info["n_matching_orders"] == 1
    assert info["aut"] == 4


@pytest.mark.parametrize("spec,aut", [
    (pt.clique(3), 6), (pt.clique(4), 24), (pt.clique(5), 120), (pt.clique(14), math.factorial(14)),
    (pt.star(3), 2), (pt.star(4), 6), (pt.star(5), 24), (pt.chain(4), 2), (pt.chain(6), 2),
    ({"k": 5, "edges": [(i, (i + 1) % 5) for i in range(5)]}, 10), (DIAMOND, 4),
    ({"k": 4, "edges": [(0, 1), (1, 2), (2, 0), (0, 3)]}, 2),
    (pt.P7_TRIANGLE_NO_K4, 6), (pt.P8_INDUCED_DIAMOND, 4), (pt.PA_TWO_COMMON_FRIENDS, 4),
])
def test_aut_and_orbit_product(spec, aut, orc):
    info = pg.plan_pattern(spec).info()
    assert info["aut"] == aut
    assert math.prod(info["orbit_size"]) == aut
    if spec["k"] <= 8:
        assert orc.aut(spec) == aut


def test_plan_time_small():
    for spec in pt.all_vertex_induced(5) + [pt.clique(14)]:
        assert pg.plan_pattern(spec).info()["plan_ms"] < 50.0


def test_generator_cardinalities():
    assert [len(pt.all_vertex_induced(k)) for k in (2, 3, 4, 5)] == [1, 2, 6, 21]
    assert len(pt.all_edge_induced(3)) == 3
    assert len(pt.all_edge_induced(2)) == 1


def _min_connected_cover_size(spec):
    k = spec["k"]
    E = {tuple(sorted(e)) for e in spec["edges"]}
    A = {tuple(sorted(e)) for e in spec.get("anti", []) or []}
    if spec.get("induced"):
        A |= {p for p in itertools.combinations(range(k), 2) if p not in E}
    for s in range(1, k + 1):
        for S in itertools.combinations(range(k), s):
            S = set(S)
            if any(a not in S and b not in S for a, b in E | A):
                continue
            seen, todo = {min(S)}, [min(S)]
            while todo:
                x = todo.pop()
                for a, b in E:
                    for u, w in ((a, b), (b, a)):
                        if u == x and w in S and w not in seen:
                            seen.add(w)
                            todo.append(w)
            if seen == S:
                return s
    return k


PLAN_PATTERNS = (pt.all_vertex_induced(3) + pt.all_vertex_induced(4) + pt.all_vertex_induced(5)
                 + [pt.clique(k) for k in (3, 4, 5, 6)] + [pt.star(k) for k in (2, 3, 4, 5)]
                 + [pt.chain(k) for k in (3, 4, 5)] + pt.all_edge_induced(3) + pt.all_edge_induced(4)
                 + [DIAMOND, pt.P7_TRIANGLE_NO_K4, pt.P8_INDUCED_DIAMOND, pt.PA_TWO_COMMON_FRIENDS,
                    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(0, 2)]},
                    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "anti": [(0, 2)]},
                    {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[1]]},
                    {"k": 2, "edges": [(0, 1)], "av": [[0, 1]]},
                    {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "av": [[0, 2]]},
                    {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0, 2], [1]]},
                    {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "av": [[1, 2, 3]]},
                    {"k": 5, "edges": [(0, 1), (1, 2), (2, 3), (3, 4)], "av": [[0, 4]]}])


@pytest.mark.parametrize("pi", range(len(PLAN_PATTERNS)))
def test_core_is_minimum_connected_cover(pi):
    spec = PLAN_PATTERNS[pi]
    info = pg.plan_pattern(spec).info()
    assert info["core_size"] == _min_connected_cover_size(spec)


@pytest.mark.parametrize("pi", range(len(PLAN_PATTERNS)))
@pytest.mark.parametrize("mode", [pg.PG_PLAN_LINEAR_EXT, pg.PG_PLAN_PARTIAL_ORDER])
def test_programs_count_like_oracle(pi, mode, orc):
    spec = PLAN_PATTERNS[pi]
    plan = pg.plan_pattern(spec, mode=mode)
    progs = plan.programs()
    for seed in (1, 2):
        g = gg.gnp(9, 0.5, seed=seed + 10 * pi)
        expect = orc.count(orc.Graph.from_tuple(g), spec)
        assert interp_count(g, progs) == expect, (spec, seed)


def _orbit_key(row, auts):
    return min(tuple(row[p[i]] for i in range(len(row))) for p in auts)


def _typed_auts(spec):
    k = spec["k"]
    out = []
    for pm in itertools.permutations(range(k)):
        sub = {"k": k, "edges": spec["edges"], "anti": spec.get("anti"), "induced": spec.get("induced"),
               "av": spec.get("av"), "labels": spec.get("labels")}
        img = [None] * k
        for i in range(k):
            img[i] = pm[i]
        if brute.is_valid_map(_pattern_as_graph(sub), None, sub, tuple(img)):
            out.append(pm)
    return out


def _pattern_as_graph(spec):
    k = spec["k"]
    adj = [set() for _ in range(k)]
    for a, b in spec["edges"]:
        adj[a].add(b)
        adj[b].add(a)
    return adj


@pytest.mark.parametrize("pi", range(len(PLAN_PATTERNS)))
def test_enum_programs_one_per_orbit(pi, orc):
    spec = PLAN_PATTERNS[pi]
    if spec.get("av"):
        pytest.skip("orbit keys below only cover patterns without anti-vertices")
    plan = pg.plan_pattern(spec)
    progs = plan.programs(enum_mode=True)
    g = gg.gnp(8, 0.55, seed=pi)
    rows = interp_enumerate(g, progs, spec["k"])
    adj = brute._adj_sets(*g)
    for r in rows:
        assert brute.is_valid_map(adj, None, spec, r)
    auts = [p for p in itertools.permutations(range(spec["k"]))
            if all(((p[b] in _pattern_as_graph(spec)[p[a]]) == (b in _pattern_as_graph(spec)[a]))
                   for a, b in itertools.combinations(range(spec["k"]), 2))]
    # orbits under the typed automorphisms: compare via the oracle's count
    assert len(rows) == orc.count(orc.Graph.from_tuple(g), spec)
    assert len(set(rows)) == len(rows)
    if not spec.get("anti") and not spec.get("induced"):
        keys = {_orbit_key(r, auts) for r in rows}
        assert len(keys) == len(rows)


def test_labelled_programs(orc):
    rng = np.random.Generator(np.random.PCG64(5))
    for seed in range(4):
        g = gg.gnp(9, 0.55, seed=seed)
        lab = rng.integers(0, 2, 9).astype(np.int16)
        og = orc.Graph.from_tuple(g, lab)
        for spec in ({"k": 3, "edges": [(0, 1), (1, 2)], "labels": [0, 1, 0]},
                     {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "labels": [1, 1, 0]},
                     {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [1, 0, 0, 1]},
                     {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0, 2]], "labels": [0, -1, 1], "av_labels": [1]}):
            assert interp_count(g, pg.plan_pattern(spec).programs(), labels=lab) == orc.count(og, spec)


def _random_labelled_pattern(rng, k):
    """A connected k-vertex pattern (random spanning tree plus extra edges),
    labels drawn from {-1, 0, 1, 2} so that both repeated and distinct
    labels occur; vertex-induced one time in four."""
    edges = {(int(rng.integers(0, v)), v) for v in range(1, k)}
    for a, b in itertools.combinations(range(k), 2):
        if rng.random() < 0.2:
            edges.add((a, b))
    spec = {"k": k, "edges": sorted(edges), "labels": [int(x) for x in rng.integers(-1, 3, k)]}
    if rng.random() < 0.25:
        spec["induced"] = True
    return spec


FACTOR_SHAPES = [
    # (spec, anchor, factor group sizes of every count program)
    ({"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [1, 0, 2, 3]}, None, [1, 1]),
    ({"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [1, 0, 0, 1]}, None, [1]),
    ({"k": 5, "edges": [(0, 1), (0, 2), (0, 3), (0, 4)], "labels": [0, 1, 1, 2, 3]}, 1, [1, 1]),
    ({"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [0, 1, 2, 3]}, None, [1]),
    ({"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [0, 1, 2, 3]}, 1, [1]),
    # the two ends may be one vertex (same label, or one unlabelled): enumerated
    ({"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [0, 1, 1, 0]}, None, []),
    ({"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [-1, 1, 2, 3]}, None, []),
    ({"k": 4, "edges": [(0, 1), (0, 2), (0, 3)]}, None, []),
]


@pytest.mark.parametrize("fi", range(len(FACTOR_SHAPES)))
def test_factor_groups_chosen(fi):
    """Independent groups (a label no other non-core vertex can carry)
    become factors of the count programs; enumeration never uses them."""
    spec, anchor, want = FACTOR_SHAPES[fi]
    plan = pg.plan_pattern(spec, anchor=anchor)
    for prog in plan.programs():
        assert sorted(f["group"] for f in prog["factors"]) == want, prog
        F = len(prog["levels"]) - 1
        for f in prog["factors"]:
            assert f["label"] >= 0 and not f["avs"]
            assert f["isect"] < (1 << F) and f["excl"] < (1 << F)
    assert all(not p["factors"] for p in plan.programs(enum_mode=True))


def test_factor_programs_count_like_oracle(orc):
    """Random labelled patterns, plain and anchored: the count programs
    (with their products of independent groups) give the oracle's count
    and valid maps / |stabiliser of the anchor|; the interpreter also
    asserts that no two sets of a product share a vertex."""
    rng = np.random.Generator(np.random.PCG64(77))
    n_fac = 0
    for trial in range(60):
        k = int(rng.integers(3, 6))
        spec = _random_labelled_pattern(rng, k)
        g = gg.gnp(10, 0.5, seed=900 + trial)
        lab = rng.integers(0, 3, 10).astype(np.int16)
        og = orc.Graph.from_tuple(g, lab)
        plan = pg.plan_pattern(spec)
        n_fac += sum(len(p["factors"]) for p in plan.programs())
        assert interp_count(g, plan.programs(), labels=lab) == orc.count(og, spec), (trial, spec)
        valid = orc.valid_maps(og, spec)
        for u in range(k):
            ap = pg.plan_pattern(spec, anchor=u)
            n_fac += sum(len(p["factors"]) for p in ap.programs())
            assert interp_count(g, ap.programs(), labels=lab) == valid // ap.info()["aut"], (trial, spec, u)
    assert n_fac > 20


def test_partial_order_gives_one_map_per_orbit(orc):
    """Grochow-Kellis: among the valid maps, exactly count() satisfy the
    partial order (the PRG-U relation read backwards)."""
    g = gg.gnp(8, 0.6, seed=3)
    adj = brute._adj_sets(*g)
    for spec in [DIAMOND, pt.clique(4), pt.star(4), pt.chain(4), pt.P8_INDUCED_DIAMOND, pt.P7_TRIANGLE_NO_K4,
                 {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(0, 2)]}]:
        order = pg.plan_pattern(spec).info()["order"]
        maps = brute.canonical_maps(g, spec)
        kept = [m for m in maps if all(m[a] < m[b] for a, b in order)]
        assert len(kept) == orc.count(orc.Graph.from_tuple(g), spec)
        assert len(maps) == len(kept) * orc.aut(spec)


@pytest.mark.parametrize("bad", [
    {"k": 1, "edges": []},
    {"k": 17, "edges": [(i, i + 1) for i in range(16)]},
    {"k": 4, "edges": [(0, 1), (2, 3)]},                       # disconnected
    {"k": 3, "edges": [(0, 1), (1, 2)], "anti": [(0, 1)]},     # edge and anti-edge
    {"k": 3, "edges": [(0, 1), (0, 5)]},                       # id out of range
    {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[]]},           # anti-vertex without anti-edges
])
def test_invalid_patterns_rejected(bad):
    with pytest.raises(pg.PGError) as e:
        pg.plan_pattern(bad)
    assert e.value.status == pg.PG_EINVAL


def test_anti_vertex_with_true_edge_rejected():
    d, keep = pg.pattern_desc({"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0]]})
    d.edges[2].type = pg.PG_EDGE
    import ctypes
    h = ctypes.c_void_p()
    assert pg.lib().pg_plan_pattern(ctypes.byref(d), ctypes.byref(h)) == pg.PG_EINVAL


ANCHOR_PATTERNS = [s for s in PLAN_PATTERNS if s["k"] <= 5]


@pytest.mark.parametrize("pi", range(0, len(ANCHOR_PATTERNS), 2))
def test_anchored_programs_reach_every_domain_vertex(pi, orc):
    """An anchored plan (domains for MNI): its count programs count valid
    maps / |stabiliser of the anchor| and its enumeration programs reach
    every data vertex of the anchor's domain."""
    spec = ANCHOR_PATTERNS[pi]
    g = gg.gnp(9, 0.5, seed=300 + pi)
    og = orc.Graph.from_tuple(g)
    valid = orc.valid_maps(og, spec)
    _, members = orc.domains(og, spec, members=True)
    for u in range(spec["k"]):
        plan = pg.plan_pattern(spec, anchor=u)
        info = plan.info()
        assert info["anchor"] == u and u in info["core"]
        assert valid % info["aut"] == 0
        assert interp_count(g, plan.programs()) == valid // info["aut"], (spec, u)
        # the anchor is a root vertex (level 0 or 1) of every program
        for prog in plan.programs() + plan.programs(enum_mode=True):
            assert u in [L["pv"] for L in prog["levels"][:2]], (spec, u)
        rows = interp_enumerate(g, plan.programs(enum_mode=True), spec["k"])
        assert {r[u] for r in rows} == set(np.flatnonzero(members[u]).tolist()), (spec, u)


def test_anchored_stabiliser_order():
    # the anchor's stabiliser: K4 -> 3!, a 3-star's centre -> 3!, a leaf -> 2!
    assert pg.plan_pattern(pt.clique(4), anchor=2).info()["aut"] == 6
    star = pt.star(4)
    assert pg.plan_pattern(star, anchor=0).info()["aut"] == 6
    assert pg.plan_pattern(star, anchor=3).info()["aut"] == 2
    assert pg.plan_pattern(pt.chain(4), anchor=0).info()["aut"] == 1
    with pytest.raises(pg.PGError):
        pg.plan_pattern(pt.clique(3), anchor=3)


def test_clique_and_induced_clique_compile_to_identical_programs():
    """A clique has no non-adjacent pair, so its vertex-induced form adds no
    anti-edge and compiles to the same programs (pg_count_ex then counts the
    two once per launch); a pattern with a non-adjacent pair does not."""
    for k in (3, 4, 5):
        a = pg.plan_pattern(pt.clique(k))
        b = pg.plan_pattern(pt.clique(k, induced=True))
        assert a.programs() == b.programs()
    s = pg.plan_pattern(pt.star(4))
    si = pg.plan_pattern(pt.star(4, induced=True))
    assert s.programs() != si.programs()
