"""GPU parity of MNI domains (pg_domain_sizes) against the oracle's domains,
over every launch variant, and of the FSM loop driven by the GPU against the
same loop driven by the oracle."""
import sys

import numpy as np
import pytest

from paper_2004_02369_amd import fsm
from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import patterns as pt

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pg():
    import torch
    assert torch.cuda.is_available()
    from paper_2004_02369_amd import pg as _pg
    _pg.lib()
    return _pg


SPECS = [
    {"k": 2, "edges": [(0, 1)], "labels": [0, 1]},
    {"k": 2, "edges": [(0, 1)], "labels": [2, 2]},
    {"k": 3, "edges": [(0, 1), (0, 2)], "labels": [1, 0, 2]},
    {"k": 3, "edges": [(0, 1), (0, 2)], "labels": [0, 1, 1]},
    {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "labels": [0, 0, 1]},
    {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)]},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [0, 1, 1, 2]},
    {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [1, 0, 0, 3]},
    {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)]},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(1, 3)]},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "induced": True},
    {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (0, 2)], "labels": [-1, 1, -1, 0]},
    {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "av": [[0, 1, 2]]},
    {"k": 5, "edges": [(0, 1), (1, 2), (2, 3), (3, 4)], "labels": [0, 1, 2, 1, 0]},
    {"k": 5, "edges": [(0, 1), (0, 2), (0, 3), (0, 4)], "labels": [0, 1, 1, 1, 2]},
]


@pytest.fixture(scope="module")
def case(orc):
    g = gg.chung_lu(3000, 12000, 2.2, 150.0, seed=41)
    lab = np.random.default_rng(42).integers(0, 4, 3000).astype(np.int16)
    og = orc.Graph.from_tuple(g, lab)
    want = [orc.domains(og, s) for s in SPECS]
    return g, lab, want


@pytest.mark.parametrize("knobs", [{}, {"hub_min_degree": -1}, {"chunk": 1, "batch_max_avg": 4},
                                   {"flags": 4, "chunk": 3}, {"grid_waves": 29}])
def test_domain_sizes_match_oracle(pg, case, knobs):
    g, lab, want = case
    G = pg.load_graph(*g, labels=lab, device=0)
    jobs = [(i, u) for i, s in enumerate(SPECS) for u in range(s["k"])]
    plans = [pg.plan_pattern(SPECS[i], anchor=u) for i, u in jobs]
    say(f"{len(plans)} anchored plans, knobs {knobs}")
    got = {}
    for s in range(0, len(plans), 64):
        sizes = pg.domain_sizes(G, plans[s:s + 64], **knobs)
        for (i, u), sz in zip(jobs[s:s + 64], sizes):
            got[(i, u)] = sz
    for (i, u) in jobs:
        assert got[(i, u)] == want[i][u], (SPECS[i], u)


def test_domain_counts_are_maps_over_stabiliser(pg, orc, case):
    g, lab, _ = case
    G = pg.load_graph(*g, labels=lab, device=0)
    og = orc.Graph.from_tuple(g, lab)
    for s in SPECS[:9]:
        valid = orc.valid_maps(og, s)
        plans = [pg.plan_pattern(s, anchor=u) for u in range(s["k"])]
        counts = pg.count(G, plans)
        for p, c in zip(plans, counts):
            assert c * p.info()["aut"] == valid, s


def test_special_graphs(pg):
    for n in (5, 9):
        G = pg.load_graph(*gg.complete(n), device=0)
        plans = [pg.plan_pattern(pt.clique(k), anchor=k - 1) for k in range(2, n + 2)]
        assert pg.domain_sizes(G, plans) == [n] * (n - 1) + [0]
    G = pg.load_graph(*gg.star(7), device=0)
    star = pt.star(4)
    assert pg.domain_sizes(G, [pg.plan_pattern(star, anchor=u) for u in range(4)]) == [1, 7, 7, 7]
    with pytest.raises(pg.PGError):
        pg.domain_sizes(G, [pg.plan_pattern(star)])


def test_fsm_loop_gpu_equals_oracle(pg, orc):
    g = gg.chung_lu(2000, 8000, 2.2, 60.0, seed=43)
    lab = np.random.default_rng(44).integers(0, 3, 2000).astype(np.int16)
    og = orc.Graph.from_tuple(g, lab)
    G = pg.load_graph(*g, labels=lab, device=0)
    for threshold in (60, 400):
        say(f"FSM, 3 edges, support {threshold}")
        ref, _ = fsm.mine(lambda c: [orc.mni_support(og, p.spec()) for p in c], [0, 1, 2], threshold, 3)
        got, stats = fsm.mine(fsm.gpu_support(G, pg), [0, 1, 2], threshold, 3)
        assert got == ref
        assert sum(len(v) for v in got.values()) > 0


def test_domains_at_labelled_workload_size(pg, orc):
    """Full size of the labelled workload (Chung-Lu n = 10^6, 10^7 edges,
    16 labels): domains of seeded random labelled 1- to 3-edge patterns,
    every anchor, against the oracle."""
    import random
    n, src, dst, lab = gg.labelled_workload("chunglu_1m_10m_l16")
    og = orc.Graph(n, src, dst, lab)
    G = pg.load_graph(n, src, dst, labels=lab, device=0)
    rng = random.Random(61)
    shapes = [(2, [(0, 1)]), (3, [(0, 1), (1, 2)]), (3, [(0, 1), (1, 2), (0, 2)]),
              (4, [(0, 1), (1, 2), (2, 3)]), (4, [(0, 1), (0, 2), (0, 3)])]
    specs = []
    for i in range(40):
        k, edges = shapes[i % len(shapes)]
        # few distinct labels per pattern, so symmetric cases occur too
        pool = rng.sample(range(16), 2)
        specs.append({"k": k, "edges": edges, "labels": [rng.choice(pool) for _ in range(k)]})
    jobs = [(i, u) for i, s in enumerate(specs) for u in range(s["k"])]
    plans = [pg.plan_pattern(specs[i], anchor=u) for i, u in jobs]
    say(f"{len(plans)} anchored plans on chunglu_1m_10m_l16")
    got = []
    for s0 in range(0, len(plans), 64):
        got += pg.domain_sizes(G, plans[s0:s0 + 64])
    want = {i: orc.domains(og, s) for i, s in enumerate(specs)}
    for (i, u), g_ in zip(jobs, got):
        assert g_ == want[i][u], (specs[i], u)


def _random_labelled(rng, k):
    edges = {(int(rng.integers(0, v)), v) for v in range(1, k)}
    for a in range(k):
        for b in range(a + 1, k):
            if rng.random() < 0.2:
                edges.add((a, b))
    # mostly distinct labels (so independent groups occur), a few unlabelled
    labels = [int(x) if rng.random() > 0.1 else -1 for x in rng.integers(0, 4, k)]
    spec = {"k": k, "edges": sorted(edges), "labels": labels}
    if rng.random() < 0.25:
        spec["induced"] = True
    return spec


@pytest.mark.parametrize("knobs", [{}, {"flags": 4, "chunk": 1}, {"batch_max_avg": 4, "hub_min_degree": -1}])
def test_products_of_independent_groups(pg, orc, case, knobs):
    """Random labelled patterns whose count programs multiply independent
    groups (factor nodes), batched with plans that have none: counts,
    existence and domains against the oracle, over launch shapes that reach
    the root, set and flattened batches."""
    g, lab, _ = case
    og = orc.Graph.from_tuple(g, lab)
    G = pg.load_graph(*g, labels=lab, device=0)
    rng = np.random.Generator(np.random.PCG64(123))
    specs = [_random_labelled(rng, int(rng.integers(3, 6))) for _ in range(32)]
    plans = [pg.plan_pattern(s) for s in specs]
    n_fac = sum(bool(p["factors"]) for pl in plans for p in pl.programs())
    say(f"{len(specs)} random labelled patterns ({n_fac} count programs with factors), knobs {knobs}")
    assert n_fac >= 15
    want = [orc.count(og, s) for s in specs]
    assert pg.count(G, plans, **knobs) == want
    for s, p, w in zip(specs[:8], plans[:8], want[:8]):
        assert pg.exists(G, p) == (w > 0), s
    jobs = [(i, u) for i in range(0, len(specs), 3) for u in range(specs[i]["k"])]
    aplans = [pg.plan_pattern(specs[i], anchor=u) for i, u in jobs]
    dom = {i: orc.domains(og, specs[i]) for i in range(0, len(specs), 3)}
    sizes = []
    for s in range(0, len(aplans), 64):
        sizes += pg.domain_sizes(G, aplans[s:s + 64], **knobs)
    for (i, u), sz in zip(jobs, sizes):
        assert sz == dom[i][u], (specs[i], u)
