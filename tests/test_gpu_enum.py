"""GPU tests of enumeration at scale: root-task windows partition the
matches, the streamed callback form sees every match once through a small
device buffer (windows halved on overflow), stops early, and agrees with the
oracle's counts and valid maps."""
import sys

import numpy as np
import pytest

from oracle import brute
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


SPECS = [pt.clique(3), pt.clique(4), pt.star(3), pt.chain(4), pt.all_vertex_induced(4)[1],
         pt.PA_TWO_COMMON_FRIENDS, pt.P7_TRIANGLE_NO_K4, {"k": 2, "edges": [(0, 1)], "av": [[0, 1]]}]


@pytest.fixture(scope="module")
def g_small():
    return gg.chung_lu(1500, 6000, 2.1, 80.0, seed=51)


def _valid(g, spec, rows):
    adj = brute._adj_sets(*g)
    return all(brute.is_valid_map(adj, None, spec, tuple(int(x) for x in r)) for r in rows)


@pytest.mark.parametrize("si", range(len(SPECS)))
def test_windows_partition_matches(pg, orc, g_small, si):
    spec = SPECS[si]
    G = pg.load_graph(*g_small, device=0)
    plan = pg.plan_pattern(spec)
    want = orc.count(orc.Graph.from_tuple(g_small), spec)
    full, tot = pg.enumerate_matches(G, plan)
    assert tot == want == len(full)
    total = pg.root_tasks(G, plan)
    assert total in (G.m, G.n, G.m + G.n)
    cuts = sorted({0, total, *np.random.default_rng(si).integers(1, total, 5).tolist()})
    parts, n = [], 0
    for a, b in zip(cuts, cuts[1:]):
        rows, t = pg.enumerate_range(G, plan, a, b, cap=max(1, want))
        assert t == len(rows)
        parts.append(rows)
        n += t
    assert n == want
    got = np.concatenate(parts) if parts else np.zeros((0, spec["k"]), np.int32)
    assert sorted(map(tuple, got.tolist())) == sorted(map(tuple, full.tolist()))
    assert _valid(g_small, spec, got[:2000])


def test_streamed_callbacks_small_buffer(pg, orc, g_small):
    G = pg.load_graph(*g_small, device=0)
    for spec in (pt.clique(3), pt.chain(4), pt.star(3)):
        plan = pg.plan_pattern(spec)
        want = orc.count(orc.Graph.from_tuple(g_small), spec)
        seen = []
        say(f"match {spec['edges']} through a 997-row buffer ({want} matches)")
        n, stopped = pg.match(G, plan, lambda ids: seen.append(ids) and False, buffer_rows=997)
        assert not stopped and n == want == len(seen) == len(set(seen))
        full, _ = pg.enumerate_matches(G, plan)
        assert sorted(seen) == sorted(map(tuple, full.tolist()))


def test_streamed_stop(pg, g_small):
    G = pg.load_graph(*g_small, device=0)
    plan = pg.plan_pattern(pt.chain(4))
    calls = []

    def fn(ids):
        calls.append(ids)
        return len(calls) >= 2500

    n, stopped = pg.match(G, plan, fn, buffer_rows=1000)
    assert stopped and n == 2500 == len(calls)


def test_window_errors(pg, g_small):
    G = pg.load_graph(*g_small, device=0)
    plan = pg.plan_pattern(pt.clique(3))
    total = pg.root_tasks(G, plan)
    for a, b in ((5, 5), (-1, 3), (0, total + 1)):
        with pytest.raises(pg.PGError):
            pg.enumerate_range(G, plan, a, b, cap=10)


def test_enumerate_at_workload_size(pg, orc):
    """K4 and triangles of the six-motif Chung-Lu workload into one device
    buffer: every row valid, no two rows on one vertex set, totals equal to
    the oracle's counts."""
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "expected.json")) as f:
        w = json.load(f)["workloads"]["chunglu_100k_1m"]
    g = gg.workload("chunglu_100k_1m")
    G = pg.load_graph(*g, device=0)
    k4 = w["induced4"][str(orc.canonical_of_edges(4, pt.clique(4)["edges"]))]["count"]
    for spec, want in ((pt.clique(3), w["triangle"]), (pt.clique(4), k4)):
        say(f"enumerate K{spec['k']} on chunglu_100k_1m: {want} rows")
        rows, tot = pg.enumerate_matches(G, pg.plan_pattern(spec), cap=want)
        assert tot == want == len(rows)
        perm = G.perm
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm), dtype=perm.dtype)
        # every row: distinct vertices, every pattern edge an edge of the
        # graph (looked up in the sorted edge keys), and no two rows on the
        # same vertex set (a clique has one match per set)
        rp, col = G.csr()
        r = inv[rows].astype(np.int64)
        n = np.int64(G.n)
        ekeys = np.repeat(np.arange(G.n, dtype=np.int64), np.diff(rp)) * n + col.astype(np.int64)
        for a in range(spec["k"]):
            for b in range(a + 1, spec["k"]):
                key = r[:, a] * n + r[:, b]
                pos = np.minimum(np.searchsorted(ekeys, key), len(ekeys) - 1)
                assert np.all(ekeys[pos] == key), (a, b)
        canon = np.sort(r, axis=1)
        order = np.lexsort(canon.T[::-1])
        canon = canon[order]
        assert np.all(np.any(canon[1:] != canon[:-1], axis=1))
