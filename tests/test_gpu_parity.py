"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit-exact.  Every test prints the case it runs before touching the GPU."""
import itertools
import math
import sys

import numpy as np
import pytest

from oracle import brute
from paper_2004_02369_amd import graphgen as gg
from paper_2004_02369_amd import patterns as pt
from tests.test_plan import PLAN_PATTERNS, DIAMOND

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def pg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2004_02369_amd import pg as _pg
    _pg.lib()
    return _pg


def G(pg, g, labels=None):
    return pg.load_graph(*g, labels=labels, device=0)


# ------------------------------------------------------------------ ingest

def test_ingest_degree_order_and_csr(pg, orc):
    g = gg.chung_lu(2000, 9000, 2.1, 150.0, seed=3)
    say("ingest chung_lu 2000/9000")
    Gd = G(pg, gg.dirty_copy(g, seed=1))
    og = orc.Graph.from_tuple(g)
    assert Gd.m == og.m
    rp, col = Gd.csr()
    deg = np.diff(rp)
    odeg = og.degrees()
    # ranks ascend by (degree, original id)
    perm = Gd.perm
    keys = list(zip(odeg[perm], perm))
    assert keys == sorted(keys)
    assert np.array_equal(deg, odeg[perm])
    # same graph: relabel the oracle's adjacency
    rank = np.empty_like(perm)
    rank[perm] = np.arange(len(perm))
    ooff, oadj = og.csr()
    for r in range(0, Gd.n, 97):
        v = perm[r]
        row = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(row) > 0)
        assert sorted(rank[oadj[ooff[v]:ooff[v + 1]]].tolist()) == row.tolist()


def test_ingest_rejects_out_of_range(pg):
    say("ingest out of range")
    with pytest.raises(pg.PGError) as e:
        pg.load_graph(5, np.array([0, 1]), np.array([1, 5]), device=0)
    assert e.value.status == pg.PG_EINVAL


# ------------------------------------------------------- tiny-graph parity

@pytest.mark.parametrize("pi", range(len(PLAN_PATTERNS)))
def test_tiny_parity_all_patterns(pg, orc, pi):
    spec = PLAN_PATTERNS[pi]
    for seed in (1, 2, 3):
        g = gg.gnp(14, 0.45, seed=seed + 31 * pi)
        say("tiny", pi, spec, seed)
        Gd = G(pg, g)
        want = orc.count(orc.Graph.from_tuple(g), spec)
        for mode in (pg.PG_PLAN_LINEAR_EXT, pg.PG_PLAN_PARTIAL_ORDER):
            assert pg.count(Gd, pg.plan_pattern(spec, mode=mode)) == want, (spec, seed, mode)


@pytest.mark.parametrize("pi", range(len(PLAN_PATTERNS)))
def test_medium_parity_all_patterns(pg, orc, pi):
    """Several tiles and ragged tails: a few hundred vertices, skewed degrees."""
    spec = PLAN_PATTERNS[pi]
    g = gg.chung_lu(400, 2400, 2.1, 60.0, seed=pi)
    say("medium", pi, spec)
    Gd = G(pg, g)
    want = orc.count(orc.Graph.from_tuple(g), spec)
    assert pg.count(Gd, pg.plan_pattern(spec)) == want


def test_labelled_parity(pg, orc):
    rng = np.random.Generator(np.random.PCG64(11))
    g = gg.chung_lu(600, 4000, 2.1, 80.0, seed=9)
    lab = rng.integers(0, 3, 600).astype(np.int16)
    say("labelled")
    Gd = G(pg, g, lab)
    og = orc.Graph.from_tuple(g, lab)
    for spec in ({"k": 3, "edges": [(0, 1), (1, 2)], "labels": [0, 1, 0]},
                 {"k": 3, "edges": [(0, 1), (1, 2), (0, 2)], "labels": [1, 1, 2]},
                 {"k": 4, "edges": [(0, 1), (0, 2), (0, 3)], "labels": [1, 0, 0, 2]},
                 {"k": 4, "edges": [(0, 1), (1, 2), (2, 3)], "labels": [-1, 1, 1, -1], "induced": True},
                 {"k": 3, "edges": [(0, 1), (1, 2)], "av": [[0, 2]], "labels": [0, -1, 1], "av_labels": [1]}):
        assert pg.count(Gd, pg.plan_pattern(spec)) == orc.count(og, spec), spec


# ---------------------------------------------------------- closed forms

def _esym(sizes, k):
    return sum(math.prod(c) for c in itertools.combinations(sizes, k))


def test_cliques_closed_forms(pg):
    for n, k in [(12, 3), (12, 5), (30, 4), (64, 4), (20, 8)]:
        say("K_n cliques", n, k)
        assert pg.count(G(pg, gg.complete(n)), pg.plan_pattern(pt.clique(k))) == math.comb(n, k)
    for sizes, k in [([3, 4, 5, 6], 4), ([2] * 7, 6), ([5, 5, 5], 3)]:
        say("multipartite", sizes, k)
        assert pg.count(G(pg, gg.complete_multipartite(sizes)), pg.plan_pattern(pt.clique(k))) == _esym(sizes, k)


def test_k256_and_bipartite(pg):
    say("K_256 triangles / K4")
    K = G(pg, gg.complete(256))
    assert pg.count(K, [pg.plan_pattern(pt.clique(3)), pg.plan_pattern(pt.clique(4))]) == \
        [math.comb(256, 3), math.comb(256, 4)]
    say("K_{300,300} 4-cycles / triangles")
    B = G(pg, gg.complete_multipartite([300, 300]))
    c4 = {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)]}
    assert pg.count(B, [pg.plan_pattern(c4), pg.plan_pattern(pt.clique(3))]) == [math.comb(300, 2) ** 2, 0]


def test_stars_degree_sums(pg, orc):
    g = gg.chung_lu(5000, 30000, 2.1, 600.0, seed=12)
    say("stars on chung_lu 5000/30000")
    Gd = G(pg, g)
    og = orc.Graph.from_tuple(g)
    for k in (3, 4, 5):
        assert pg.count(Gd, pg.plan_pattern(pt.star(k))) == orc.degree_choose_sum(og, k - 1)
    assert pg.count(Gd, pg.plan_pattern(pt.star(2))) == og.m


def test_hub_star_graph(pg):
    say("star graph hub degree n-1")
    S = G(pg, gg.star(4000))
    assert pg.count(S, pg.plan_pattern(pt.star(3))) == math.comb(4000, 2)
    assert pg.count(S, pg.plan_pattern(pt.star(3, induced=True))) == math.comb(4000, 2)
    assert pg.count(S, pg.plan_pattern(pt.clique(3))) == 0
    assert pg.count(S, pg.plan_pattern(pt.star(5))) == math.comb(4000, 4)


def test_choose_near_two_to_the_64(pg):
    """C(d, 4) for a 120,000-leaf star is about 8.6e18: exact in 64 bits
    although 4 * C(d, 4) is not, so the count must come back, not an
    overflow."""
    say("star(5) on a 120,000-leaf star")
    S = G(pg, gg.star(120000))
    want = math.comb(120000, 4)
    assert 2 ** 62 <= want < 2 ** 64
    assert pg.count(S, pg.plan_pattern(pt.star(5))) == want


def test_overflow_reported(pg):
    say("overflow")
    S = G(pg, gg.star(3000))
    with pytest.raises(pg.PGError) as e:
        pg.count(S, pg.plan_pattern(pt.star(16)))
    assert e.value.status == pg.PG_EOVERFLOW


def test_empty_and_degenerate_graphs(pg):
    say("degenerate graphs")
    E = pg.load_graph(10, np.zeros(0, np.int32), np.zeros(0, np.int32), device=0)
    assert pg.count(E, [pg.plan_pattern(pt.clique(3)), pg.plan_pattern(pt.star(3)),
                        pg.plan_pattern(pt.star(2))]) == [0, 0, 0]
    one = pg.load_graph(3, np.array([0]), np.array([2]), device=0)
    assert pg.count(one, [pg.plan_pattern(pt.star(2)), pg.plan_pattern(pt.star(3))]) == [1, 0]
    loops = pg.load_graph(4, np.array([0, 1, 1, 2, 3]), np.array([0, 2, 2, 1, 3]), device=0)
    assert loops.m == 1


# ------------------------------------------------- batching and schedules

def test_batched_equals_single_and_perturbations(pg, orc):
    g = gg.chung_lu(3000, 24000, 2.1, 300.0, seed=21)
    say("batched vs single, chung_lu 3000/24000")
    Gd = G(pg, g)
    specs = pt.all_vertex_induced(4) + [pt.clique(3), pt.star(3), pt.clique(4), DIAMOND, pt.P7_TRIANGLE_NO_K4,
                                        pt.P8_INDUCED_DIAMOND]
    plans = [pg.plan_pattern(s) for s in specs]
    batched = pg.count(Gd, plans)
    single = [pg.count(Gd, p) for p in plans]
    assert batched == single
    og = orc.Graph.from_tuple(g)
    assert batched == [orc.count(og, s) for s in specs]
    for grid, chunk, flags in [(1, 1, 0), (7, 3, 0), (64, 1000, 0), (300, 64, pg.PG_RUN_NO_MODE_B),
                               (2048, 16, pg.PG_RUN_COUNT_BYTES), (512, 64, pg.PG_RUN_NO_TASK_BATCH),
                               (100, 8, pg.PG_RUN_NO_TASK_BATCH | pg.PG_RUN_NO_MODE_B)]:
        say("perturbation", grid, chunk, flags)
        assert pg.count(Gd, plans, grid_waves=grid, chunk=chunk, flags=flags) == batched
    # intersection variants per degree bucket: bitmaps from several degrees
    # on, binary search below (or everywhere)
    for hub in (0, 32, 64, 1000, -1):
        say("variants", hub)
        assert pg.count(Gd, plans, hub_min_degree=hub) == batched


def test_identical_plans_counted_once(pg, orc):
    """K5 and the induced K5 compile to the same programs: a call holding
    both (and K5 twice, among other plans) runs them once and reports each
    its count, equal to the oracle's and to single launches."""
    g = gg.chung_lu(3000, 24000, 2.1, 300.0, seed=21)
    say("identical plans in one launch")
    Gd = G(pg, g)
    specs = [pt.clique(5), pt.clique(3), pt.all_vertex_induced(5)[-1], pt.clique(5), pt.star(3)]
    plans = [pg.plan_pattern(s) for s in specs]
    og = orc.Graph.from_tuple(g)
    want = [orc.count(og, s) for s in specs]
    assert want[0] == want[2] == want[3] > 0
    assert pg.count(Gd, plans) == want
    assert [pg.count(Gd, [p])[0] for p in plans] == want
    # the launch holds three distinct plans: its merge-model bytes are those of the three alone
    _, st_all = pg.count_ex(Gd, plans, flags=pg.PG_RUN_COUNT_BYTES)
    _, st_uniq = pg.count_ex(Gd, [plans[0], plans[1], plans[4]], flags=pg.PG_RUN_COUNT_BYTES)
    assert st_all["logical_bytes"] == st_uniq["logical_bytes"]


def test_merge_model_bytes_deterministic(pg):
    """Claims cover fixed task ranges, so the merge-model byte count of a
    launch is the same for every run and every grid size."""
    g = gg.chung_lu(3000, 24000, 2.1, 300.0, seed=21)
    say("merge-model bytes across grids")
    Gd = G(pg, g)
    plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
    seen = set()
    for grid in (64, 256, 1024, 0, 0):
        c, st = pg.count_ex(Gd, plans, grid_waves=grid, flags=pg.PG_RUN_COUNT_BYTES)
        seen.add(st["logical_bytes"])
    assert len(seen) == 1 and seen.pop() > 0


def test_wave_finish_times(pg):
    """PG_RUN_WAVE_TIMES changes no count and reports 0 <= first <= last
    finish, within the kernel's duration."""
    g = gg.chung_lu(3000, 24000, 2.1, 300.0, seed=21)
    say("wave finish times")
    Gd = G(pg, g)
    plans = [pg.plan_pattern(s) for s in pt.all_vertex_induced(4)]
    want = pg.count(Gd, plans)
    c, st = pg.count_ex(Gd, plans, flags=pg.PG_RUN_WAVE_TIMES)
    assert c == want
    assert 0 <= st["wave_done_first_ms"] <= st["wave_done_last_ms"] <= st["kernel_ms"] * 1.5 + 1.0


def test_relabelling_invariance(pg):
    g = gg.chung_lu(2500, 15000, 2.1, 250.0, seed=5)
    specs = pt.all_vertex_induced(4)
    plans = [pg.plan_pattern(s) for s in specs]
    base = pg.count(G(pg, g), plans)
    for seed in (1, 2):
        say("relabel", seed)
        assert pg.count(G(pg, gg.relabel(g, seed)), plans) == base


# ------------------------------------------------------ existence, matches

def test_clique_existence(pg):
    say("14-clique existence")
    yes = G(pg, gg.complete_multipartite([2] * 14))
    no = G(pg, gg.complete_multipartite([3] * 13))
    p14 = pg.plan_pattern(pt.clique(14))
    assert pg.exists(yes, p14) is True
    assert pg.exists(no, p14) is False
    assert pg.count(yes, p14) == 2 ** 14


def _orbit_keys(rows, spec):
    """One key per orbit of matches under the typed automorphisms (permutations
    keeping true edges, anti-edges, anti-vertex neighbourhoods and labels)."""
    k, E, A, av, labels, avl = brute._pattern_sets(spec)
    av_items = sorted((tuple(sorted(a)), l) for a, l in zip(av, avl))
    auts = []
    for p in itertools.permutations(range(k)):
        if any(labels[i] != labels[p[i]] for i in range(k)):
            continue
        if not all(((frozenset((p[a], p[b])) in E) == (frozenset((a, b)) in E)) and
                   ((frozenset((p[a], p[b])) in A) == (frozenset((a, b)) in A))
                   for a, b in itertools.combinations(range(k), 2)):
            continue
        if sorted((tuple(sorted(p[x] for x in a)), l) for a, l in zip(av, avl)) != av_items:
            continue
        auts.append(p)
    assert len(auts) == brute.typed_aut(spec)
    return {min(tuple(r[p[i]] for i in range(k)) for p in auts) for r in rows}


def test_enumerate_matches_orbits(pg, orc):
    g = gg.gnp(40, 0.3, seed=8)
    say("enumerate")
    Gd = G(pg, g)
    adj = brute._adj_sets(*g)
    for spec in (pt.clique(3), pt.star(4), DIAMOND, pt.chain(4), pt.clique(4), {"k": 4, "edges": [(0, 1), (1, 2), (2, 0), (0, 3)]},
                 pt.P8_INDUCED_DIAMOND, pt.PA_TWO_COMMON_FRIENDS, pt.star(4, induced=True), pt.chain(4, induced=True),
                 pt.P7_TRIANGLE_NO_K4, {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(0, 2)]}):
        plan = pg.plan_pattern(spec)
        rows, total = pg.enumerate_matches(Gd, plan)
        want = orc.count(orc.Graph.from_tuple(g), spec)
        assert total == want == len(rows) == pg.count(Gd, plan)
        for r in rows:
            assert brute.is_valid_map(adj, None, spec, tuple(int(x) for x in r))
        assert len({tuple(r) for r in rows.tolist()}) == len(rows)
        # one row per orbit of the typed pattern's automorphisms
        assert len(_orbit_keys(rows.tolist(), spec)) == len(rows), spec


def test_enumerate_capacity(pg):
    say("enumerate capacity")
    K = G(pg, gg.complete(20))
    rows, total = pg.enumerate_matches(K, pg.plan_pattern(pt.clique(3)), cap=100)
    assert total == math.comb(20, 3) and len(rows) == 100


def test_match_callback_and_stop(pg, orc):
    g = gg.gnp(30, 0.35, seed=4)
    say("match callback")
    Gd = G(pg, g)
    plan = pg.plan_pattern(pt.clique(3))
    seen = []
    n, stopped = pg.match(Gd, plan, lambda ids: seen.append(ids) and False)
    assert n == len(seen) == orc.count(orc.Graph.from_tuple(g), pt.clique(3)) and not stopped
    n2, stopped2 = pg.match(Gd, plan, lambda ids: True)
    assert n2 == 1 and stopped2


def test_anti_vertex_p7_medium(pg, orc):
    g = gg.chung_lu(3000, 20000, 2.1, 300.0, seed=31)
    say("p7 anti-vertex")
    want = orc.count(orc.Graph.from_tuple(g), pt.P7_TRIANGLE_NO_K4)
    assert pg.count(G(pg, g), pg.plan_pattern(pt.P7_TRIANGLE_NO_K4)) == want
    assert pg.count(G(pg, gg.complete(9)), pg.plan_pattern(pt.P7_TRIANGLE_NO_K4)) == 0


def test_share_groups_equal_oracle(pg, orc):
    """Plans whose level-2 nodes apply one set operation over different id
    ranges share one materialisation per root task (share groups): counts
    with sharing, without it (PG_RUN_NO_SHARE), one launch per plan, and
    under grids, claims and batching limits that send parents down the
    one-at-a-time path, all equal the oracle's."""
    g = gg.chung_lu(900, 6000, 2.1, 70.0, seed=44)
    say("share groups, chung_lu 900/6000")
    Gd = G(pg, g)
    specs = ([pt.clique(3), pt.star(3), pt.star(3, induced=True), pt.clique(4), pt.clique(5)]
             + list(pt.EDGE_CORE_5.values()) + pt.all_vertex_induced(4) + [DIAMOND, pt.P8_INDUCED_DIAMOND])
    plans = [pg.plan_pattern(s) for s in specs]
    og = orc.Graph.from_tuple(g)
    want = [orc.count(og, s) for s in specs]
    assert pg.count(Gd, plans) == want
    assert pg.count(Gd, plans, flags=pg.PG_RUN_NO_SHARE) == want
    assert [pg.count(Gd, p) for p in plans] == want
    for grid, chunk, bma, flags in [(1, 1, 0, 0), (37, 5, 1, 0), (512, 64, 2, 0), (64, 16, 0, pg.PG_RUN_NO_MODE_B),
                                    (256, 8, 0, pg.PG_RUN_COUNT_BYTES), (128, 4, 0, pg.PG_RUN_NO_TASK_BATCH)]:
        say("share perturbation", grid, chunk, bma, flags)
        assert pg.count(Gd, plans, grid_waves=grid, chunk=chunk, batch_max_avg=bma, flags=flags) == want
    # existence of a share-group member stops early and finds the same answer
    assert pg.exists(Gd, pg.plan_pattern(pt.EDGE_CORE_5["book3"])) is (want[specs.index(pt.EDGE_CORE_5["book3"])] > 0)


def test_task_windows_partition_the_counts(pg, orc):
    """Counts over root-task windows that partition a launch's tasks (edges
    first, then vertices) sum to the full counts, through the synchronous
    call and through jobs; windows outside the launch are refused."""
    import torch
    g = gg.chung_lu(2000, 14000, 2.1, 200.0, seed=9)
    say("task windows, chung_lu 2000/14000")
    Gd = G(pg, g)
    specs = pt.all_vertex_induced(4) + [pt.clique(3), pt.star(3), pt.EDGE_CORE_5["cricket"]]
    plans = [pg.plan_pattern(s) for s in specs]
    og = orc.Graph.from_tuple(g)
    want = [orc.count(og, s) for s in specs]
    assert pg.count(Gd, plans) == want
    T = pg.launch_tasks(Gd, plans)
    assert T == Gd.m + Gd.n  # an edge-rooted and a vertex-rooted plan
    rng = np.random.Generator(np.random.PCG64(3))
    cuts = [0] + sorted(rng.choice(np.arange(1, T), 9, replace=False).tolist()) + [T]
    total = [0] * len(specs)
    s = torch.cuda.current_stream(0)
    for a, b in zip(cuts[:-1], cuts[1:]):
        c = pg.count(Gd, plans, task_begin=a, task_end=b)
        nb = pg.job_workspace_size(Gd, plans, task_begin=a, task_end=b)
        ws = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
        off = (-ws.data_ptr()) % 256
        j, _ = pg.submit(Gd, plans, ws[off:off + nb], s, task_begin=a, task_end=b).finish()
        assert j == c
        total = [x + y for x, y in zip(total, c)]
    assert total == want
    assert pg.count(Gd, plans, task_begin=cuts[5]) == [x - y for x, y in zip(
        want, [sum(col) for col in zip(*[pg.count(Gd, plans, task_begin=a, task_end=b)
                                          for a, b in zip(cuts[:5], cuts[1:6])])])]
    for a, b in ((5, 5), (0, T + 1), (T, 0)):
        with pytest.raises(pg.PGError) as e:
            pg.count(Gd, plans, task_begin=a, task_end=b)
        assert e.value.status == pg.PG_EINVAL
