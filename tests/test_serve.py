"""Host logic of the serving loop (no GPU): the workspace pool and the
admission / continuous-batching policy."""
import random

import pytest

from paper_2004_02369_amd import serve
from paper_2004_02369_amd.serve import ALIGN, MAX_PLANS, Pool, Query, Request, next_batch


def test_pool_first_fit_alignment_and_coalescing():
    p = Pool(10 * ALIGN + 17)
    assert p.size == 10 * ALIGN
    a = p.alloc(1)
    b = p.alloc(ALIGN + 1)
    c = p.alloc(3 * ALIGN)
    assert (a, b, c) == (0, ALIGN, 3 * ALIGN)
    assert all(o % ALIGN == 0 for o in (a, b, c))
    assert p.used == 6 * ALIGN
    assert p.alloc(5 * ALIGN) is None
    p.free(b)
    assert p.alloc(2 * ALIGN) == ALIGN  # the hole is reused first
    p.free(a)
    p.free(ALIGN)
    p.free(c)
    assert p.free_list == [(0, 10 * ALIGN)] and p.used == 0


def test_pool_random_never_overlaps():
    rng = random.Random(3)
    p = Pool(1 << 20)
    live = {}
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            p.free(off)
            del live[off]
        else:
            n = rng.randint(1, 40000)
            off = p.alloc(n)
            if off is None:
                assert p.largest_free() < -(-n // ALIGN) * ALIGN
                continue
            assert off % ALIGN == 0 and off + n <= p.size
            for o, m in live.items():
                assert off + n <= o or o + m <= off
            live[off] = n
    assert p.used == sum(-(-n // ALIGN) * ALIGN for n in live.values())
    for off in list(live):
        p.free(off)
    assert p.free_list == [(0, p.size)]


class FakePlan:
    def __init__(self, name, depth=4):
        self.name, self.depth = name, depth


def _size(per_plan=1000, base=ALIGN):
    # workspace grows with the deepest plan and the trie size
    return lambda plans, kind, heavy=False: base + per_plan * len(plans) + 100000 * max(p.depth for p in plans)


def _q(name, kind="count", plans=None):
    return Query(name, kind, plans or [FakePlan(name)])


def _reqs(queries):
    return [Request(i, q, 0.0) for i, q in enumerate(queries)]


def test_count_requests_merge_and_deduplicate():
    tri, wedge = _q("tri"), _q("wedge")
    ex = _q("k6", "exists")
    queue = _reqs([tri, ex, wedge, tri, wedge])
    pool = Pool(1 << 24)
    b, rej = next_batch(queue, _size(), pool)
    assert rej is None
    assert [r.rid for r in b.requests] == [0, 2, 3, 4]   # the existence query keeps its place
    assert [p.name for p in b.plans] == ["tri", "wedge"]  # identical plans counted once
    assert b.index == [[0], [1], [0], [1]]
    assert b.kind == "count" and b.offset == 0


def test_existence_runs_alone_with_its_repeats():
    ex = _q("k6", "exists")
    queue = _reqs([ex, _q("tri"), _q("k8", "exists"), ex, _q("k6b", "exists", plans=list(ex.plans))])
    b, _ = next_batch(queue, _size(), Pool(1 << 24))
    assert [r.rid for r in b.requests] == [0, 3, 4] and b.kind == "exists"
    assert len(b.plans) == 1 and b.index == [[0], [0], [0]]


def test_batch_capped_at_64_unique_plans():
    qs = [_q(f"p{i}", plans=[FakePlan(f"a{i}"), FakePlan(f"b{i}")]) for i in range(40)]
    b, _ = next_batch(_reqs(qs), _size(), Pool(1 << 30))
    assert len(b.plans) == MAX_PLANS and len(b.requests) == 32
    # a request whose plans are already in the batch still joins it
    shared = [FakePlan(f"s{i}") for i in range(64)]
    qs = [_q("big", plans=shared), _q("sub", plans=shared[:3]), _q("new")]
    b, _ = next_batch(_reqs(qs), _size(), Pool(1 << 30))
    assert [r.query.name for r in b.requests] == ["big", "sub"]


def test_admission_waits_for_memory_and_cuts_from_the_back():
    size = _size(per_plan=100000)
    pool = Pool(1 << 20)
    queue = _reqs([_q(f"q{i}") for i in range(8)])
    need1 = size([FakePlan("x")], "count")
    # 1 request fits, 8 do not: the batch is cut to what fits
    b, _ = next_batch(queue, size, pool)
    assert 1 <= len(b.requests) < 8
    assert size(b.plans, "count") <= pool.size
    # the pool is now nearly full: nothing more fits, nothing is rejected
    queue2 = _reqs([_q("late")])
    hold = pool.alloc(pool.largest_free())
    b2, rej = next_batch(queue2, size, pool)
    assert b2 is None and rej is None
    pool.free(hold)
    assert next_batch(queue2, size, pool) == (None, None)  # the first launch still holds its workspace
    pool.free(b.offset)
    b3, _ = next_batch(queue2, size, pool)
    assert b3 is not None and need1 <= pool.used


def test_request_larger_than_pool_is_rejected():
    deep = _q("deep", plans=[FakePlan("deep", depth=50)])
    b, rej = next_batch(_reqs([deep]), _size(), Pool(1 << 20))
    assert b is None and rej.query.name == "deep"


def test_query_validation():
    with pytest.raises(ValueError):
        Query("x", "exists", [FakePlan("a"), FakePlan("b")])
    with pytest.raises(ValueError):
        Query("x", "maybe", [FakePlan("a")])
    with pytest.raises(ValueError):
        Query("x", "count", [])


def test_summary_percentiles():
    q = _q("tri")
    reqs = []
    for i in range(100):
        r = Request(i, q, 10.0)
        r.done = 10.0 + (i + 1) / 1000.0
        r.result = [2]
        reqs.append(r)
    s = serve.summarize(reqs, 10.0)
    assert s["p50_ms"] == pytest.approx(50.0) and s["p99_ms"] == pytest.approx(99.0)
    assert s["completed"] == 100 and s["errors"] == 0
    assert s["completed_qps"] == pytest.approx(1000.0)
    assert s["matches_per_s"] == pytest.approx(2000.0)


def test_poisson_arrivals_seeded():
    t1, p1 = serve.poisson_arrivals(200.0, 5000, 21, seed=9)
    t2, p2 = serve.poisson_arrivals(200.0, 5000, 21, seed=9)
    assert (t1 == t2).all() and (p1 == p2).all()
    assert (t1[1:] > t1[:-1]).all()
    assert t1[-1] / 5000 == pytest.approx(1 / 200.0, rel=0.05)
    assert set(p1.tolist()) == set(range(21))


def _pol(costs, **kw):
    pol = serve.Policy(**kw)
    for p, ms in costs.items():
        pol.est[id(p)] = ms
    return pol


def test_policy_classes_do_not_mix():
    light_p, heavy_p, heavy_q = FakePlan("l"), FakePlan("h"), FakePlan("h2")
    pol = _pol({light_p: 5.0, heavy_p: 900.0, heavy_q: 800.0}, light_ms=50.0, merge_cap_ms=200.0)
    L, H, H2 = _q("l", plans=[light_p]), _q("h", plans=[heavy_p]), _q("h2", plans=[heavy_q])
    queue = _reqs([H, L, H, H2, L])
    b, _ = next_batch(queue, _size(), Pool(1 << 30), pol)
    # heavy head: the repeat of its plan joins for free, the other heavy plan
    # would exceed max(900, cap) and the light ones belong to the other class
    assert b.heavy and [r.rid for r in b.requests] == [0, 2]
    # heavy launches not allowed now: the oldest light request leads
    b2, _ = next_batch(queue, _size(), Pool(1 << 30), pol, allow_heavy=False)
    assert not b2.heavy and [r.rid for r in b2.requests] == [1, 4]
    # nothing light waiting and heavy not allowed: nothing starts
    assert next_batch(_reqs([H, H2]), _size(), Pool(1 << 30), pol, allow_heavy=False) == (None, None)


def test_policy_merge_cap():
    ps = [FakePlan(f"p{i}") for i in range(10)]
    pol = _pol({p: 30.0 for p in ps}, light_ms=50.0, merge_cap_ms=100.0)
    b, _ = next_batch(_reqs([_q(f"q{i}", plans=[p]) for i, p in enumerate(ps)]), _size(), Pool(1 << 30), pol)
    assert len(b.plans) == 3                        # 3 x 30 ms <= 100 ms < 4 x 30 ms
    # unknown plans cost nothing: everything light merges up to 64 plans
    b, _ = next_batch(_reqs([_q(f"u{i}") for i in range(70)]), _size(), Pool(1 << 30), serve.Policy())
    assert len(b.plans) == MAX_PLANS


def test_policy_observe():
    a, b = FakePlan("a"), FakePlan("b")
    pol = serve.Policy(light_ms=50.0)
    pol.observe([a], 10.0)
    pol.observe([a], 30.0)
    assert pol.est[id(a)] == pytest.approx(20.0)
    pol.observe([a, b], 50.0)
    assert pol.est[id(a)] == pytest.approx(20.0) and pol.est[id(b)] == pytest.approx(25.0)
    assert pol.heavy(Request(0, _q("x", plans=[a, b]), 0.0)) is False
    assert pol.heavy(Request(0, _q("x", plans=[a, b, FakePlan("c")]), 0.0)) is False
    pol.est[id(b)] = 45.0
    assert pol.heavy(Request(0, _q("x", plans=[a, b]), 0.0)) is True


def test_pattern_key_identifies_same_patterns():
    from paper_2004_02369_amd import patterns as pt
    k4 = pt.clique(4)
    assert serve.pattern_key(k4) == serve.pattern_key(dict(k4, induced=True))
    assert serve.pattern_key(pt.star(4)) != serve.pattern_key(pt.star(4, induced=True))
    assert serve.pattern_key(pt.chain(3)) != serve.pattern_key(dict(pt.chain(3), labels=[0, 1, 0]))


def test_task_windows_partition_and_grow():
    for total, n in [(1, 5), (10, 1), (10, 3), (1000, 16), (67108864, 16), (5, 16), (2, 2)]:
        w = serve.task_windows(total, n)
        assert w[0][0] == 0 and w[-1][1] == total
        assert all(a < b for a, b in w) and all(w[i][1] == w[i + 1][0] for i in range(len(w) - 1))
        assert len(w) <= max(1, min(n, total))
    w = serve.task_windows(1 << 20, 8)
    sizes = [b - a for a, b in w]
    assert len(w) == 8 and all(abs(sizes[i + 1] / sizes[i] - 2) < 0.01 for i in range(7))
