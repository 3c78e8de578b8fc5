"""GPU test of pg_count_noalloc, the counting entry point that allocates no
device memory (its launch memory is a fixed device array of the library):
it returns what pg_count_ex returns, on two calls in a row (the second on a
smaller input), with a grid it has to shrink, and refuses a launch whose
single wavefront's scratch exceeds the array."""
import sys

import numpy as np
import pytest

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


def test_noalloc_equals_count_ex_twice(pg):
    import torch
    s = torch.cuda.current_stream(0)
    say("noalloc: chung_lu 3000/24000, six induced 4-motifs + triangle + K4 + K5")
    g1 = pg.load_graph(*gg.chung_lu(3000, 24000, 2.1, 300.0, seed=21), device=0)
    plans1 = [pg.plan_pattern(x) for x in pt.all_vertex_induced(4) + [pt.clique(3), pt.clique(4), pt.clique(5)]]
    want1, _ = pg.count_ex(g1, plans1, stream=s)
    assert pg.count_noalloc(g1, plans1, stream=s) == want1
    say("noalloc: second call, ER 500/3000, triangle + wedge")
    g2 = pg.load_graph(*gg.erdos_renyi_m(500, 3000, seed=3), device=0)
    plans2 = [pg.plan_pattern(pt.clique(3)), pg.plan_pattern(pt.star(3))]
    want2, _ = pg.count_ex(g2, plans2, stream=s)
    assert pg.count_noalloc(g2, plans2, stream=s) == want2
    say("noalloc: the first input again, with a grid larger than the array holds")
    assert pg.count_noalloc(g1, plans1, stream=s, grid_waves=100000) == want1


def test_noalloc_refuses_oversize(pg):
    say("noalloc: 16-clique on a 6,000,000-leaf star (13 levels x 6M ints per wavefront)")
    n, u, v = gg.star(6_000_000)
    G = pg.load_graph(n, u, v, device=0)
    with pytest.raises(pg.PGError) as e:
        pg.count_noalloc(G, [pg.plan_pattern(pt.clique(16))])
    assert e.value.status == pg.PG_ENOMEM and "exceeds the fixed" in str(e.value)
    # the array is still usable afterwards
    assert pg.count_noalloc(G, [pg.plan_pattern(pt.star(3))]) == [6_000_000 * 5_999_999 // 2]
