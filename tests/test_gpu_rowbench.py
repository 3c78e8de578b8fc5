"""GPU test of the measurement kernels: every intersection variant gives
|N(u) & N(v)| = the oracle's triangle count of the edge (u, v), on a
skewed graph whose rows span every length bucket, and the streaming read
sums the buffer it reads."""
import sys

import numpy as np
import pytest

from paper_2004_02369_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_row_intersections_equal_edge_triangles(orc):
    import torch
    from paper_2004_02369_amd import rowbench as rb
    g = gg.disjoint_union(gg.chung_lu(6000, 60000, 2.1, 1500.0, seed=3), gg.hub_plus_er(9000, 20000, seed=4))
    og = orc.Graph.from_tuple(g)
    off, adj, t = orc.edge_triangles(og)
    say(f"row intersections on {og.n} vertices, {og.m} edges, d_max {int(np.diff(off).max())}")
    dev = torch.device("cuda:0")
    rp, col = torch.from_numpy(off).to(dev), torch.from_numpy(adj).to(dev)
    src = np.repeat(np.arange(og.n, dtype=np.int32), np.diff(off))
    pu, pv = torch.from_numpy(src).to(dev), torch.from_numpy(adj.astype(np.int32)).to(dev)
    for name, var in rb.VARIANTS.items():
        for grid in (0, 7):
            say(f"variant {name} grid {grid}")
            out = torch.full((len(adj),), -1, dtype=torch.int32, device=dev)
            rb.intersect(var, rp, col, pu, pv, out, grid=grid)
            assert np.array_equal(out.cpu().numpy().astype(np.int64), t), name


def test_stream_read_checksum():
    import torch
    from paper_2004_02369_amd import rowbench as rb
    say("stream read checksum")
    buf = torch.arange(1 << 22, dtype=torch.int32, device="cuda:0")
    ms, ck = rb.stream_read(buf, reps=2)
    n = 1 << 22
    assert ck == 3 * (n * (n - 1) // 2) % (1 << 64) and ms > 0
