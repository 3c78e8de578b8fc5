"""Writes tests/golden/expected.json: exact counts on the seeded synthetic
workloads, computed by the CPU oracle only (never by the HIP path).

    python tests/golden/make_golden.py              # every block
    python tests/golden/make_golden.py serve_cl5k   # only the named blocks

Routes: the generic matcher (valid maps / |Aut_t|) and the existence search
for cliques, stars and anti-edge patterns; closed forms + inversion for the
six vertex-induced 4-motifs; the ESU census for the 21 vertex-induced
5-motifs of small R-MAT graphs; closed forms of 5-vertex non-induced counts
(exact linear checks on a 5-motif census) where the census is too costly.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
from paper_2004_02369_amd import graphgen as gg  # noqa: E402

CLIQUE = lambda k: {"k": k, "edges": [(a, b) for a in range(k) for b in range(a + 1, k)]}
STAR = lambda k, induced=False: {"k": k, "edges": [(0, i) for i in range(1, k)], "induced": induced}
WEDGE = {"k": 3, "edges": [(0, 1), (0, 2)]}

# R-MAT stand-ins small enough for the full 5-motif census
RMAT_SMALL = dict(scale=9, m=4 * (1 << 9), seed=20109)
RMAT_10 = dict(scale=10, m=4 * (1 << 10), seed=20110)
# the serving catalogue's graph for answers checked against the oracle
SERVE_CL5K = dict(n=5000, m=25000, gamma=2.1, w_max=200.0, seed=41)
# a hub of degree 40,000 (longer than one wavefront's 32,768-int arena)
HUB40K = dict(n_leaves=40000, m_leaves=120000, seed=43)

# The serving catalogue's patterns, written out: counts of 3-5 vertices,
# clique existence, anti-edge patterns (Sec. 3.1.1, Sec. 3.2.2).
SERVE_SPECS = (
    [("count", CLIQUE(3)), ("count", WEDGE), ("count", STAR(3, induced=True)),
     ("count", CLIQUE(4)), ("count", CLIQUE(5))]
    + [("exists", CLIQUE(k)) for k in (6, 8, 10, 12, 14)]
    + [("count", {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0), (1, 3)], "induced": True}),
       ("count", {"k": 4, "edges": [(0, 1), (1, 2), (2, 3), (3, 0)], "anti": [(1, 3)]}),
       ("count", {"k": 5, "edges": [(0, 1), (0, 2), (0, 3), (1, 4)]}),
       ("count", {"k": 5, "edges": [(0, 1), (0, 2), (1, 3), (2, 4)]}),
       ("count", {"k": 5, "edges": [(0, 1), (0, 2), (1, 2), (0, 3), (0, 4)]}),
       ("count", {"k": 5, "edges": [(0, 1), (0, 2), (1, 2), (0, 3), (1, 4)]}),
       ("count", {"k": 5, "edges": [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (0, 4), (1, 4)]})])


def census_block(og, k):
    return {str(rep): {"edges": orc.class_edges(k, rep), "count": c} for rep, c in orc.motif_census(og, k).items()}


def induced4_block(og):
    return {str(orc.canonical_of_edges(4, orc.FOUR_NAMES[n])): {"edges": orc.FOUR_NAMES[n], "count": c}
            for n, c in orc.induced4_closed_form(og).items()}


def b_er_2k_20k():
    og = orc.Graph.from_tuple(gg.workload("er_2k_20k"))
    return {"m": og.m,
            "triangle": orc.count(og, CLIQUE(3)),
            "wedge": orc.count(og, WEDGE),
            "wedge_induced": orc.count(og, dict(WEDGE, induced=True)),
            "clique4": orc.count(og, CLIQUE(4)),
            "clique5": orc.count(og, CLIQUE(5)),
            "induced4": induced4_block(og),
            "sum_c_d_2": orc.degree_choose_sum(og, 2)}


def b_rmat9_2k():
    og = orc.Graph.from_tuple(gg.rmat(**RMAT_SMALL))
    return {"params": RMAT_SMALL, "m": og.m, "induced5": census_block(og, 5),
            "induced4": census_block(og, 4), "clique5": orc.count(og, CLIQUE(5)),
            "sum_c_d_4": orc.degree_choose_sum(og, 4)}


def b_rmat10_4k():
    og = orc.Graph.from_tuple(gg.rmat(**RMAT_10))
    return {"params": RMAT_10, "m": og.m, "induced5": census_block(og, 5),
            "clique5": orc.count(og, CLIQUE(5)), "sum_c_d_4": orc.degree_choose_sum(og, 4),
            "noninduced5": orc.noninduced5_closed_forms(og)}


def b_rmat12_64k():
    """The scaled-down 5-motif workload: its census is beyond the oracle
    (about 10^12 connected 5-sets), so only closed-form rows are stored."""
    og = orc.Graph.from_tuple(gg.workload("rmat12_64k"))
    return {"m": og.m, "sum_c_d_4": orc.degree_choose_sum(og, 4), "noninduced5": orc.noninduced5_closed_forms(og)}


def b_chunglu_100k_1m():
    og = orc.Graph.from_tuple(gg.workload("chunglu_100k_1m"))
    nc = orc.noninduced4(og)
    return {"m": og.m, "d_max": int(og.degrees().max()), "induced4": induced4_block(og),
            "triangle": nc["triangle"], "sum_c_d_2": orc.degree_choose_sum(og, 2),
            "sum_c_d_3": orc.degree_choose_sum(og, 3)}


def b_serve_cl5k():
    g = gg.chung_lu(SERVE_CL5K["n"], SERVE_CL5K["m"], SERVE_CL5K["gamma"], SERVE_CL5K["w_max"],
                    seed=SERVE_CL5K["seed"])
    og = orc.Graph.from_tuple(g)
    ans = []
    for kind, spec in SERVE_SPECS:
        ans.append({"kind": kind, "spec": spec,
                    "answer": orc.exists(og, spec) if kind == "exists" else orc.count(og, spec)})
    # the six vertex-induced 4-motifs (closed forms) and the 4-star (sum C(d, 4))
    for name, c in orc.induced4_closed_form(og).items():
        ans.append({"kind": "count", "spec": {"k": 4, "edges": orc.FOUR_NAMES[name], "induced": True}, "answer": c})
    ans.append({"kind": "count", "spec": STAR(5), "answer": orc.degree_choose_sum(og, 4)})
    return {"params": SERVE_CL5K, "m": og.m, "answers": ans}


def b_hub40k():
    og = orc.Graph.from_tuple(gg.hub_plus_er(**HUB40K))
    nc = orc.noninduced4(og)
    return {"params": HUB40K, "m": og.m, "d_max": int(og.degrees().max()), "triangle": nc["triangle"],
            "induced4": induced4_block(og), "sum_c_d_2": orc.degree_choose_sum(og, 2),
            "sum_c_d_3": orc.degree_choose_sum(og, 3)}


BLOCKS = {"er_2k_20k": b_er_2k_20k, "rmat9_2k": b_rmat9_2k, "chunglu_100k_1m": b_chunglu_100k_1m,
          "serve_cl5k": b_serve_cl5k, "hub40k": b_hub40k, "rmat10_4k": b_rmat10_4k, "rmat12_64k": b_rmat12_64k}


def main():
    path = os.path.join(HERE, "expected.json")
    names = sys.argv[1:] or list(BLOCKS)
    out = {"_note": "exact counts from the CPU oracle; regenerate with make_golden.py", "workloads": {}}
    if sys.argv[1:] and os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    t0 = time.time()
    for name in names:
        out["workloads"][name] = BLOCKS[name]()
        print(name, round(time.time() - t0, 1), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
