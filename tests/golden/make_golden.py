"""Writes tests/golden/expected.json: exact counts on the seeded synthetic
workloads, computed by the CPU oracle only (never by the HIP path).

    python tests/golden/make_golden.py            # all workloads (~10 min, 8 cores)

Routes: the generic matcher (valid maps / |Aut_t|) for cliques and stars,
closed forms + inversion for the six vertex-induced 4-motifs, and the ESU
census for the 21 vertex-induced 5-motifs of a small R-MAT graph.
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
WEDGE = {"k": 3, "edges": [(0, 1), (0, 2)]}

# R-MAT stand-in small enough for the full 5-motif census
RMAT_SMALL = dict(scale=9, m=4 * (1 << 9), seed=20109)


def census_block(og, k):
    return {str(rep): {"edges": orc.class_edges(k, rep), "count": c} for rep, c in orc.motif_census(og, k).items()}


def main():
    out = {"_note": "exact counts from the CPU oracle; regenerate with make_golden.py", "workloads": {}}
    t0 = time.time()

    # ER 2,000 / 20,000
    g = gg.workload("er_2k_20k")
    og = orc.Graph.from_tuple(g)
    w = {"m": og.m,
         "triangle": orc.count(og, CLIQUE(3)),
         "wedge": orc.count(og, WEDGE),
         "wedge_induced": orc.count(og, dict(WEDGE, induced=True)),
         "clique4": orc.count(og, CLIQUE(4)),
         "clique5": orc.count(og, CLIQUE(5)),
         "induced4": {str(orc.canonical_of_edges(4, e)): {"edges": e, "count": c}
                      for e, c in ((orc.FOUR_NAMES[n], v) for n, v in orc.induced4_closed_form(og).items())},
         "sum_c_d_2": orc.degree_choose_sum(og, 2)}
    out["workloads"]["er_2k_20k"] = w
    print("er_2k_20k", round(time.time() - t0, 1), flush=True)

    # R-MAT small: 21 induced 5-motifs (ESU) + K5 (generic matcher)
    g = gg.rmat(**RMAT_SMALL)
    og = orc.Graph.from_tuple(g)
    out["workloads"]["rmat9_2k"] = {"params": RMAT_SMALL, "m": og.m, "induced5": census_block(og, 5),
                                    "induced4": census_block(og, 4), "clique5": orc.count(og, CLIQUE(5)),
                                    "sum_c_d_4": orc.degree_choose_sum(og, 4)}
    print("rmat9_2k", round(time.time() - t0, 1), flush=True)

    # Chung-Lu 100,000 / 1,000,000: six induced 4-motifs
    g = gg.workload("chunglu_100k_1m")
    og = orc.Graph.from_tuple(g)
    ind = orc.induced4_closed_form(og)
    nc = orc.noninduced4(og)
    out["workloads"]["chunglu_100k_1m"] = {
        "m": og.m, "d_max": int(og.degrees().max()),
        "induced4": {str(orc.canonical_of_edges(4, orc.FOUR_NAMES[n])): {"edges": orc.FOUR_NAMES[n], "count": c}
                     for n, c in ind.items()},
        "triangle": nc["triangle"], "sum_c_d_2": orc.degree_choose_sum(og, 2),
        "sum_c_d_3": orc.degree_choose_sum(og, 3)}
    print("chunglu_100k_1m", round(time.time() - t0, 1), flush=True)

    with open(os.path.join(HERE, "expected.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
