"""Slow reference interpreter of the level programs exported by
pg_plan_programs (test helper).  It evaluates each level's stated
constraints literally over all vertices of a tiny graph, so it checks the
plan compiler's output (symmetry breaking, core, matching orders, groups,
anti-vertex triggers, base sets) against the oracle on the CPU, with no
GPU involved.  It also asserts the invariants the GPU relies on: every
candidate differs from every earlier image, a level's base set contains
its candidates, t_isect / t_diff are what the base leaves untested, and a
program's factor sets never share a vertex with each other or with the
last level's candidates (which makes their product exact)."""
from __future__ import annotations

import math


def _bits(x):
    y = 0
    while x:
        if x & 1:
            yield y
        x >>= 1
        y += 1


def _adj(n, src, dst):
    adj = [set() for _ in range(n)]
    for a, b in zip(map(int, src), map(int, dst)):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def _ok(v, L, m, adj, labels):
    for y in _bits(L["isect"]):
        if v not in adj[m[y]]:
            return False
    for y in _bits(L["diff"]):
        if v in adj[m[y]]:
            return False
    for y in _bits(L["lo"]):
        if not v > m[y]:
            return False
    for y in _bits(L["hi"]):
        if not v < m[y]:
            return False
    for y in _bits(L["excl"]):
        if v == m[y]:
            return False
    if L["label"] >= 0 and (labels is None or labels[v] != L["label"]):
        return False
    mm = m + [v]
    for c in L["avs"]:
        common = None
        for a in _bits(c["nbr"]):
            part = set(adj[mm[a]]) - {mm[y] for y in _bits(c["xmask"][a])}
            common = part if common is None else common & part
        if c["label"] >= 0:
            common = {w for w in common if labels is not None and labels[w] == c["label"]}
        if common:
            return False
    return True


def _walk(n, adj, labels, levels, emit_fn=None, factors=()):
    F = len(levels) - 1
    assert emit_fn is None or not factors
    for x, L in list(enumerate(levels)) + [(F, Fl) for Fl in factors]:
        if L["base"] >= 0:
            B = levels[L["base"]]
            assert L["isect"] == L["t_isect"] | B["isect"] and L["diff"] == L["t_diff"] | B["diff"]
        elif x >= 2:
            assert L["isect"] == L["t_isect"] and L["diff"] == L["t_diff"]
        if x >= 1:
            assert L["isect"], "every level after the root is adjacent to an earlier one"

    def rec(x, m, sets):
        L = levels[x]
        cands = [v for v in range(n) if _ok(v, L, m, adj, labels)]
        for v in cands:
            assert v not in m, "candidate equals an earlier image"
        if L["base"] >= 0:
            assert set(cands) <= set(sets[L["base"]]), "base set does not contain the candidates"
        if x == F:
            if emit_fn is not None:
                assert L["group"] == 1
                for v in cands:
                    emit_fn(m + [v])
                return len(cands)
            ways = math.comb(len(cands), L["group"])
            # factors: independent groups at this depth; the product is
            # exact only if no two of these sets can share a vertex
            seen = set(cands)
            for Fl in factors:
                fc = [v for v in range(n) if _ok(v, Fl, m, adj, labels)]
                for v in fc:
                    assert v not in m, "factor candidate equals an earlier image"
                if Fl["base"] >= 0:
                    assert set(fc) <= set(sets[Fl["base"]]), "base set does not contain the candidates"
                assert not (seen & set(fc)), "factor sets overlap"
                seen |= set(fc)
                ways *= math.comb(len(fc), Fl["group"])
            return ways
        return sum(rec(x + 1, m + [v], sets + [cands]) for v in cands)

    return rec(0, [], [])


def interp_count(graph, programs, labels=None) -> int:
    n, src, dst = graph
    adj = _adj(n, src, dst)
    return sum(p["mult"] * _walk(n, adj, labels, p["levels"], factors=p.get("factors", ())) for p in programs)


def interp_enumerate(graph, programs, k, labels=None) -> list[tuple]:
    n, src, dst = graph
    adj = _adj(n, src, dst)
    out = []
    for p in programs:
        assert p["mult"] == 1 and not p.get("factors")
        pv = [L["pv"] for L in p["levels"]]

        def emit(m, pv=pv):
            row = [None] * k
            for lev, v in enumerate(m):
                row[pv[lev]] = v
            out.append(tuple(row))
        _walk(n, adj, labels, p["levels"], emit)
    return out
