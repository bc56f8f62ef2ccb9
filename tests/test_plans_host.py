"""Host-only checks of the matching plans and coalescing groups that
registration builds (gamma_describe_query; no GPU).

Structure: one plan per directed query edge, each a connected matching
order starting with its edge; the whole-query permutations are
label-, edge- and edge-label-preserving automorphisms of the query
(Sec. V-B, k = 0); the core permutations are automorphisms of the query
without its degree-1 vertices and fix the removed vertices (k > 0); a
representative's core comes first in its order and its position masks hold
the positions its permutations move each vertex to.

Semantics, by brute force on tiny graphs: for every data edge (a, b) in
both orientations, the matches found from the seeded plans, continued under
their permutations the way the search does it, are exactly the matches of
every plan, each once (a match g derived from f is g(v) = f(pi(v))), both
with whole-query coalescing and with core coalescing."""
import itertools
import random
from collections import Counter

import numpy as np
import pytest

from oracle import closed_forms as CF
from paper_2401_17018_amd import describe_query

SHAPES = [
    (4, [(0, 1), (1, 2), (2, 0), (1, 3)], (0, 1, 1, 2)),                                        # triangle + leaf
    (6, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 5)], (0, 0, 0, 0, 1, 2)),                  # 4-cycle + 2 leaves
    (6, [(0, 1), (1, 2), (2, 0), (1, 3), (3, 0), (0, 4), (2, 5)], (0, 0, 0, 0, 1, 2)),          # diamond + 2 leaves
    (3, [(0, 1), (1, 2), (2, 0)], (0, 0, 0)),                                                   # triangle
    (4, [(0, 1), (1, 2), (2, 3), (3, 0)], (0, 0, 0, 0)),                                        # 4-cycle
    (4, [(0, 1), (0, 2), (0, 3)], (1, 0, 0, 0)),                                                # star
    (5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (0, 4)], (0, 0, 0, 0, 1)),             # K4 + leaf (k = 0)
]


def _random_query(rng):
    k = rng.randint(3, 6)
    kc = rng.randint(3, k)
    edges = set()
    for v in range(1, kc):
        u = rng.randrange(v)
        edges.add((u, v))
    for _ in range(rng.randint(0, kc)):
        a, b = rng.sample(range(kc), 2)
        edges.add((min(a, b), max(a, b)))
    for v in range(kc, k):
        edges.add((rng.randrange(kc), v))
    labels = tuple(rng.choice((0, 0, 1)) if v < kc else rng.randint(0, 2) for v in range(k))
    return k, sorted(edges), labels


def _is_aut(perm, verts, labels, E):
    """perm restricted to verts is a bijection of verts preserving labels and the labelled edge set E."""
    img = [perm[v] for v in verts]
    if sorted(img) != sorted(verts) or any(labels[perm[v]] != labels[v] for v in verts):
        return False
    return all(((min(perm[a], perm[b]), max(perm[a], perm[b])) in E and E[(min(perm[a], perm[b]), max(perm[a], perm[b]))] == el)
               for (a, b), el in E.items())


def _check_structure(k, edges, labels, elabels):
    plans, perms = describe_query(k, labels, edges, elabels)
    m = len(edges)
    assert len(plans) == 2 * m
    adj = [set() for _ in range(k)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    assert sorted((p["x"], p["y"]) for p in plans) == sorted([(a, b) for a, b in edges] + [(b, a) for a, b in edges])
    for p in plans:
        o = p["order"]
        assert sorted(o) == list(range(k)) and o[:2] == [p["x"], p["y"]]
        assert all(adj[o[l]] & set(o[:l]) for l in range(2, k))
    E = {(min(a, b), max(a, b)): (elabels[i] if elabels else 0) for i, (a, b) in enumerate(edges)}
    deg = [len(adj[v]) for v in range(k)]
    core = [v for v in range(k) if deg[v] >= 2]
    Ec = {e: el for e, el in E.items() if e[0] in core and e[1] in core}
    for p in plans:
        if p["n_perm"] >= 1:
            for j in range(p["perm_first"], p["perm_first"] + p["n_perm"]):
                assert _is_aut(perms[j], list(range(k)), labels, E)
        if p["n_cperm"] >= 2:
            assert p["n_core"] == len(core) and sorted(p["order"][:p["n_core"]]) == core
            want = [0] * k
            for j in range(p["cperm_first"], p["cperm_first"] + p["n_cperm"]):
                pi = perms[j]
                assert _is_aut(pi, core, labels, Ec)
                assert all(pi[v] == v for v in range(k) if v not in core)
                inv = [0] * k
                for v in range(k):
                    inv[pi[v]] = v
                for u in range(k):
                    want[u] |= 1 << inv[u]
            assert p["omask"] == want
        else:
            assert p["omask"] == [1 << u for u in range(k)]
    return plans, perms


def _graph(rng, n, qlabels, nel, p):
    # the query's labels, each at least as often as in the query, so that
    # matches can occur
    glab = list(qlabels) + [rng.choice(qlabels) for _ in range(n - len(qlabels))]
    rng.shuffle(glab)
    gel = {}
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < p:
                gel[(a, b)] = gel[(b, a)] = rng.randrange(nel)
    return glab, gel


def _extend(n, glab, gel, k, labels, qe, fixed, verts):
    free = [v for v in verts if v not in fixed]
    used = set(fixed.values())
    for img in itertools.permutations([c for c in range(n) if c not in used], len(free)):
        f = dict(fixed)
        f.update(zip(free, img))
        if all(glab[f[v]] == labels[v] for v in f) and all(
                gel.get((f[a], f[b])) == el for (a, b), el in qe.items() if a in f and b in f):
            yield f


def _check_semantics(k, edges, labels, elabels, plans, perms, rng, cases=3):
    qe = {(a, b): (elabels[i] if elabels else 0) for i, (a, b) in enumerate(edges)}
    allv = list(range(k))
    total = 0
    for _ in range(cases):
        n = rng.randint(max(5, k + 1), k + 2)
        glab, gel = _graph(rng, n, labels, (max(elabels) + 1) if elabels else 1, rng.uniform(0.7, 0.95))
        ref, k0, core = Counter(), Counter(), Counter()
        for (a, b) in gel:
            for p in plans:
                fixed = {p["x"]: a, p["y"]: b}
                found = [tuple(f[v] for v in allv) for f in _extend(n, glab, gel, k, labels, qe, fixed, allv)]
                for t in found:
                    ref[(a, b, t)] += 1
                # whole-query coalescing: representatives only, each match stands for its permutations
                if p["n_perm"] >= 1:
                    for t in found:
                        for j in range(p["perm_first"], p["perm_first"] + p["n_perm"]):
                            k0[(a, b, tuple(t[perms[j][v]] for v in allv))] += 1
                # core coalescing (applies where no plan has whole-query permutations)
                if p["n_perm"] == 0 or p["n_cperm"] == 0:
                    continue
                if p["n_cperm"] == 1:
                    for t in found:
                        for j in range(p["perm_first"], p["perm_first"] + p["n_perm"]):
                            core[(a, b, tuple(t[perms[j][v]] for v in allv))] += 1
                    continue
                cv = p["order"][:p["n_core"]]
                for fc in _extend(n, glab, gel, k, labels, qe, fixed, cv):
                    for j in range(p["cperm_first"], p["cperm_first"] + p["n_cperm"]):
                        g = {v: fc[perms[j][v]] for v in cv}
                        for f in _extend(n, glab, gel, k, labels, qe, g, allv):
                            core[(a, b, tuple(f[v] for v in allv))] += 1
        assert k0 == ref and core == ref
        total += sum(ref.values())
    return total


@pytest.mark.parametrize("i", range(len(SHAPES)))
def test_named_shapes(i):
    k, edges, labels = SHAPES[i]
    plans, perms = _check_structure(k, edges, labels, None)
    n_aut = len(CF.automorphisms(k, labels, edges))
    if n_aut > 1:
        # k = 0 groups: every representative stands for a whole number of orbit members
        assert sum(p["n_perm"] for p in plans) == 2 * len(edges)
        assert all(p["n_cperm"] == 1 for p in plans)
    if i < 3:
        assert n_aut == 1 and any(p["n_cperm"] >= 2 for p in plans)
    assert _check_semantics(k, edges, labels, None, plans, perms, random.Random(100 + i)) > 0


def test_random_queries():
    rng = random.Random(7)
    n_core_groups = n_k0_groups = total = 0
    for _ in range(60):
        k, edges, labels = _random_query(rng)
        elabels = [rng.randrange(2) for _ in edges] if rng.random() < 0.3 else None
        plans, perms = _check_structure(k, edges, labels, elabels)
        n_core_groups += sum(p["n_cperm"] >= 2 for p in plans)
        n_k0_groups += sum(p["n_perm"] >= 2 for p in plans)
        total += _check_semantics(k, edges, labels, elabels, plans, perms, rng, cases=1)
    assert n_core_groups > 0 and n_k0_groups > 0 and total > 0


def test_core_orbit_larger_than_a_group():
    """K5 with differently labelled leaves on four of its vertices: no
    automorphism of the query, the core's 20 directed edges form one orbit,
    split into groups of at most 16 permutations."""
    k = 9
    edges = [(a, b) for a in range(5) for b in range(a + 1, 5)] + [(0, 5), (1, 6), (2, 7), (3, 8)]
    labels = (0, 0, 0, 0, 0, 1, 2, 3, 4)
    plans, perms = _check_structure(k, edges, labels, None)
    reps = [p for p in plans if p["n_cperm"] >= 2]
    assert sorted(p["n_cperm"] for p in reps) == [4, 16]
    assert sum(p["n_cperm"] == 0 for p in plans) == 20 - len(reps)
    assert all(p["n_cperm"] == 1 for p in plans if p["x"] >= 5 or p["y"] >= 5)


def test_edge_labels_break_core_symmetry():
    k, edges, labels = 4, [(0, 1), (1, 2), (2, 0), (1, 3)], (0, 1, 1, 2)
    sym, _ = _check_structure(k, edges, labels, [1, 0, 1, 1])
    asym, _ = _check_structure(k, edges, labels, [1, 0, 0, 1])
    assert any(p["n_cperm"] >= 2 for p in sym)
    assert all(p["n_cperm"] == 1 for p in asym)


def test_invalid_query_raises():
    from paper_2401_17018_amd import GammaError
    with pytest.raises(GammaError):
        describe_query(4, [0] * 4, [[0, 1], [0, 2], [1, 2]])  # disconnected
    with pytest.raises(GammaError):
        describe_query(3, [0] * 3, [[0, 1], [1, 2]], elabels=[0, 300])
