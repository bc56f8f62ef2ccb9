"""Pins for the oracle's vertex updates (Sec. II-A: a vertex deletion is the
deletion of its incident edges, a vertex insertion adds the vertex before
its edges are inserted).

The reduction is checked against the definitions directly: the matches a
vertex deletion removes are exactly the matches of G whose image contains a
deleted vertex, computed by brute-force enumeration without going through
any edge batch; isolated vertices change no match of a query with an edge."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import workloads as W
from oracle import brute as O1
from oracle import plain as O2
from oracle import vertices as OV


def _graph(seed, n, extra, n_labels):
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = set()
    for _ in range(n + extra):
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u != v:
            edges.add((min(u, v), max(u, v)))
    return W.graph_from_edges(n, sorted(edges), rng.integers(0, n_labels, n).tolist()), rng


def _query(rng, k, n_labels):
    edges = {(i - 1, i) for i in range(1, k)}
    if k >= 3 and rng.random() < 0.5:
        edges.add((0, k - 1))
    return W.query_from_edges(k, sorted(edges), rng.integers(0, n_labels, k).tolist())


def _matches(g, q, E):
    return O1.all_matches(g.n, g.labels, O1.adjacency(g.n, E), q.k, q.labels, [tuple(e) for e in q.edges.tolist()])


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(4, 9), k=st.integers(2, 4), extra=st.integers(0, 12),
       n_labels=st.integers(1, 2), n_vdel=st.integers(1, 3))
def test_vertex_deletion_removes_the_matches_through_it(seed, n, k, extra, n_labels, n_vdel):
    g, rng = _graph(seed, n, extra, n_labels)
    q = _query(rng, k, n_labels)
    vdel = rng.integers(0, n, n_vdel).tolist()  # may repeat
    empty = W.Batch(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint8))
    status, merged = OV.deletion_batch(g, empty, vdel)
    assert status == "ok"
    E = O1.edge_set(g)
    M = _matches(g, q, E)
    through = {f for f in M if set(f) & set(vdel)}
    r = O1.bdsm(g, q, merged)
    assert r["status"] == "ok"
    assert r["plus"] == set() and r["minus"] == through
    assert r["E2"] == {e for e in E if not set(e) & set(vdel)}
    # O2 agrees on the merged batch
    o = O2.run(g, q, merged, want_tuples=True)
    assert o.status == 0 and o.tuple_set(0) == through and o.tuple_set(1) == set()


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(5, 9), k=st.integers(2, 4), extra=st.integers(2, 12))
def test_vertex_deletion_with_edge_updates(seed, n, k, extra):
    """Explicit insertions away from the deleted vertex, explicit deletions
    anywhere (those at the deleted vertex collapse as duplicates): the
    result is the set difference for G' = (E + I - D) minus the edges at the
    deleted vertex."""
    g, rng = _graph(seed, n, extra, 2)
    q = _query(rng, k, 2)
    v = int(rng.integers(0, n))
    E = O1.edge_set(g)
    present = sorted(E)
    D = {present[i] for i in rng.permutation(len(present))[:2]}
    I = set()
    for _ in range(20):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        e = (min(a, b), max(a, b))
        if a != b and v not in e and e not in E:
            I.add(e)
        if len(I) == 3:
            break
    ups = [("+",) + e for e in sorted(I)] + [("-",) + e for e in sorted(D)]
    status, merged = OV.deletion_batch(g, W.batch_from_list(ups), [v])
    assert status == "ok"
    E2 = {e for e in (E | I) - D if v not in e}
    M1, M2 = _matches(g, q, E), _matches(g, q, E2)
    r = O1.bdsm(g, q, merged)
    assert r["status"] == "ok" and r["E2"] == E2
    assert r["plus"] == M2 - M1 and r["minus"] == M1 - M2
    o = O2.run(g, q, merged, want_tuples=True)
    assert o.status == 0 and o.tuple_set(1) == M2 - M1 and o.tuple_set(0) == M1 - M2


def test_vertex_deletion_errors():
    g = W.graph_from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)], [0, 0, 0, 0, 0])
    ins_at_dead = W.batch_from_list([("+", 0, 2)])
    assert OV.deletion_batch(g, ins_at_dead, [2])[0] == "conflict"
    assert OV.deletion_batch(g, ins_at_dead, [0])[0] == "conflict"
    assert OV.deletion_batch(g, ins_at_dead, [4])[0] == "ok"
    assert OV.deletion_batch(g, ins_at_dead, [5])[0] == "invalid"
    # an explicit deletion of an edge at the deleted vertex is a duplicate
    status, merged = OV.deletion_batch(g, W.batch_from_list([("-", 2, 1)]), [1])
    assert status == "ok" and len(merged) == 3
    r = O1.bdsm(g, W.query_from_edges(2, [(0, 1)], (0, 0)), merged)
    assert r["n_dup"] == 1 and r["D"] == [(0, 1), (1, 2)]
    # deleting an isolated vertex contributes nothing
    g2 = W.graph_from_edges(3, [(0, 1)], [0, 0, 0])
    status, merged = OV.deletion_batch(g2, W.batch_from_list([]), [2])
    assert status == "ok" and len(merged) == 0


@pytest.mark.parametrize("seed", range(4))
def test_vertex_insertion(seed):
    """New vertices are isolated: no match of a query with an edge changes;
    their edges then arrive as ordinary insertions."""
    g, rng = _graph(seed, 7, 8, 2)
    q = _query(rng, 3, 2)
    new_labels = rng.integers(0, 2, 3).tolist()
    g2 = OV.with_vertices(g, new_labels)
    assert g2.n == g.n + 3 and list(g2.labels[g.n:]) == new_labels
    assert O1.edge_set(g2) == O1.edge_set(g)
    assert _matches(g2, q, O1.edge_set(g2)) == _matches(g, q, O1.edge_set(g))
    ups = [("+", g.n + i, int(w)) for i in range(3) for w in rng.permutation(g.n)[:3].tolist()]
    ups.append(("+", g.n, g.n + 1))
    b = W.batch_from_list(ups)
    r = O1.bdsm(g2, q, b)
    assert r["status"] == "ok" and r["minus"] == set()
    assert all(set(f) & {g.n, g.n + 1, g.n + 2} for f in r["plus"])
    o = O2.run(g2, q, b, want_tuples=True)
    assert o.status == 0 and o.tuple_set(1) == r["plus"]


def test_vertex_deletion_on_labelled_graph():
    """On an edge-labelled graph a deleted vertex takes each of its edges
    with that edge's label."""
    g = W.graph_from_labelled_edges(5, [(0, 1, 0), (1, 3, 1), (1, 2, 1), (2, 3, 0), (3, 4, 2)], [0] * 5, 3)
    q = W.query_from_edges(2, [(0, 1)], (0, 0), elabels=[1])
    empty = W.Batch(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint8), np.zeros(0, np.uint32))
    status, merged = OV.deletion_batch(g, empty, [1])
    assert status == "ok" and len(merged) == 3 and sorted(merged.elab.tolist()) == [0, 1, 1]
    r = O1.bdsm_el(g, q, merged)
    assert r["status"] == "ok" and r["plus"] == set()
    assert r["minus"] == {(1, 3), (3, 1), (1, 2), (2, 1)}
    assert r["E2"] == {(2, 3, 0), (3, 4, 2)}
    o = O2.run(g, q, merged)
    assert o.tuple_set(0) == r["minus"]
