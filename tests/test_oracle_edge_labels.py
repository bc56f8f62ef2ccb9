"""Pins for the oracle on edge-labelled graphs (Sec. II-A: the labelling
function covers vertices and edges; a query edge with label e maps onto a
data edge with label e).

O2 (the incremental enumerator) is checked against O1 (brute force over the
labelled triples), and O1 itself against something other than itself: the
subdivision identity, under which an edge-labelled match is exactly a
vertex-labelled match once every edge becomes a middle vertex carrying the
edge's label, checked through the unlabelled brute force that the other
pin files already tie to the definitions.  With one edge label everything
must reduce to the unlabelled results."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import workloads as W
from oracle import brute as O1
from oracle import plain as O2


def _labelled_graph(rng, n, m_try, n_labels, n_el):
    tri = set()
    pairs = set()
    for _ in range(m_try):
        u, v = (int(x) for x in rng.integers(0, n, 2))
        if u == v:
            continue
        p = (min(u, v), max(u, v))
        e = int(rng.integers(0, n_el))
        if p in pairs:
            continue
        pairs.add(p)
        tri.add(p + (e,))
    return W.graph_from_labelled_edges(n, sorted(tri), rng.integers(0, n_labels, n).tolist(), n_el)


def _labelled_query(rng, k, n_labels, n_el):
    edges = {(i - 1, i) for i in range(1, k)}
    if k >= 3 and rng.random() < 0.6:
        edges.add((0, k - 1))
    if k >= 4 and rng.random() < 0.4:
        edges.add((1, k - 1))
    edges = sorted(edges)
    return W.query_from_edges(k, edges, rng.integers(0, n_labels, k).tolist(),
                              elabels=rng.integers(0, n_el, len(edges)).tolist())


def _labelled_batch(rng, g, n_upd, adversarial):
    """Insertions and deletions of labelled triples, with duplicates and
    no-ops when adversarial (deletions of a pair under a label it does not
    carry, insertions of present triples).  At most one triple per pair;
    new insertions go to absent pairs."""
    E = sorted(O1.edge_set_el(g))
    pairs = {(a, b) for (a, b, _) in E}
    ups, used = [], {}
    for _ in range(n_upd * 3):
        if len(ups) >= n_upd:
            break
        if E and rng.random() < 0.4:
            a, b, e = E[int(rng.integers(0, len(E)))]
            op = 0 if not adversarial or rng.random() < 0.7 else 1
            if adversarial and op == 0 and rng.random() < 0.3:
                e = int(rng.integers(0, g.n_elabels))
        else:
            a, b = (int(x) for x in rng.integers(0, g.n, 2))
            if a == b or (min(a, b), max(a, b)) in pairs:
                continue
            e, op = int(rng.integers(0, g.n_elabels)), 1
        p = (min(a, b), max(a, b))
        if p in used and used[p] != (op, e):
            continue
        used[p] = (op, e)
        ups.append((a, b, e, op))
        if adversarial and rng.random() < 0.15:
            ups.append((b, a, e, op))  # duplicate, other orientation
    src = np.array([u[0] for u in ups], np.uint32)
    dst = np.array([u[1] for u in ups], np.uint32)
    el = np.array([u[2] for u in ups], np.uint32)
    op = np.array([u[3] for u in ups], np.uint8)
    return W.Batch(src, dst, op, el)


def _check_o2_equals_o1(g, q, b, threads=1):
    r1 = O1.bdsm_el(g, q, b)
    r2 = O2.run(g, q, b, threads=threads)
    assert r1["status"] == "ok" and r2.status == 0
    assert r2.tuple_set(1) == r1["plus"] and r2.tuple_set(0) == r1["minus"]
    assert r2.count == (len(r1["minus"]), len(r1["plus"]))
    assert (r2.n_noop, r2.n_dup) == (r1["n_noop"], r1["n_dup"])
    assert sorted(zip(r2.canon_lo.tolist(), r2.canon_hi.tolist(), r2.canon_e.tolist())) == sorted(r1["I"] + r1["D"])
    # G' of O2 equals O1's E2
    rp, col, el = O2.updated_graph_el(g, b)
    g2 = W.Graph(g.n, rp, col, g.labels, elab=el, n_elabels=g.n_elabels)
    assert O1.edge_set_el(g2) == r1["E2"]
    return r1, r2


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(3, 8), k=st.integers(2, 4), extra=st.integers(0, 14),
       n_labels=st.integers(1, 2), n_el=st.integers(1, 3), adversarial=st.booleans())
def test_o2_equals_o1_labelled(seed, n, k, extra, n_labels, n_el, adversarial):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = _labelled_graph(rng, n, 2 * n + extra, n_labels, n_el)
    q = _labelled_query(rng, k, n_labels, n_el)
    b = _labelled_batch(rng, g, 10, adversarial)
    _check_o2_equals_o1(g, q, b)


# ---------------------------------------------------------------- subdivision


def _subdivide(g, q, b):
    """Vertex-labelled (G_sub, Q_sub, B_sub): every labelled edge (present or
    inserted by the batch) becomes a middle vertex with label L_V + e joined
    to both ends; query edge i becomes query vertex k + i."""
    LV = int(max(int(g.labels.max()), int(q.labels.max()))) + 1
    E = sorted(O1.edge_set_el(g))
    ins = [(min(s, d), max(s, d), int(e)) for s, d, e, o in zip(b.src.tolist(), b.dst.tolist(), b.elab.tolist(),
                                                                  b.op.tolist())]
    mids = {t: g.n + i for i, t in enumerate(sorted(set(E) | set(ins)))}
    labels = list(g.labels.tolist()) + [LV + t[2] for t in sorted(mids)]
    sub_edges = []
    for (lo, hi, e) in E:
        s = mids[(lo, hi, e)]
        sub_edges += [(lo, s), (hi, s)]
    gs = W.graph_from_edges(len(labels), sub_edges, labels)
    ups = []
    for s, d, e, o in zip(b.src.tolist(), b.dst.tolist(), b.elab.tolist(), b.op.tolist()):
        m = mids[(min(s, d), max(s, d), int(e))]
        sign = "+" if o else "-"
        ups += [(sign, s, m), (sign, m, d)]
    bs = W.batch_from_list(ups)
    qk, qe = q.k, [tuple(x) for x in q.edges.tolist()]
    qedges, qlabels = [], list(q.labels.tolist())
    for i, ((a, c), e) in enumerate(zip(qe, q.elabels.tolist())):
        qedges += [(a, qk + i), (qk + i, c)]
        qlabels.append(LV + int(e))
    qs = W.query_from_edges(qk + len(qe), qedges, qlabels)
    return gs, qs, bs


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(3, 7), k=st.integers(2, 4), extra=st.integers(0, 8),
       n_el=st.integers(1, 3))
def test_subdivision_identity(seed, n, k, extra, n_el):
    rng = np.random.Generator(np.random.PCG64(seed))
    g = _labelled_graph(rng, n, n + extra, 2, n_el)
    q = _labelled_query(rng, k, 2, n_el)
    b = _labelled_batch(rng, g, 4, False)
    gs, qs, bs = _subdivide(g, q, b)
    qe = [tuple(x) for x in q.edges.tolist()]
    # static match sets: projection to the original query vertices is a bijection
    M = O1.all_matches_el(g.n, g.labels, O1.edge_set_el(g), q.k, q.labels, qe, q.elabels.tolist())
    Ms = O1.all_matches(gs.n, gs.labels, O1.adjacency(gs.n, O1.edge_set(gs)), qs.k, qs.labels,
                        [tuple(x) for x in qs.edges.tolist()])
    assert {t[:q.k] for t in Ms} == M and len(Ms) == len(M)
    # incremental matches
    r = O1.bdsm_el(g, q, b)
    rs = O1.bdsm(gs, qs, bs)
    assert r["status"] == rs["status"] == "ok"
    assert {t[:q.k] for t in rs["plus"]} == r["plus"] and len(rs["plus"]) == len(r["plus"])
    assert {t[:q.k] for t in rs["minus"]} == r["minus"] and len(rs["minus"]) == len(r["minus"])


# ---------------------------------------------------------------- reductions


@pytest.mark.parametrize("seed", range(5))
def test_one_edge_label_is_unlabelled(seed):
    """With every label 0 the labelled oracles give the unlabelled results
    (tuples, checksums, attribution)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = _labelled_graph(rng, 30, 120, 2, 1)
    gu = W.Graph(g.n, g.row_ptr, g.col, g.labels)
    q = _labelled_query(rng, 4, 2, 1)
    qu = W.Query(q.k, q.labels, q.edges)
    b = _labelled_batch(rng, g, 25, True)
    bu = W.Batch(b.src, b.dst, b.op)
    r = O2.run(g, q, b, threads=2)
    ru = O2.run(gu, qu, bu, threads=2)
    assert r.tuple_set(0) == ru.tuple_set(0) and r.tuple_set(1) == ru.tuple_set(1)
    assert r.hsum == ru.hsum and r.hxor == ru.hxor
    assert np.array_equal(r.seed_count, ru.seed_count) and np.array_equal(r.seed_hsum, ru.seed_hsum)
    assert O1.bdsm_el(g, q, b)["plus"] == O1.bdsm(gu, qu, bu)["plus"]


def test_labels_restrict_matches():
    """A triangle whose edges carry labels 0, 1, 2: the query with the same
    labels matches it once per rotation that fits, a query asking for a
    label the triangle lacks does not."""
    g = W.graph_from_labelled_edges(3, [(0, 1, 0), (1, 2, 1), (0, 2, 2)], [0, 0, 0], 3)
    tri = [(0, 1), (1, 2), (2, 0)]
    E = O1.edge_set_el(g)
    assert O1.all_matches_el(3, g.labels, E, 3, [0, 0, 0], tri, [0, 1, 2]) == {(0, 1, 2)}
    assert O1.all_matches_el(3, g.labels, E, 3, [0, 0, 0], tri, [0, 0, 0]) == set()
    # deleting the label-1 edge removes the match; deleting it under label 0 is a no-op
    q = W.query_from_edges(3, tri, [0, 0, 0], elabels=[0, 1, 2])
    b = W.Batch(np.array([2], np.uint32), np.array([1], np.uint32), np.array([0], np.uint8), np.array([1], np.uint32))
    r1, r2 = _check_o2_equals_o1(g, q, b)
    assert r1["minus"] == {(0, 1, 2)} and r1["D"] == [(1, 2, 1)]
    wrong = W.Batch(np.array([2], np.uint32), np.array([1], np.uint32), np.array([0], np.uint8),
                    np.array([0], np.uint32))
    r1, r2 = _check_o2_equals_o1(g, q, wrong)
    assert r1["minus"] == set() and r2.n_noop == 1


def test_label_conflicts():
    g = W.graph_from_labelled_edges(4, [(0, 1, 0), (1, 2, 1)], [0, 0, 0, 0], 2)
    q = W.query_from_edges(2, [(0, 1)], [0, 0], elabels=[0])
    two_labels = W.Batch(np.array([2, 3], np.uint32), np.array([3, 2], np.uint32), np.array([1, 1], np.uint8),
                         np.array([0, 1], np.uint32))
    assert O1.bdsm_el(g, q, two_labels)["status"] == "conflict"
    assert O2.run(g, q, two_labels).status == -2
    bad = W.Batch(np.array([2], np.uint32), np.array([3], np.uint32), np.array([1], np.uint8), np.array([2], np.uint32))
    assert O1.bdsm_el(g, q, bad)["status"] == "invalid"
    assert O2.run(g, q, bad).status == -1
    # inserting a present pair under another label is invalid (the graph is simple)
    relabel = W.Batch(np.array([1], np.uint32), np.array([0], np.uint32), np.array([1], np.uint8),
                      np.array([1], np.uint32))
    assert O1.bdsm_el(g, q, relabel)["status"] == "invalid"
    assert O2.run(g, q, relabel).status == -1
    # deleting a pair under a label it does not carry is a no-op
    wrong = W.Batch(np.array([1], np.uint32), np.array([2], np.uint32), np.array([0], np.uint8),
                    np.array([0], np.uint32))
    r = O2.run(g, q, wrong)
    assert r.status == 0 and r.n_noop == 1 and r.n_canonical == 0
    # a graph with two edges on one pair is not accepted
    multi = W.graph_from_labelled_edges(2, [(0, 1, 0), (0, 1, 1)], [0, 0], 2)
    with pytest.raises(ValueError):
        O2.run(multi, q, wrong)


def test_planted_edge_label_mistake_is_caught():
    caught = False
    for seed in range(40):
        rng = np.random.Generator(np.random.PCG64(1000 + seed))
        g = _labelled_graph(rng, 7, 16, 1, 3)
        q = _labelled_query(rng, 3, 1, 3)
        b = _labelled_batch(rng, g, 6, False)
        r1 = O1.bdsm_el(g, q, b)
        r2 = O2.run(g, q, b, mutant=O2.MUT_NO_EDGE_LABEL_CHECK)
        if r2.tuple_set(1) != r1["plus"] or r2.tuple_set(0) != r1["minus"]:
            caught = True
            break
    assert caught
