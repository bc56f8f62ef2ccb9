"""GPU: coalesced search over a k-degenerated automorphic subgraph (Sec. V-B).

For a query whose own automorphism group is trivial but whose core (the
query without its degree-1 vertices) is symmetric, coalesced_search = 3
searches the core-edge plans of one orbit once, permutes each core match
found by the core's automorphisms and matches the removed vertices anew for
every permutation.  Results must equal the oracle's (which searches every
directed edge with no coalescing) and the library's own with coalescing
off, exactly: tuple sets, counts, checksums and per-update attribution."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from test_gpu_parity import _er, _mixed_batch, _skewed_graph, check_against_o2, make_ctx
from test_gpu_tuning import _same

pytestmark = pytest.mark.gpu

# (k, edges, vertex labels): symmetric cores whose leaves break the symmetry
CORE_SYMMETRIC = {
    # triangle A-B-B with a leaf on one B vertex (core group of order 2)
    "triangle_leaf": (4, [(0, 1), (1, 2), (2, 0), (1, 3)], (0, 1, 1, 2)),
    # 4-cycle with differently labelled leaves on two adjacent vertices (order 8)
    "cycle4_leaves": (6, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 5)], (0, 0, 0, 0, 1, 2)),
    # two triangles on a shared edge, leaves on a shared and an unshared vertex (order 4)
    "diamond_leaves": (6, [(0, 1), (1, 2), (2, 0), (1, 3), (3, 0), (0, 4), (2, 5)], (0, 0, 0, 0, 1, 2)),
    # K4 with three differently labelled leaves (order 24: one orbit of 12 directed edges)
    "k4_leaves": (7, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (0, 4), (1, 5), (2, 6)],
                  (0, 0, 0, 0, 1, 2, 3)),
    # 5-cycle with differently labelled leaves on two adjacent vertices (order 10)
    "cycle5_leaves": (7, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 5), (1, 6)], (0, 0, 0, 0, 0, 1, 2)),
}


def _query(name, elabels=None):
    k, edges, labels = CORE_SYMMETRIC[name]
    return W.query_from_edges(k, edges, labels, elabels=elabels)


def _run(g, qs, b, mode, elab=False, **tuning):
    # a search that does not end fails the test (the deadline aborts it)
    with make_ctx(cap=1 << 22, deadline_ms=30000) as ctx:
        if elab:
            ctx.load_graph(g.row_ptr, g.col, g.labels, elabels=g.elab, n_elabels=g.n_elabels)
        else:
            ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges, elabels=q.elabels if elab else None)
        ctx.set_tuning(coalesced_search=mode, **tuning)
        return ctx.apply_batch(b.src, b.dst, b.op, elab=b.elab if elab else None, tuples=True, seed_attr=True,
                               per_update=True)


def _keys(a, b):
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    return (np.minimum(a, b) << np.uint64(32)) | np.maximum(a, b)


def _graph_for(name, seed):
    # the denser shapes need a dense graph to occur at all
    if name in ("k4_leaves", "diamond_leaves"):
        return _er(150, 3600, seed, 4)
    return _er(400, 3200, seed, 4)


def test_shapes_have_trivial_groups_and_symmetric_cores():
    """The queries above are what the mode is for: no automorphism of the
    whole query, a core with one."""
    for name, (k, edges, labels) in CORE_SYMMETRIC.items():
        assert len(CF.automorphisms(k, labels, edges)) == 1, name
        deg = np.zeros(k, int)
        for a, b in edges:
            deg[a] += 1
            deg[b] += 1
        core = [u for u in range(k) if deg[u] >= 2]
        cid = {u: i for i, u in enumerate(core)}
        ce = [(cid[a], cid[b]) for a, b in edges if a in cid and b in cid]
        assert len(CF.automorphisms(len(core), [labels[u] for u in core], ce)) > 1, name


@pytest.mark.parametrize("name", sorted(CORE_SYMMETRIC))
def test_core_coalescing_matches_oracle(name):
    q = _query(name)
    k = q.k
    g = _graph_for(name, 31 + k)
    b = _mixed_batch(g, 5 + k, 200, 80)
    print("[core] %s: n=%d m=%d updates=%d" % (name, g.n, g.m, len(b)), flush=True)
    on = _run(g, [q], b, 3)
    off = _run(g, [q], b, 1)
    _same(on, off)
    for sign in (0, 1):
        assert on.tuple_set(0, sign, k) == off.tuple_set(0, sign, k)
    check_against_o2(on, g, q, b, check_tuples=not on.truncated)
    assert on.count(0, 1) + on.count(0, 0) > 0
    # only the representatives of the core-edge orbits are seeded
    assert on.stats["n_seeds"] < off.stats["n_seeds"]


@pytest.mark.parametrize("name", ["triangle_leaf", "cycle4_leaves", "k4_leaves"])
def test_core_coalescing_with_handover(name):
    """Long core ranges on a skewed graph, hand-over forced as often as
    possible: parts of core levels are handed over while the donor is past
    the core under a permuted prefix, and parts of the levels past the core
    under each permutation."""
    q = _query(name)
    lo, hi = W.rmat_edges(11, 16000, 7)
    rp, col = W.csr_from_edges(1 << 11, lo, hi)
    g = W.Graph(1 << 11, rp, col, W.labels_uniform(1 << 11, 6, 8))
    b = _mixed_batch(g, 17, 300, 120)
    tun = dict(waves_per_cu=4, poll_cycles=500, split_inner=2, split_leaf=2, handover_gate=1024)
    on = _run(g, [q], b, 3, **tun)
    off = _run(g, [q], b, 1)
    _same(on, off)
    assert on.stats["steals"] > 0
    # every hand-over splits a piece of at least two units, so hand-overs
    # stay within a small multiple of the search nodes (a piece handed on
    # unsplit could circulate among idle waves without end)
    assert on.stats["steals"] < 4 * on.stats["dfs_nodes"] + 1000
    check_against_o2(on, g, q, b, check_tuples=not on.truncated)


def test_core_coalescing_edge_labels():
    """Edge labels take part in the core's automorphisms: the triangle's two
    edges at its A vertex share a label, so B-B swaps; with another label on
    one of them the core has no symmetry left and nothing is coalesced."""
    # every pair carries one label, a function of the pair: deletions then
    # name their edge's label and insertions a fixed one
    g = _er(200, 4000, 41, 3)
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr).astype(np.int64))
    g = W.Graph(g.n, g.row_ptr, g.col, g.labels, elab=W.pair_edge_labels(_keys(src, g.col), 2, 43), n_elabels=2)
    b = _mixed_batch(g, 45, 220, 90)
    b = W.Batch(b.src, b.dst, b.op, W.pair_edge_labels(_keys(b.src, b.dst), 2, 43))
    k, edges, labels = 4, [(0, 1), (1, 2), (2, 0), (1, 3)], (0, 1, 1, 2)
    sym = W.query_from_edges(k, edges, labels, elabels=[1, 0, 1, 1])
    asym = W.query_from_edges(k, edges, labels, elabels=[1, 0, 0, 1])
    for q, coalesced in ((sym, True), (asym, False)):
        on = _run(g, [q], b, 3, elab=True)
        off = _run(g, [q], b, 1, elab=True)
        _same(on, off)
        for sign in (0, 1):
            assert on.tuple_set(0, sign, k) == off.tuple_set(0, sign, k)
        check_against_o2(on, g, q, b, check_tuples=not on.truncated)
        assert on.count(0, 1) + on.count(0, 0) > 0
        if coalesced:
            assert on.stats["n_seeds"] < off.stats["n_seeds"]
        else:
            assert on.stats["n_seeds"] == off.stats["n_seeds"]


@pytest.mark.parametrize("query_launch", [1, 2])
def test_core_coalescing_many_queries(query_launch):
    """Core-coalesced, whole-query-coalesced and plain queries in one launch
    (a symmetric query keeps its k = 0 groups under mode 3)."""
    g = _er(300, 3000, 53, 4)
    qs = [_query("triangle_leaf"), _query("cycle5_leaves"),
          W.query_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)], (0, 0, 0, 0)),
          W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 1, 2, 3))]
    b = _mixed_batch(g, 55, 250, 100)
    on = _run(g, qs, b, 3, query_launch=query_launch)
    off = _run(g, qs, b, 1, query_launch=query_launch)
    k0 = _run(g, qs, b, 2, query_launch=query_launch)
    _same(on, off)
    _same(k0, off)
    for qid, q in enumerate(qs):
        check_against_o2(on, g, q, b, qid=qid, check_tuples=not on.truncated)


def test_mode_switches_on_one_context():
    """Switching the mode rebuilds the candidate filters (relaxed over the
    core's orbits under mode 3, exact otherwise); dry runs in every mode and
    then a committed batch agree with the oracle."""
    g = _er(300, 3600, 61, 4)
    q = _query("triangle_leaf")
    b = _mixed_batch(g, 63, 200, 80)
    ref = None
    with make_ctx(cap=1 << 22) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        for mode in (3, 2, 3, 1, 3):
            ctx.set_tuning(coalesced_search=mode)
            r = ctx.apply_batch(b.src, b.dst, b.op, tuples=True, per_update=True, dry_run=True)
            if ref is None:
                ref = r
                check_against_o2(r, g, q, b)
            else:
                _same(r, ref)
        ctx.set_tuning(coalesced_search=3)
        r = ctx.apply_batch(b.src, b.dst, b.op, tuples=True, per_update=True)
        _same(r, ref)
        rp, col, _ = ctx.export_graph()
        g1 = W.Graph(g.n, rp, col, g.labels)
        b2 = _mixed_batch(g1, 65, 150, 60)
        r2 = ctx.apply_batch(b2.src, b2.dst, b2.op, tuples=True, per_update=True)
    check_against_o2(r2, g1, q, b2)


def test_core_orbit_split_into_groups():
    """K5 with differently labelled leaves on four of its vertices: the
    core's 20 directed edges form one orbit, searched as two groups (16 and
    4 permutations)."""
    k = 9
    edges = [(a, b) for a in range(5) for b in range(a + 1, 5)] + [(0, 5), (1, 6), (2, 7), (3, 8)]
    q = W.query_from_edges(k, edges, (0, 0, 0, 0, 0, 1, 2, 3, 4))
    n = 150
    lo, hi = W.er_edges(n, 3200, 77)
    rp, col = W.csr_from_edges(n, lo, hi)
    rng = np.random.Generator(np.random.PCG64(78))
    g = W.Graph(n, rp, col, np.where(rng.random(n) < 0.4, 0, rng.integers(1, 5, n)).astype(np.uint32))
    b = _mixed_batch(g, 79, 200, 80)
    on = _run(g, [q], b, 3)
    off = _run(g, [q], b, 1)
    _same(on, off)
    for sign in (0, 1):
        assert on.tuple_set(0, sign, k) == off.tuple_set(0, sign, k)
    check_against_o2(on, g, q, b, check_tuples=not on.truncated)
    assert on.count(0, 1) + on.count(0, 0) > 0
    assert on.stats["n_seeds"] < off.stats["n_seeds"]


def test_served_stream_with_core_coalescing():
    """A served stream whose queries are core-coalesced: every device batch
    the server forms reports what coalescing off reports for the same
    batch on the same graph state, and the oracle agrees."""
    from paper_2401_17018_amd import Server
    from test_gpu_serve import _request_stream
    g = _er(400, 3600, 61, 4)
    qs = [_query("triangle_leaf"), _query("cycle4_leaves")]
    reqs = _request_stream(g, 5, 24, 60)
    with make_ctx(cap=0, deadline_ms=30000) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        ctx.set_tuning(coalesced_search=3)
        with Server(ctx, max_batch_updates=150) as srv:
            for r in reqs:
                srv.submit(*r)
            srv.drain()
            n_bat = srv.counts()[2]
            batches = [srv.batch(i) for i in range(n_bat)]
    assert sum(b["n_requests"] for b in batches) == len(reqs)
    total = 0
    with make_ctx(cap=0, deadline_ms=30000) as plain:
        plain.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            plain.register_query(q.k, q.labels, q.edges)
        plain.set_tuning(coalesced_search=1)
        for b in batches:
            rs = reqs[b["first_ticket"]:b["first_ticket"] + b["n_requests"]]
            merged = W.Batch(np.concatenate([r[0] for r in rs]), np.concatenate([r[1] for r in rs]),
                             np.concatenate([r[2] for r in rs]))
            rp, col, lab = plain.export_graph()
            before = W.Graph(len(lab), rp, col, lab)
            res = plain.apply_batch(merged.src, merged.dst, merged.op, hash=True)
            assert np.array_equal(res.counts, b["counts"])
            assert np.array_equal(res.hash_sum, b["hash_sum"]) and np.array_equal(res.hash_xor, b["hash_xor"])
            for qid, q in enumerate(qs):
                ref = _o2(before, q, merged, qid)
                assert [int(res.counts[qid, 0]), int(res.counts[qid, 1])] == [ref.count[0], ref.count[1]]
            total += int(res.counts.sum())
    assert total > 0


def _o2(g, q, b, qid):
    from oracle import plain as O2
    r = O2.run(g, q, b, qid=qid, threads=4, want_tuples=False)
    assert r.status == 0
    return r


def test_vertex_deletions_with_core_coalescing():
    """Vertex deletions expanded on the device, under coalescing over the
    core: equal to coalescing off and to the oracle on the merged batch."""
    from test_gpu_vertices import _vertex_case
    g = _er(400, 3600, 71, 4)
    qs = [_query("triangle_leaf"), _query("cycle4_leaves")]
    b, vdel, merged = _vertex_case(g, 73, 150, 50, 6)
    outs = []
    for mode in (3, 1):
        with make_ctx(cap=1 << 22, deadline_ms=30000) as ctx:
            ctx.load_graph(g.row_ptr, g.col, g.labels)
            for q in qs:
                ctx.register_query(q.k, q.labels, q.edges)
            ctx.set_tuning(coalesced_search=mode)
            outs.append(ctx.apply_batch(b.src, b.dst, b.op, delete_vertices=vdel, tuples=True, per_update=True))
    _same(outs[0], outs[1])
    for qid, q in enumerate(qs):
        for sign in (0, 1):
            assert outs[0].tuple_set(qid, sign, q.k) == outs[1].tuple_set(qid, sign, q.k)
        ref = _o2(g, q, merged, qid)
        assert [outs[0].count(qid, 0), outs[0].count(qid, 1)] == [ref.count[0], ref.count[1]]
    assert int(outs[0].counts.sum()) > 0
