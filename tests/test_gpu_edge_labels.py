"""GPU: edge-labelled graphs (Sec. II-A: the labelling function covers edges;
a query edge with label e maps only onto data edges with label e).

The library keeps one row per (vertex, edge label); everything else of the
path is the unlabelled one.  Results must equal the oracle's exactly: tuple
sets, counts, checksums, the canonical batch with per-update attribution,
and G' after the batch.  Inputs: seeded graphs whose edge labels follow a
skewed distribution (a few frequent labels and a tail), labelled queries of
several shapes, and batches with insertions, deletions, duplicates and
no-ops (deletions under a wrong label, insertions of present triples)."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import plain as O2
from oracle import vertices as OV
from paper_2401_17018_amd import GammaError, capi
from test_gpu_parity import _er, make_ctx

pytestmark = pytest.mark.gpu


def _labelled_er(n, m, seed, n_labels, n_el, skew=1.0):
    return W.with_edge_labels(_er(n, m, seed, n_labels), n_el, seed + 17, skew)


def _labelled_rmat(scale, m, seed, n_labels, n_el):
    lo, hi = W.rmat_edges(scale, m, seed)
    rp, col = W.csr_from_edges(1 << scale, lo, hi)
    g = W.Graph(1 << scale, rp, col, W.labels_uniform(1 << scale, n_labels, seed + 1))
    return W.with_edge_labels(g, n_el, seed + 29, 1.2)


def _edge_label_of(g):
    """Undirected edge key lo << 32 | hi -> label."""
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr).astype(np.int64))
    keep = src < g.col.astype(np.uint64)
    keys = (src[keep] << np.uint64(32)) | g.col.astype(np.uint64)[keep]
    return dict(zip(keys.tolist(), g.elab[keep].tolist()))


def _labelled_batch(g, seed, n_ins, n_del, n_noop=0, n_dup=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    lab = _edge_label_of(g)
    keys = np.array(sorted(lab), dtype=np.uint64)
    ups = []
    used = set()
    for k in keys[rng.permutation(len(keys))[:n_del]].tolist():
        ups.append((k >> 32, k & 0xFFFFFFFF, lab[k], 0))
        used.add(k)
    draws = W.skewed_edge_label_draws(n_ins, g.n_elabels, seed + 5)
    while len(ups) < n_del + n_ins:
        u, v = (int(x) for x in rng.integers(0, g.n, 2))
        k = (min(u, v) << 32) | max(u, v)
        if u == v or k in lab or k in used:
            continue
        used.add(k)
        ups.append((u, v, int(draws[len(ups) - n_del]), 1))
    for k in keys[rng.permutation(len(keys))].tolist():
        if n_noop <= 0:
            break
        if k in used:
            continue
        used.add(k)
        if g.n_elabels > 1 and rng.random() < 0.5:
            ups.append((k >> 32, k & 0xFFFFFFFF, (lab[k] + 1) % g.n_elabels, 0))  # deletion under a wrong label
        else:
            ups.append((k & 0xFFFFFFFF, k >> 32, lab[k], 1))  # insertion of a present triple
        n_noop -= 1
    for i in rng.permutation(len(ups))[:n_dup].tolist():
        a, b, e, o = ups[i]
        ups.append((b, a, e, o))
    order = rng.permutation(len(ups))
    ups = [ups[i] for i in order]
    flip = rng.random(len(ups)) < 0.5
    src = np.array([b if f else a for (a, b, _, _), f in zip(ups, flip)], np.uint32)
    dst = np.array([a if f else b for (a, b, _, _), f in zip(ups, flip)], np.uint32)
    return W.Batch(src, dst, np.array([u[3] for u in ups], np.uint8), np.array([u[2] for u in ups], np.uint32))


def _setup(ctx, g, qs):
    ctx.load_graph(g.row_ptr, g.col, g.labels, elabels=g.elab, n_elabels=g.n_elabels)
    for q in qs:
        ctx.register_query(q.k, q.labels, q.edges, elabels=q.elabels)


def _run(g, qs, b, cap=1 << 22, tuples=True, **tuning):
    with make_ctx(cap=cap) as ctx:
        _setup(ctx, g, qs)
        if tuning:
            ctx.set_tuning(**tuning)
        res = ctx.apply_batch(b.src, b.dst, b.op, elab=b.elab, tuples=tuples, seed_attr=tuples, per_update=True,
                              canonical=True)
        after = ctx.export_graph_el()
    return res, after


def _check(res, g, q, b, qid=0, check_tuples=True):
    ref = O2.run(g, q, b, qid=qid, threads=4, want_tuples=check_tuples)
    assert ref.status == 0
    for sign in (0, 1):
        assert res.count(qid, sign) == ref.count[sign], (qid, sign, res.count(qid, sign), ref.count[sign])
        assert int(res.hash_sum[qid, sign]) == ref.hsum[sign] and int(res.hash_xor[qid, sign]) == ref.hxor[sign]
        if check_tuples:
            assert res.tuple_set(qid, sign, q.k) == ref.tuple_set(sign)
    assert np.array_equal(res.canon_lo, ref.canon_lo) and np.array_equal(res.canon_hi, ref.canon_hi)
    assert np.array_equal(res.canon_sign, ref.canon_sign)
    return ref


def _check_graph(after, g, b):
    rp, col, el = O2.updated_graph_el(g, b)
    arp, acol, alab, ael, nel = after
    assert nel == g.n_elabels and np.array_equal(alab, g.labels)
    assert np.array_equal(arp, rp) and np.array_equal(acol, col) and np.array_equal(ael, el)


QUERIES = {
    "path3": (3, [(0, 1), (1, 2)], (0, 1, 0), [0, 1]),
    "triangle": (3, [(0, 1), (1, 2), (2, 0)], (0, 1, 2), [0, 0, 1]),
    "cycle4_chord": (4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)], (0, 1, 0, 1), [1, 0, 1, 0, 0]),
    "star": (4, [(0, 1), (0, 2), (0, 3)], (2, 0, 1, 0), [0, 1, 0]),
    "path5": (5, [(0, 1), (1, 2), (2, 3), (3, 4)], (0, 1, 2, 0, 1), [0, 0, 1, 0, 2]),
}


@pytest.mark.parametrize("n_el", [2, 5, 7])
def test_labelled_queries_match_oracle(n_el):
    g = _labelled_er(1200, 9000, 50 + n_el, 3, n_el)
    qs = [W.query_from_edges(k, e, l, elabels=[x % n_el for x in el]) for (k, e, l, el) in QUERIES.values()]
    b = _labelled_batch(g, n_el, 400, 150, n_noop=60, n_dup=30)
    print("[elabels] n_el=%d: %d updates" % (n_el, len(b)), flush=True)
    res, after = _run(g, qs, b)
    assert res.stats["n_noop"] == 60 and res.stats["n_duplicate"] == 30
    refs = [_check(res, g, q, b, qid=i, check_tuples=not res.truncated) for i, q in enumerate(qs)]
    assert sum(r.count[0] + r.count[1] for r in refs) > 0
    # per-update attribution of query 0
    assert np.array_equal(res.upd_count, np.sum([r.seed_count for r in refs], axis=0))
    _check_graph(after, g, b)


def test_labelled_skewed_graph_with_handover():
    g = _labelled_rmat(12, 30000, 3, 2, 4)
    qs = [W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 1, 0, 1), elabels=[0, 0, 1]),
          W.query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 1), elabels=[0, 1, 1])]
    b = _labelled_batch(g, 8, 300, 100)
    on, _ = _run(g, qs, b, waves_per_cu=4, poll_cycles=500, split_inner=2, split_leaf=2, handover_gate=1024)
    off, after = _run(g, qs, b, steal=2)
    assert on.stats["steals"] > 0
    assert np.array_equal(on.counts, off.counts) and np.array_equal(on.upd_count, off.upd_count)
    for qid, q in enumerate(qs):
        _check(on, g, q, b, qid=qid, check_tuples=not on.truncated)
    _check_graph(after, g, b)


def test_one_edge_label_equals_unlabelled():
    g = _er(900, 6000, 61, 3)
    gl = W.Graph(g.n, g.row_ptr, g.col, g.labels, elab=np.zeros_like(g.col), n_elabels=1)
    q = W.query_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], (0, 1, 0, 2))
    b = _labelled_batch(gl, 4, 300, 100)
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        plain = ctx.apply_batch(b.src, b.dst, b.op, tuples=True, per_update=True)
    ql = W.query_from_edges(q.k, q.edges.tolist(), q.labels.tolist(), elabels=[0] * q.m)
    res, _ = _run(gl, [ql], b)
    assert np.array_equal(res.counts, plain.counts) and np.array_equal(res.hash_sum, plain.hash_sum)
    assert np.array_equal(res.upd_count, plain.upd_count)
    assert res.tuple_set(0, 1, 4) == plain.tuple_set(0, 1, 4)


def test_coalesced_search_respects_edge_labels():
    """Automorphisms must preserve edge labels: a triangle with labels
    (0, 0, 1) keeps only the swap that fixes its label-1 edge."""
    g = _labelled_er(150, 3500, 71, 1, 2, skew=0.3)
    shapes = [(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 0), [0, 0, 1]),
              (3, [(0, 1), (1, 2), (2, 0)], (0, 0, 0), [1, 1, 1]),
              (4, [(0, 1), (1, 2), (2, 3), (3, 0)], (0, 0, 0, 0), [0, 1, 0, 1])]
    b = _labelled_batch(g, 9, 150, 60)
    for (k, e, l, el) in shapes:
        q = W.query_from_edges(k, e, l, elabels=el)
        on, _ = _run(g, [q], b, coalesced_search=2)
        off, _ = _run(g, [q], b, coalesced_search=1)
        assert np.array_equal(on.counts, off.counts) and np.array_equal(on.hash_xor, off.hash_xor)
        assert np.array_equal(on.upd_count, off.upd_count)
        assert on.tuple_set(0, 1, k) == off.tuple_set(0, 1, k)
        _check(on, g, q, b, check_tuples=not on.truncated)
        assert on.count(0, 1) + on.count(0, 0) > 0


def test_label_errors_leave_graph():
    g = _labelled_er(300, 1500, 81, 2, 3)
    lab = _edge_label_of(g)
    k0 = min(lab)
    a, c = k0 >> 32, k0 & 0xFFFFFFFF
    q = W.query_from_edges(2, [(0, 1)], (0, 1), elabels=[0])
    u32 = lambda *x: np.array(x, np.uint32)
    with make_ctx(cap=0) as ctx:
        _setup(ctx, g, [q])
        before = ctx.export_graph_el()
        cases = [
            ((u32(5, 6), u32(6, 5), np.array([1, 1], np.uint8), u32(0, 1)), capi.GAMMA_ECONFLICT),  # two labels, one pair
            ((u32(5), u32(6), np.array([1], np.uint8), u32(3)), capi.GAMMA_EINVAL),  # label >= n_elabels
            ((u32(a), u32(c), np.array([1], np.uint8), u32((lab[k0] + 1) % 3)), capi.GAMMA_EINVAL),  # relabel
        ]
        for (s, d, o, el), want in cases:
            with pytest.raises(GammaError) as ei:
                ctx.apply_batch(s, d, o, elab=el)
            assert ei.value.status == want
            now = ctx.export_graph_el()
            for x, y in zip(now[:4], before[:4]):
                assert np.array_equal(x, y)
        # a mirror entry with another label, and two edges on one pair, are rejected at load
        bad = g.elab.copy()
        bad[0] = (bad[0] + 1) % 3
        with pytest.raises(GammaError) as ei:
            ctx.load_graph(g.row_ptr, g.col, g.labels, elabels=bad, n_elabels=3)
        assert ei.value.status == capi.GAMMA_EINVAL
        multi = W.Graph(2, np.array([0, 2, 4], np.uint64), u32(1, 1, 0, 0), u32(0, 0), elab=u32(0, 1, 0, 1),
                        n_elabels=2)
        with pytest.raises(GammaError) as ei:
            ctx.load_graph(multi.row_ptr, multi.col, multi.labels, elabels=multi.elab, n_elabels=2)
        assert ei.value.status == capi.GAMMA_EINVAL
        now = ctx.export_graph_el()
        assert np.array_equal(now[1], before[1]) and np.array_equal(now[3], before[3])


def test_query_labels_the_graph_lacks():
    g = _labelled_er(400, 2500, 91, 1, 3)
    qs = [W.query_from_edges(2, [(0, 1)], (0, 0), elabels=[5]),  # beyond n_elabels: no rows at all
          W.query_from_edges(2, [(0, 1)], (0, 0), elabels=[2])]
    b = _labelled_batch(g, 3, 200, 50)
    res, _ = _run(g, qs, b)
    assert res.counts[0].sum() == 0
    ref = _check(res, g, qs[1], b, qid=1)
    n2 = int(np.sum(b.elab[b.op == 1] == 2))
    assert ref.count[1] == 2 * n2  # every inserted label-2 edge, both orientations (all pairs are new)


def test_labelled_vertex_deletion_and_sequence():
    g = _labelled_er(700, 5000, 101, 2, 4)
    q = W.query_from_edges(3, [(0, 1), (1, 2)], (0, 1, 0), elabels=[1, 0])
    b1 = _labelled_batch(g, 11, 200, 80)
    deg = np.diff(g.row_ptr)
    vdel = np.argsort(-deg)[:3].astype(np.uint32)
    dead = set(vdel.tolist())
    keep = np.array([not (o == 1 and (int(s) in dead or int(d) in dead)) for s, d, o in zip(b1.src, b1.dst, b1.op)])
    b1 = W.Batch(b1.src[keep], b1.dst[keep], b1.op[keep], b1.elab[keep])
    status, merged = OV.deletion_batch(g, b1, vdel)
    assert status == "ok"
    with make_ctx() as ctx:
        _setup(ctx, g, [q])
        r1 = ctx.apply_batch(b1.src, b1.dst, b1.op, elab=b1.elab, delete_vertices=vdel, tuples=True,
                             canonical=True)
        g1 = ctx.export_graph_el()
        G1 = W.Graph(g.n, g1[0], g1[1], g1[2], elab=g1[3], n_elabels=g1[4])
        b2 = _labelled_batch(G1, 12, 150, 150)
        r2 = ctx.apply_batch(b2.src, b2.dst, b2.op, elab=b2.elab, tuples=True, canonical=True)
        g2 = ctx.export_graph_el()
    _check(r1, g, q, merged)
    _check_graph(g1, g, merged)
    assert all(g1[0][v + 1] == g1[0][v] for v in vdel.tolist())
    _check(r2, G1, q, b2)
    _check_graph(g2, G1, b2)
