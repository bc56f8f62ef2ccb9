"""GPU: the documented limits and degenerate inputs.

* a batch of exactly 2^20 updates (the per-call maximum) is applied and
  agrees with the oracle; 2^20 + 1 updates are rejected with the graph
  unchanged;
* queries of the maximum size, 16 vertices (planted on a random walk
  through an inserted edge, so the planted match must be found), agree
  with the oracle tuple for tuple; 17 vertices are rejected;
* a graph with no edges at all receives a batch of insertions, then one of
  deletions."""
import numpy as np
import pytest

import workloads as W
from oracle import plain as O2
from paper_2401_17018_amd import GammaError, capi
from test_gpu_parity import _er, check_against_o2, make_ctx

pytestmark = pytest.mark.gpu


def test_max_batch_size():
    n = 1 << 16
    g = _er(n, 200000, 61, 2)
    q = W.query_from_edges(2, [(0, 1)], (0, 1))
    rng = np.random.Generator(np.random.PCG64(61))
    m = 1 << 20
    src = rng.integers(0, n, m).astype(np.uint32)
    dst = rng.integers(0, n, m).astype(np.uint32)
    dst[src == dst] = (dst[src == dst] + 1) % n  # no self loops
    op = (rng.random(m) < 0.9).astype(np.uint8)
    # deletions name present edges so that they are not all no-ops
    E = g.edge_keys()
    pick = E[rng.integers(0, len(E), m)]
    dele = op == 0
    src[dele] = (pick[dele] >> np.uint64(32)).astype(np.uint32)
    dst[dele] = (pick[dele] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    # an edge both inserted and deleted would be a conflict: insertions keep to absent pairs
    keys = (np.minimum(src, dst).astype(np.uint64) << np.uint64(32)) | np.maximum(src, dst).astype(np.uint64)
    bad = (op == 1) & (np.isin(keys, E) | np.isin(keys, keys[dele]))
    op[bad] = 0
    src[bad] = (pick[bad] >> np.uint64(32)).astype(np.uint32)
    dst[bad] = (pick[bad] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    b = W.Batch(src, dst, op)
    assert len(b) == 1 << 20
    with make_ctx(cap=0) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        s1 = np.concatenate([src, src[:1]])
        d1 = np.concatenate([dst, dst[:1]])
        o1 = np.concatenate([op, op[:1]])
        with pytest.raises(GammaError) as ei:
            ctx.apply_batch(s1, d1, o1)
        assert ei.value.status == capi.GAMMA_EINVAL
        rp, col, _ = ctx.export_graph()
        assert np.array_equal(rp, g.row_ptr) and np.array_equal(col, g.col)
        res = ctx.apply_batch(src, dst, op, hash=True)
    ref = check_against_o2(res, g, q, b, check_tuples=False)
    assert res.stats["n_input"] == 1 << 20 and ref.n_insert > 900000 and ref.count[1] > 0 and ref.count[0] > 0


@pytest.mark.parametrize("kind,seed", [("sparse", 1), ("induced", 3)])
def test_max_query_size(kind, seed):
    n, m, L = (4000, 14000, 8) if kind == "sparse" else (3000, 12000, 6)
    lo, hi = W.er_edges(n, m, seed)
    rp, col = W.csr_from_edges(n, lo, hi)
    g = W.Graph(n, rp, col, W.labels_uniform(n, L, seed + 1))
    rng = np.random.Generator(np.random.PCG64(seed))
    E = set(g.edge_keys().tolist())
    ins = set()
    while len(ins) < 400:
        u, v = (int(x) for x in rng.integers(0, n, 2))
        k = (min(u, v) << 32) | max(u, v)
        if u != v and k not in E:
            ins.add(k)
    ins = np.array(sorted(ins), np.uint64)
    q = W.extract_query(g, ins, 16, kind, seed + 11)
    assert q.k == 16
    b = W.make_batch(ins, g.edge_keys()[rng.permutation(g.m)[:100]], W.Draws(seed, 99))
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        res = ctx.apply_batch(b.src, b.dst, b.op, tuples=True, per_update=True)
        with pytest.raises(GammaError) as ei:
            ctx.register_query(17, [0] * 17, [(i, i + 1) for i in range(16)])
        assert ei.value.status == capi.GAMMA_EUNSUPPORTED
    ref = check_against_o2(res, g, q, b)
    assert tuple(int(x) for x in q.planted) in res.tuple_set(0, 1, 16)
    assert np.array_equal(res.upd_count, ref.seed_count)


def test_graph_without_edges():
    n = 300
    g = W.Graph(n, np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32), W.labels_uniform(n, 2, 5))
    qs = [W.query_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], (0, 1, 0, 1)),
          W.query_from_edges(2, [(0, 1)], (1, 1))]
    lo, hi = W.er_edges(n, 2500, 71)
    keys = (lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64)
    b1 = W.make_batch(keys, np.zeros(0, np.uint64), W.Draws(71, 1))
    b2 = W.make_batch(np.zeros(0, np.uint64), keys[::2], W.Draws(71, 2))
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        r1 = ctx.apply_batch(b1.src, b1.dst, b1.op, tuples=True)
        rp1, col1, _ = ctx.export_graph()
        r2 = ctx.apply_batch(b2.src, b2.dst, b2.op, tuples=True)
    g1 = W.Graph(n, rp1, col1, g.labels)
    for qid, q in enumerate(qs):
        check_against_o2(r1, g, q, b1, qid=qid)
        check_against_o2(r2, g1, q, b2, qid=qid)
    assert r1.counts[:, 0].sum() == 0 and r1.counts[:, 1].sum() > 0
    assert r2.counts[:, 1].sum() == 0 and r2.counts[:, 0].sum() > 0
