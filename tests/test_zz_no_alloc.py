"""GPU: gamma_apply_batch_noalloc (the entry point for callers that cannot
allocate device memory) against gamma_apply_batch and the oracle.

Two batches in a row, the second smaller, each applied through the
no-allocation entry point after a dry run of the same batch through
gamma_apply_batch from the same graph state: counts, checksums, the
canonical batch and per-update attribution must be identical, and equal to
the oracle's.  Also: the graph after both batches equals the oracle's G'',
tuple output is refused, and a batch whose buffers exceed the static
scratch is refused with the graph unchanged."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import plain as O2
from paper_2401_17018_amd import Context, GammaError, capi

pytestmark = pytest.mark.gpu


def _graph_and_batches():
    g, pl, ph = W.rmat_graph_with_pool(14, 8 << 14, 6000, 3, 1.2, 7, name="noalloc-rmat14")
    pool = W.keys_of(pl, ph)
    shadow = W.EdgeShadow(g)
    bd = W.Draws(W.sub_seed(7, W.TAG_BATCH), W.TAG_BATCH)
    batches = []
    for ins, nd in ((pool[:4000], 1000), (pool[4000:4600], 150)):
        dels = shadow.sample_deletions(nd, bd, set())
        shadow.add(ins)
        batches.append(W.make_batch(ins, dels, bd))
    qs = [W.query_from_edges(3, [(0, 1), (1, 2), (0, 2)], (0, 0, 1), "dense"),
          W.query_from_edges(4, [(0, 1), (1, 2), (2, 3), (0, 2)], (1, 0, 0, 2), "sparse")]
    return g, qs, batches


def _same(a, b):
    assert np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.hash_sum, b.hash_sum) and np.array_equal(a.hash_xor, b.hash_xor)
    assert np.array_equal(a.canon_lo, b.canon_lo) and np.array_equal(a.canon_hi, b.canon_hi)
    assert np.array_equal(a.canon_sign, b.canon_sign)
    assert np.array_equal(a.upd_count, b.upd_count)
    assert np.array_equal(a.upd_hash_sum, b.upd_hash_sum) and np.array_equal(a.upd_hash_xor, b.upd_hash_xor)


def test_noalloc_equals_apply_batch_twice_second_smaller():
    g, qs, batches = _graph_and_batches()
    assert len(batches[1]) < len(batches[0])
    cur = g
    with Context(device=0, tuple_capacity=1 << 16) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        for i, b in enumerate(batches):
            print("[noalloc] batch %d: %d updates" % (i, len(b)), flush=True)
            ref = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, canonical=True, dry_run=True)
            got = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, canonical=True, noalloc=True)
            _same(ref, got)
            assert int(got.counts.sum()) > 0
            # the oracle on the same graph state, query by query
            tot = np.zeros_like(got.upd_count)
            for qi, q in enumerate(qs):
                o = O2.run(cur, q, b, qid=qi, threads=4, want_tuples=False)
                assert o.status == 0
                assert np.array_equal(o.canon_lo, got.canon_lo) and np.array_equal(o.canon_hi, got.canon_hi)
                for sign in (0, 1):
                    assert got.count(qi, sign) == o.count[sign]
                    assert int(got.hash_sum[qi, sign]) == o.hsum[sign]
                    assert int(got.hash_xor[qi, sign]) == o.hxor[sign]
                tot += o.seed_count
            assert np.array_equal(got.upd_count, tot)
            rp, col = O2.updated_graph(cur, b)
            cur = W.Graph(cur.n, rp, col, cur.labels)
        rp, col, lab = ctx.export_graph()
        assert np.array_equal(rp, cur.row_ptr) and np.array_equal(col, cur.col)


def test_noalloc_refusals_leave_the_graph_unchanged():
    g, qs, batches = _graph_and_batches()
    with Context(device=0, tuple_capacity=1 << 10) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(qs[0].k, qs[0].labels, qs[0].edges)
        b = batches[0]
        with pytest.raises(GammaError) as e:
            ctx.apply_batch(b.src, b.dst, b.op, tuples=True, noalloc=True)
        assert e.value.status == capi.GAMMA_EUNSUPPORTED
        # 2^20 insertions of absent pairs: far more buffers than the scratch holds
        rng = np.random.Generator(np.random.PCG64(3))
        present = set(g.edge_keys().tolist())
        keys = set()
        while len(keys) < (1 << 20):
            a = rng.integers(0, g.n, 1 << 20, dtype=np.uint64)
            c = rng.integers(0, g.n, 1 << 20, dtype=np.uint64)
            k = (np.minimum(a, c) << np.uint64(32)) | np.maximum(a, c)
            keys.update(int(x) for x in k[a != c].tolist() if int(x) not in present)
        big = np.array(sorted(keys)[: 1 << 20], dtype=np.uint64)
        src = (big >> np.uint64(32)).astype(np.uint32)
        dst = (big & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        with pytest.raises(GammaError) as e:
            ctx.apply_batch(src, dst, np.ones(len(src), np.uint8), noalloc=True)
        assert e.value.status == capi.GAMMA_ENOMEM
        rp, col, lab = ctx.export_graph()
        assert np.array_equal(rp, g.row_ptr) and np.array_equal(col, g.col)
        # and the context still works, through both entry points
        ref = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, canonical=True, dry_run=True)
        got = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, canonical=True, noalloc=True)
        _same(ref, got)
