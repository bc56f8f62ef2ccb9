"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer set work: every comparison is exact (tuple sets, counts, hashes,
canonical batches, per-update attribution)."""
import glob
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import brute as O1
from oracle import closed_forms as CF
from oracle import plain as O2
from paper_2401_17018_amd import Context, GammaError, capi

pytestmark = pytest.mark.gpu

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "h*.json")))


def make_ctx(cap=1 << 20, **kw):
    return Context(device=0, tuple_capacity=cap, **kw)


def run_gpu(g, queries, b, cap=1 << 20, **kw):
    with make_ctx(cap) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in queries:
            ctx.register_query(q.k, q.labels, q.edges)
        return ctx.apply_batch(b.src, b.dst, b.op, tuples=True, seed_attr=True, per_update=True,
                               canonical=True, **kw)


def check_against_o2(res, g, q, b, qid=0, check_tuples=True):
    ref = O2.run(g, q, b, qid=qid, threads=4)
    assert ref.status == 0
    for sign in (0, 1):
        assert res.count(qid, sign) == ref.count[sign], (sign, res.count(qid, sign), ref.count[sign])
        assert int(res.hash_sum[qid, sign]) == ref.hsum[sign]
        assert int(res.hash_xor[qid, sign]) == ref.hxor[sign]
        if check_tuples:
            assert res.tuple_set(qid, sign, q.k) == ref.tuple_set(sign)
    return ref


def load_fixture(path):
    d = json.load(open(path))
    g = W.graph_from_edges(d["n"], [tuple(e) for e in d["edges"]], d["labels"])
    q = W.query_from_edges(d["k"], [tuple(e) for e in d["qedges"]], d["qlabels"])
    b = W.batch_from_list([tuple(u) for u in d["batch"]])
    return d, g, q, b


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p) for p in GOLDEN])
def test_golden_on_gpu(path):
    d, g, q, b = load_fixture(path)
    res = run_gpu(g, [q], b)
    for sign, key in ((1, "plus"), (0, "minus")):
        exp = {tuple(t) for t in d[key]}
        assert res.tuple_set(0, sign, q.k) == exp
        assert res.count(0, sign) == len(exp)
        rows = np.array(sorted(exp), dtype=np.uint32).reshape(-1, q.k)
        assert CF.multiset_hash(rows, 0, sign) == (len(exp), int(res.hash_sum[0, sign]), int(res.hash_xor[0, sign]))
    if "plus_ord" in d:
        sel = res.meta == 1
        assert set(res.ord[sel].tolist()) == {d["plus_ord"]}


CASES = [(s, 4 + s % 9, 2 + s % 4, 1 + s % 3, bool(s % 2)) for s in range(48)]


@pytest.mark.parametrize("seed,n,k,labels,adv", CASES)
def test_random_small_vs_oracle(seed, n, k, labels, adv):
    g, q, b = W.random_small(1000 + seed, n=n, p=0.5, n_labels=labels, k=k, extra_q_edges=seed % 4,
                             n_ins=4, n_del=3, adversarial=adv)
    res = run_gpu(g, [q], b)
    ref = check_against_o2(res, g, q, b)
    # canonical batch and its order
    assert np.array_equal(res.canon_lo, ref.canon_lo) and np.array_equal(res.canon_hi, ref.canon_hi)
    assert np.array_equal(res.canon_sign, ref.canon_sign)
    assert res.stats["n_noop"] == ref.n_noop and res.stats["n_duplicate"] == ref.n_dup
    # attribution: each tuple's seed ord, and per-update totals
    got = {(s, tuple(int(x) for x in t[:q.k]), int(o)) for t, m, o in zip(res.tuples, res.meta, res.ord)
           for s in [int(m) & 1]}
    exp = {(int(s), tuple(int(x) for x in t), int(o)) for t, s, o in zip(ref.tuples, ref.sign, ref.ord)}
    assert got == exp
    assert np.array_equal(res.upd_count, ref.seed_count)
    assert np.array_equal(res.upd_hash_sum, ref.seed_hsum) and np.array_equal(res.upd_hash_xor, ref.seed_hxor)


def test_brute_force_agrees_on_gpu_cases():
    """A few GPU cases straight against the brute-force set difference (O1)."""
    for seed in range(8):
        g, q, b = W.random_small(77 + seed, n=8, p=0.5, n_labels=2, k=3 + seed % 2, extra_q_edges=1,
                                 n_ins=3, n_del=3, adversarial=True)
        r1 = O1.bdsm(g, q, b)
        res = run_gpu(g, [q], b)
        assert res.tuple_set(0, 1, q.k) == r1["plus"] and res.tuple_set(0, 0, q.k) == r1["minus"]


def _er(n, m, seed, L):
    lo, hi = W.er_edges(n, m, seed)
    rp, col = W.csr_from_edges(n, lo, hi)
    return W.Graph(n, rp, col, W.labels_uniform(n, L, seed + 1))


def _mixed_batch(g, seed, n_ins, n_del):
    rng = np.random.Generator(np.random.PCG64(seed))
    E = g.edge_keys()
    dels = E[rng.permutation(len(E))[:n_del]]
    present = set(E.tolist())
    ins = set()
    while len(ins) < n_ins:
        u, v = (int(x) for x in rng.integers(0, g.n, 2))
        key = (min(u, v) << 32) | max(u, v)
        if u != v and key not in present:
            ins.add(key)
    return W.make_batch(np.array(sorted(ins), np.uint64), dels, W.Draws(seed, 99))


@pytest.mark.parametrize("n_upd", [1, 2, 63, 64, 65, 127, 1000, 4099])
def test_ragged_batch_sizes(n_upd):
    g = _er(2000, 12000, 5, 3)
    q = W.query_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], (0, 1, 0, 2))
    b = _mixed_batch(g, n_upd, n_upd - n_upd // 3, n_upd // 3)
    res = run_gpu(g, [q], b)
    check_against_o2(res, g, q, b)


def test_tiny_config():
    w = W.tiny()
    res = run_gpu(w.graph, w.queries, w.batches[0])
    check_against_o2(res, w.graph, w.queries[0], w.batches[0])


def test_sequence_of_batches_and_export():
    g = _er(500, 3000, 17, 2)
    q = W.query_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)], (0, 1, 0, 1))
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        cur = g
        for t in range(6):
            b = _mixed_batch(cur, 100 + t, 150, 100)
            res = ctx.apply_batch(b.src, b.dst, b.op, tuples=True)
            check_against_o2(res, cur, q, b)
            rp, col = O2.updated_graph(cur, b)
            cur = W.Graph(g.n, rp, col, g.labels)
            erp, ecol, elab = ctx.export_graph()
            assert np.array_equal(erp, rp) and np.array_equal(ecol, col) and np.array_equal(elab, g.labels)


def test_errors_leave_graph_unchanged():
    g = _er(100, 400, 3, 2)
    q = W.query_from_edges(3, [(0, 1), (1, 2)], (0, 0, 1))
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        e0 = g.edge_keys()[0]
        a, c = int(e0 >> 32), int(e0 & 0xFFFFFFFF)
        bad = [
            (W.batch_from_list([("+", 5, 5)]), capi.GAMMA_EINVAL),
            (W.batch_from_list([("+", 5, 1000)]), capi.GAMMA_EINVAL),
            (W.batch_from_list([("-", a, c), ("+", c, a)]), capi.GAMMA_ECONFLICT),
        ]
        for b, st in bad:
            with pytest.raises(GammaError) as ei:
                ctx.apply_batch(b.src, b.dst, b.op)
            assert ei.value.status == st
            rp, col, lab = ctx.export_graph()
            assert np.array_equal(rp, g.row_ptr) and np.array_equal(col, g.col)
        b = _mixed_batch(g, 1, 20, 10)
        res = ctx.apply_batch(b.src, b.dst, b.op, tuples=True)
        check_against_o2(res, g, q, b)


def test_empty_and_noop_batches():
    g = _er(100, 400, 4, 2)
    q = W.query_from_edges(3, [(0, 1), (1, 2)], (0, 0, 1))
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        res = ctx.apply_batch(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint8))
        assert res.counts.sum() == 0 and res.stats["n_canonical"] == 0
        e = g.edge_keys()[:5]
        ups = [("+", int(x >> 32), int(x & 0xFFFFFFFF)) for x in e]  # all present: no-ops
        b = W.batch_from_list(ups + ups)  # and duplicated
        res = ctx.apply_batch(b.src, b.dst, b.op)
        assert res.counts.sum() == 0 and res.stats["n_noop"] == 5 and res.stats["n_duplicate"] == 5
        rp, col, _ = ctx.export_graph()
        assert np.array_equal(col, g.col)


def test_many_queries_one_launch():
    g = _er(800, 6000, 9, 3)
    rng = np.random.Generator(np.random.PCG64(3))
    qs = []
    for i, k in enumerate([2, 3, 4, 5, 6, 4, 3]):
        edges = {(j - 1, j) for j in range(1, k)}
        for _ in range(i % 3):
            a, c = sorted(rng.choice(k, 2, replace=False).tolist())
            edges.add((a, c))
        qs.append(W.query_from_edges(k, sorted(edges), rng.integers(0, 3, k).tolist()))
    b = _mixed_batch(g, 5, 300, 150)
    res = run_gpu(g, qs, b)
    for qid, q in enumerate(qs):
        check_against_o2(res, g, q, b, qid=qid)


def test_truncation_keeps_counts_exact():
    g = _er(300, 3000, 8, 1)
    q = W.query_from_edges(3, [(0, 1), (1, 2)], (0, 0, 0))
    b = _mixed_batch(g, 2, 100, 50)
    with make_ctx(cap=100) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        res = ctx.apply_batch(b.src, b.dst, b.op, tuples=True)
    assert res.truncated and res.n_tuples == 100 and res.n_tuples_found > 100
    check_against_o2(res, g, q, b, check_tuples=False)


def test_labels_wide_and_absent():
    """Large label values, and a query label that no data vertex carries."""
    g = _er(400, 2500, 12, 3)
    g.labels = (g.labels * 20000 + 7).astype(np.uint32)  # 7, 20007, 40007
    q1 = W.query_from_edges(3, [(0, 1), (1, 2), (0, 2)], (7, 20007, 7))
    q2 = W.query_from_edges(3, [(0, 1), (1, 2)], (7, 65000, 7))
    b = _mixed_batch(g, 4, 200, 100)
    res = run_gpu(g, [q1, q2], b)
    check_against_o2(res, g, q1, b, qid=0)
    assert res.counts[1].sum() == 0


def star_and_edge_check(g, b):
    """A star (centre label 0, leaves labels 1 and 2) and a single-edge query
    (labels 0-1) on a full-size graph, against closed forms computed from
    the oracle's canonical batch and updated graph."""
    qs = [W.query_from_edges(3, [(0, 1), (0, 2)], (0, 1, 2)),
          W.query_from_edges(2, [(0, 1)], (0, 1))]
    with make_ctx(cap=0) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        res = ctx.apply_batch(b.src, b.dst, b.op, canonical=True)
    # the oracle's canonical batch (a sampled run does no search work)
    ref = O2.run(g, qs[1], b, qid=1, threads=16, sample_mod=1 << 30, sample_rem=1, want_tuples=False)
    assert ref.status == 0
    assert np.array_equal(res.canon_lo, ref.canon_lo) and np.array_equal(res.canon_hi, ref.canon_hi)
    assert np.array_equal(res.canon_sign, ref.canon_sign)
    ins = [(int(a), int(c)) for a, c, s in zip(ref.canon_lo, ref.canon_hi, ref.canon_sign) if s]
    dels = [(int(a), int(c)) for a, c, s in zip(ref.canon_lo, ref.canon_hi, ref.canon_sign) if not s]
    assert res.count(1, 1) == CF.single_edge_delta(ins, g.labels, 0, 1)
    assert res.count(1, 0) == CF.single_edge_delta(dels, g.labels, 0, 1)
    # star: count centres' neighbour labels before and after
    rp2, col2 = O2.updated_graph(g, b)

    def star_total(rp, col):
        src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp).astype(np.int64))
        lab = g.labels[col]
        cnt1 = np.bincount(src[lab == 1], minlength=g.n).astype(np.int64)
        cnt2 = np.bincount(src[lab == 2], minlength=g.n).astype(np.int64)
        centre = g.labels == 0
        # products stay below 2^63: a centre has fewer than 2^31 neighbours
        return int(np.sum((cnt1 * cnt2)[centre], dtype=np.int64))

    assert res.count(0, 1) - res.count(0, 0) == star_total(rp2, col2) - star_total(g.row_ptr, g.col)
    return res


def test_star_and_edge_closed_forms_on_mid_graph():
    """Full-size mid R-MAT graph: star and single-edge queries against closed forms."""
    w = W.mid()
    star_and_edge_check(w.graph, w.batches[0])


def _skewed_graph(seed):
    """A small R-MAT graph: hubs give long candidate ranges to split."""
    lo, hi = W.rmat_edges(12, 30000, seed)
    rp, col = W.csr_from_edges(1 << 12, lo, hi)
    return W.Graph(1 << 12, rp, col, W.labels_uniform(1 << 12, 2, seed + 1))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_work_handover_on_off_identical(seed):
    """Results do not depend on the hand-over of work between waves."""
    g = _skewed_graph(seed)
    q = W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 1, 0, 1))
    b = _mixed_batch(g, seed, 300, 100)
    outs = []
    for steal in (False, True):
        with make_ctx(cap=1 << 22, steal=steal) as ctx:
            ctx.load_graph(g.row_ptr, g.col, g.labels)
            ctx.register_query(q.k, q.labels, q.edges)
            outs.append(ctx.apply_batch(b.src, b.dst, b.op, tuples=True, per_update=True))
    off, on = outs
    assert np.array_equal(off.counts, on.counts)
    assert np.array_equal(off.hash_sum, on.hash_sum) and np.array_equal(off.hash_xor, on.hash_xor)
    assert np.array_equal(off.upd_count, on.upd_count)
    assert on.stats["steals"] > 0 and off.stats["steals"] == 0
    check_against_o2(on, g, q, b, check_tuples=not on.truncated)


def test_deadline_aborts_and_leaves_graph_unchanged():
    """A search past its deadline stops cooperatively (every wave polls the
    abort word), returns ETIMEDOUT and leaves the graph as before the batch."""
    lo, hi = W.rmat_edges(14, 200000, 9)
    rp, col = W.csr_from_edges(1 << 14, lo, hi)
    g = W.Graph(1 << 14, rp, col, np.zeros(1 << 14, np.uint32))
    q = W.query_from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)], (0,) * 6)
    b = _mixed_batch(g, 3, 2000, 500)
    with make_ctx(cap=0, deadline_ms=1) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        with pytest.raises(GammaError) as ei:
            ctx.apply_batch(b.src, b.dst, b.op)
        assert ei.value.status == capi.GAMMA_ETIMEDOUT
        assert ei.value.stats["seeds_started"] <= ei.value.stats["n_seeds"]
        erp, ecol, _ = ctx.export_graph()
        assert np.array_equal(erp, g.row_ptr) and np.array_equal(ecol, g.col)
        res = ctx.apply_batch(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint8))
        assert res.counts.sum() == 0


def test_per_query_time_limit_reports_unsolved_queries():
    """With one search launch per query the deadline is a time limit per
    query (Sec. VI-A): a query with ~10^11 incremental matches passes it and
    is reported unsolved (open seeds), the light queries before and after it
    finish with the figures they have without a deadline, and the batch is
    not committed.  With one launch for all queries the deadline covers the
    launch, and the light queries' figures are exact where they report no
    open seed."""
    lo, hi = W.rmat_edges(14, 200000, 9)
    rp, col = W.csr_from_edges(1 << 14, lo, hi)
    g = W.Graph(1 << 14, rp, col, np.zeros(1 << 14, np.uint32))
    light = W.query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0,) * 3)
    heavy = W.query_from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)], (0,) * 6)
    k4 = W.query_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2), (1, 3)], (0,) * 4)
    b = _mixed_batch(g, 3, 2000, 500)
    with make_ctx(cap=0) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in (light, heavy, k4):
            ctx.register_query(q.k, q.labels, q.edges)
        ctx.set_query_active(1, False)
        ref = ctx.apply_batch(b.src, b.dst, b.op, hash=True, dry_run=True)
        assert ref.count(1, 1) == 0 and ref.count(1, 0) == 0 and not ref.open_seeds.any()
        assert ref.counts[0].sum() > 0 and ref.counts[2].sum() > 0
        ctx.set_query_active(1, True)
        ctx.set_tuning(query_launch=2)
        ctx.set_deadline(200)  # the light queries (10^5 and 10^7 matches) take a few ms each
        with pytest.raises(GammaError) as ei:
            ctx.apply_batch(b.src, b.dst, b.op, hash=True)
        e = ei.value
        assert e.status == capi.GAMMA_ETIMEDOUT
        assert e.open_seeds[1] > 0 and e.open_seeds[0] == 0 and e.open_seeds[2] == 0
        for qi in (0, 2):
            assert [int(x) for x in e.counts[qi]] == [int(x) for x in ref.counts[qi]]
            assert [int(x) for x in e.hash_sum[qi]] == [int(x) for x in ref.hash_sum[qi]]
            assert [int(x) for x in e.hash_xor[qi]] == [int(x) for x in ref.hash_xor[qi]]
        erp, ecol, _ = ctx.export_graph()
        assert np.array_equal(erp, g.row_ptr) and np.array_equal(ecol, g.col)
        ctx.set_tuning(query_launch=1)
        with pytest.raises(GammaError) as ei:
            ctx.apply_batch(b.src, b.dst, b.op, hash=True)
        e = ei.value
        assert e.open_seeds[1] > 0
        for qi in (0, 2):
            if e.open_seeds[qi] == 0:
                assert [int(x) for x in e.counts[qi]] == [int(x) for x in ref.counts[qi]]
        # without a deadline the light queries' results are unchanged by the heavy one's absence
        ctx.set_query_active(1, False)
        ctx.set_deadline(0)
        res = ctx.apply_batch(b.src, b.dst, b.op, hash=True)
        assert np.array_equal(res.counts, ref.counts) and np.array_equal(res.hash_sum, ref.hash_sum)


@pytest.mark.parametrize("query_launch", [1, 2])
def test_paused_query_is_kept_current(query_launch):
    """A paused query gets no seeds and reports nothing, the other queries'
    results are unchanged, and its candidate table follows every batch: once
    resumed it reports what a context that never paused it reports."""
    g = _er(3000, 24000, 41, 3)
    qa = W.query_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], (0, 1, 0, 2))
    qb = W.query_from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)], (1, 0, 1, 2, 0))
    b1 = _mixed_batch(g, 51, 400, 150)
    rp, col = O2.updated_graph(g, b1)
    g1 = W.Graph(g.n, rp, col, g.labels)
    b2 = _mixed_batch(g1, 52, 400, 150)
    outs = []
    for pause in (False, True):
        with make_ctx(cap=0) as ctx:
            ctx.set_tuning(query_launch=query_launch)
            ctx.load_graph(g.row_ptr, g.col, g.labels)
            ctx.register_query(qa.k, qa.labels, qa.edges)
            ctx.register_query(qb.k, qb.labels, qb.edges)
            if pause:
                ctx.set_query_active(1, False)
            r1 = ctx.apply_batch(b1.src, b1.dst, b1.op, hash=True, per_update=True)
            if pause:
                ctx.set_query_active(1, True)
            r2 = ctx.apply_batch(b2.src, b2.dst, b2.op, hash=True)
            outs.append((r1, r2))
    (n1, n2), (p1, p2) = outs
    assert p1.counts[1].sum() == 0 and p1.hash_sum[1].sum() == 0
    assert np.array_equal(p1.counts[0], n1.counts[0]) and np.array_equal(p1.hash_sum[0], n1.hash_sum[0])
    assert n1.counts[1].sum() > 0 and n2.counts[1].sum() > 0
    assert np.array_equal(p2.counts, n2.counts) and np.array_equal(p2.hash_sum, n2.hash_sum)
    assert np.array_equal(p2.hash_xor, n2.hash_xor)
    ref = O2.run(g1, qb, b2, qid=1, want_tuples=False)
    assert (int(n2.counts[1][0]), int(n2.counts[1][1])) == ref.count
