"""GPU: dry runs, per-query search launches, search tunables and the
autotuner.  None of them may change a result, so every comparison is exact
(counts, multiset hashes, per-update attribution, tuple sets against the
oracle)."""
import json

import numpy as np
import pytest

import workloads as W
from oracle import plain as O2
from paper_2401_17018_amd import GammaError, capi
from test_gpu_parity import _er, _mixed_batch, _skewed_graph, check_against_o2, make_ctx

pytestmark = pytest.mark.gpu


def _queries(seed, ks, n_labels=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    qs = []
    for i, k in enumerate(ks):
        edges = {(j - 1, j) for j in range(1, k)}
        for _ in range(i % 3):
            a, c = sorted(rng.choice(k, 2, replace=False).tolist())
            edges.add((a, c))
        qs.append(W.query_from_edges(k, sorted(edges), rng.integers(0, n_labels, k).tolist()))
    return qs


def _same(a, b):
    assert np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.hash_sum, b.hash_sum) and np.array_equal(a.hash_xor, b.hash_xor)
    if a.upd_count is not None or b.upd_count is not None:
        assert np.array_equal(a.upd_count, b.upd_count)
        assert np.array_equal(a.upd_hash_sum, b.upd_hash_sum)


def test_dry_run_matches_apply_and_keeps_graph():
    """A dry run reports what the batch would do and leaves the graph as it
    was, also when repeated until the arena has to be compacted."""
    g = _er(1500, 9000, 21, 3)
    qs = _queries(4, [3, 4, 5])
    b = _mixed_batch(g, 8, 400, 200)
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        dry = [ctx.apply_batch(b.src, b.dst, b.op, per_update=True, dry_run=True) for _ in range(12)]
        erp, ecol, elab = ctx.export_graph()
        assert np.array_equal(erp, g.row_ptr) and np.array_equal(ecol, g.col)
        for d in dry[1:]:
            _same(dry[0], d)
        real = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, tuples=True)
        _same(dry[0], real)
        erp2, ecol2, _ = ctx.export_graph()
        assert not np.array_equal(ecol2, g.col)
    for qid, q in enumerate(qs):
        check_against_o2(real, g, q, b, qid=qid)


def test_per_query_launches_identical():
    """One search launch per query gives what one launch for all gives."""
    g = _er(800, 6000, 9, 3)
    qs = _queries(3, [2, 3, 4, 5, 6, 4, 3])
    b = _mixed_batch(g, 5, 300, 150)
    outs = []
    for mode in (1, 2):
        with make_ctx() as ctx:
            ctx.load_graph(g.row_ptr, g.col, g.labels)
            for q in qs:
                ctx.register_query(q.k, q.labels, q.edges)
            assert ctx.set_tuning(query_launch=mode)["query_launch"] == mode
            outs.append(ctx.apply_batch(b.src, b.dst, b.op, per_update=True, tuples=True))
    _same(outs[0], outs[1])
    for qid, q in enumerate(qs):
        check_against_o2(outs[1], g, q, b, qid=qid)


TUNINGS = [
    dict(waves_per_cu=4, steal=1, poll_cycles=500, split_inner=2, split_leaf=2, handover_gate=1024),  # hand over almost anything
    dict(waves_per_cu=8, steal=1, group_seeds=2),  # seeds sorted by their first data vertex
    dict(waves_per_cu=8, steal=1, group_seeds=3),  # grouped by (query, edge, a), shared level-2 lists
    dict(waves_per_cu=4, steal=1, poll_cycles=500, split_inner=2, split_leaf=2, handover_gate=1024,
         group_seeds=3),  # ... with level-2 ranges of group lists handed over
    dict(waves_per_cu=32, steal=1, poll_cycles=1000000, split_inner=1 << 20, split_leaf=1 << 20),
    dict(waves_per_cu=12, steal=2),
    dict(waves_per_cu=1, steal=1, poll_cycles=3000, handover_gate=1),
    dict(waves_per_cu=8, steal=1, shared_leaf=1),  # every survivor walks its own last level, sets up every level
    dict(waves_per_cu=8, steal=1, shared_leaf=3),  # shared last level, every inner level set up anew
]


@pytest.mark.parametrize("seed", [1, 2])
def test_tunables_do_not_change_results(seed):
    g = _skewed_graph(seed)
    q = W.query_from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 1)], (0, 1, 0, 1, 0))
    b = _mixed_batch(g, seed, 300, 100)
    outs = []
    with make_ctx(cap=1 << 22) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        for t in TUNINGS:
            got = ctx.set_tuning(**t)
            assert all(got[k] == v for k, v in t.items())
            outs.append(ctx.apply_batch(b.src, b.dst, b.op, per_update=True, tuples=True, dry_run=True))
    for o in outs[1:]:
        _same(outs[0], o)
    assert outs[0].stats["steals"] > 0 and outs[5].stats["steals"] == 0
    assert 0 < outs[2].stats["n_groups"] < outs[2].stats["n_seeds"]
    check_against_o2(outs[0], g, q, b, check_tuples=not outs[0].truncated)


def test_set_tuning_rejects_out_of_range():
    with make_ctx(cap=0) as ctx:
        before = ctx.get_tuning()
        for bad in (dict(split_inner=1), dict(waves_per_cu=33), dict(steal=3), dict(query_launch=7),
                    dict(poll_cycles=10), dict(handover_gate=2000), dict(group_seeds=4),
                    dict(shared_leaf=4)):
            with pytest.raises(GammaError) as ei:
                ctx.set_tuning(**bad)
            assert ei.value.status == capi.GAMMA_EINVAL
            assert ctx.get_tuning() == before


def test_autotune_keeps_graph_and_caches(tmp_path):
    g = _skewed_graph(4)
    qs = [W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 1, 0, 1)),
          W.query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 1))]
    calib = _mixed_batch(g, 11, 200, 50)
    b = _mixed_batch(g, 12, 300, 100)
    cache = str(tmp_path / "tune.json")
    with make_ctx() as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        r1 = ctx.autotune(calib.src, calib.dst, calib.op, max_points=6, reps=1, cache=cache)
        assert not r1["from_cache"] and r1["best_ms"] > 0 and r1["best_ms"] <= r1["base_ms"]
        assert ctx.get_tuning() == r1["tuning"]
        erp, ecol, _ = ctx.export_graph()
        assert np.array_equal(erp, g.row_ptr) and np.array_equal(ecol, g.col)
        r2 = ctx.autotune(calib.src, calib.dst, calib.op, cache=cache)
        assert r2["from_cache"] and r2["tuning"] == r1["tuning"]
        assert r1["key"] in json.load(open(cache))
        res = ctx.apply_batch(b.src, b.dst, b.op, tuples=True)
    for qid, q in enumerate(qs):
        check_against_o2(res, g, q, b, qid=qid)


def test_deadline_with_per_query_launches():
    """The deadline spans all of a batch's search launches; the batch is
    rolled back."""
    lo, hi = W.rmat_edges(14, 200000, 9)
    rp, col = W.csr_from_edges(1 << 14, lo, hi)
    g = W.Graph(1 << 14, rp, col, np.zeros(1 << 14, np.uint32))
    q = W.query_from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)], (0,) * 6)
    b = _mixed_batch(g, 3, 2000, 500)
    with make_ctx(cap=0, deadline_ms=1) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        ctx.register_query(q.k, q.labels, q.edges)
        ctx.set_tuning(query_launch=2)
        with pytest.raises(GammaError) as ei:
            ctx.apply_batch(b.src, b.dst, b.op)
        assert ei.value.status == capi.GAMMA_ETIMEDOUT
        erp, ecol, _ = ctx.export_graph()
        assert np.array_equal(erp, g.row_ptr) and np.array_equal(ecol, g.col)


def _hub_batch(g, hubs, per_hub, seed):
    """Insertions of absent edges at a few hub vertices (many seeds share a
    first data vertex), plus deletions at the same hubs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    E = set(g.edge_keys().tolist())
    ups = []
    for h in hubs:
        others = rng.permutation(g.n)
        n_ins = 0
        for v in others.tolist():
            if v == h:
                continue
            key = (min(h, v) << 32) | max(h, v)
            if key not in E and n_ins < per_hub:
                ups.append(("+", h, v))
                n_ins += 1
        row = g.neighbors(h)[: per_hub // 3]
        ups += [("-", h, int(v)) for v in row.tolist()]
    keys = set()
    out = []
    for op, a, b in ups:
        k = (min(a, b), max(a, b))
        if k not in keys:
            keys.add(k)
            out.append((op, a, b))
    return W.batch_from_list(out)


@pytest.mark.parametrize("qname", ["triangle", "path", "diamond"])
def test_update_edge_grouping_shares_level_two(qname):
    """Grouping by (query, directed query edge, a) with level 2's list built
    once per group (group_seeds = 3): batches whose updates share hub
    endpoints form groups; counts, checksums, per-update attribution and
    tuples equal the ungrouped search and the oracle, in the lean build
    (attribution only) and the full one (tuples), with hand-over forced."""
    g = _skewed_graph(7)
    deg = np.diff(g.row_ptr.astype(np.int64))
    hubs = np.argsort(-deg)[:4].tolist()
    b = _hub_batch(g, hubs, 60, 3)
    q = {"triangle": W.query_from_edges(3, [(0, 1), (1, 2), (0, 2)], (0, 0, 0)),
         "path": W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 0, 0, 0)),
         "diamond": W.query_from_edges(4, [(0, 1), (1, 2), (2, 3), (0, 3), (0, 2)], (0, 0, 0, 0))}[qname]
    with make_ctx(cap=1 << 22) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        res = {}
        for name, t in [("plain", dict(group_seeds=1)), ("grouped", dict(group_seeds=3)),
                        ("grouped_handover", dict(group_seeds=3, poll_cycles=500, split_inner=2, split_leaf=2,
                                                  handover_gate=1024, waves_per_cu=4))]:
            ctx.set_tuning(**t)
            lean = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, dry_run=True)
            full = ctx.apply_batch(b.src, b.dst, b.op, per_update=True, tuples=True, dry_run=True)
            res[name] = (lean, full)
    plain_lean, plain_full = res["plain"]
    for name in ("grouped", "grouped_handover"):
        lean, full = res[name]
        assert 0 < lean.stats["n_groups"] < lean.stats["n_seeds"], lean.stats
        _same(plain_lean, lean)
        _same(plain_full, full)
    assert int(plain_lean.counts.sum()) > 0
    check_against_o2(res["grouped_handover"][1], g, q, b, check_tuples=not res["grouped_handover"][1].truncated)


SHARED_QUERIES = {
    "star4": (4, [(0, 1), (0, 2), (0, 3)], (0, 1, 1, 0)),
    "star5_equal": (5, [(0, 1), (0, 2), (0, 3), (0, 4)], (0, 0, 0, 0, 0)),  # the survivor itself is a candidate
    "tree_cycle6": (6, [(0, 1), (1, 2), (2, 0), (2, 3), (1, 4), (0, 5)], (0, 1, 0, 1, 0, 1)),
    "two_static_lists": (5, [(0, 1), (1, 2), (0, 3), (1, 3), (2, 4)], (0, 1, 0, 1, 1)),
    # static inner levels; on the uniform-degree graph below (hub rows would
    # give a 7-vertex tree ~10^13 matches per batch)
    "tree7": (7, [(0, 1), (0, 2), (1, 3), (1, 4), (2, 5), (2, 6)], (0, 1, 2, 0, 1, 2, 0)),
}


@pytest.mark.parametrize("qname", list(SHARED_QUERIES))
def test_shared_last_level_identical(qname):
    """A last level whose lists all come from vertices matched before
    order[k-2] is walked once per level-(k-2) chunk and paired with every
    survivor (shared_leaf = 3), and inner levels whose lists do not come
    from the vertex matched before them keep their set-up between that
    vertex's candidates (shared_leaf = 2).  Counts, checksums and per-update
    attribution equal the plain descent (shared_leaf = 1) and the oracle,
    with and without forced hand-over; so do the candidates and nodes."""
    from paper_2401_17018_amd import describe_query
    k, edges, labels = SHARED_QUERIES[qname]
    q = W.query_from_edges(k, edges, labels)
    adj = {(a, c) for a, c in edges} | {(c, a) for a, c in edges}
    plans, _ = describe_query(q.k, q.labels, q.edges)
    assert any((p["order"][k - 1], p["order"][k - 2]) not in adj for p in plans)
    g = _er(3000, 15000, 5, 3) if qname == "tree7" else _skewed_graph(5)
    b = _mixed_batch(g, 8, 300, 100)
    res = {}
    with make_ctx(cap=0, deadline_ms=60000) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        for name, t in [("off", dict(shared_leaf=1)), ("leaf", dict(shared_leaf=3)), ("on", dict(shared_leaf=2)),
                        ("on_handover", dict(shared_leaf=2, poll_cycles=500, split_inner=2, split_leaf=2,
                                             handover_gate=1024, waves_per_cu=4))]:
            ctx.set_tuning(coalesced_search=1, **t)
            res[name] = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, dry_run=True)
    off = res["off"]
    for name in ("leaf", "on", "on_handover"):
        _same(off, res[name])
        assert np.array_equal(off.upd_hash_xor, res[name].upd_hash_xor)
        assert res[name].stats["cand_scanned"] == off.stats["cand_scanned"]
        assert res[name].stats["dfs_nodes"] == off.stats["dfs_nodes"]
    assert int(off.counts.sum()) > 0
    ref = O2.run(g, q, b, qid=0, want_tuples=False)
    assert (int(off.counts[0, 0]), int(off.counts[0, 1])) == ref.count
    assert (int(res["on"].hash_sum[0, 0]), int(res["on"].hash_sum[0, 1])) == ref.hsum
    assert (int(res["on"].hash_xor[0, 0]), int(res["on"].hash_xor[0, 1])) == ref.hxor
    assert np.array_equal(res["on"].upd_count, ref.seed_count)
    assert np.array_equal(res["on"].upd_hash_sum, ref.seed_hsum)
