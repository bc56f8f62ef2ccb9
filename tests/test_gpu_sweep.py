"""GPU: a seeded sweep of small random cases against the oracle.

Each case draws a graph (ER or R-MAT-like skew, 1 to 3 vertex labels, with
or without edge labels), a connected query of 2 to 7 vertices and a batch
(insertions only, deletions only, mixed, with duplicates and no-ops, or
empty), then compares tuple sets, counts, checksums, the canonical batch and
per-update attribution with O2 (tuple sets below 10^6 matches), and the
same batch searched for counts, checksums and attribution only (no tuples:
the lean build of the search kernel on graphs without edge labels).  All
cases run in this one process."""
import numpy as np
import pytest

import workloads as W
from oracle import plain as O2
from test_gpu_parity import make_ctx

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    n = int(rng.integers(20, 400))
    m = int(rng.integers(n, 6 * n))
    L = int(rng.integers(1, 4))
    if rng.random() < 0.5:
        lo, hi = W.er_edges(n, m, seed + 3)
    else:
        scale = max(5, int(np.ceil(np.log2(n))))
        n = 1 << scale
        lo, hi = W.rmat_edges(scale, m, seed + 3)
    rp, col = W.csr_from_edges(n, lo, hi)
    g = W.Graph(n, rp, col, W.labels_uniform(n, L, seed + 5))
    n_el = int(rng.integers(1, 4)) if rng.random() < 0.4 else 1
    if n_el > 1:
        g = W.with_edge_labels(g, n_el, seed + 7)
    # a connected query: a random tree plus a few extra edges
    k = int(rng.integers(2, 8))
    edges = {(int(rng.integers(0, v)), v) for v in range(1, k)}
    for _ in range(int(rng.integers(0, k))):
        a, b = (int(x) for x in rng.integers(0, k, 2))
        if a != b:
            edges.add((min(a, b), max(a, b)))
    edges = sorted(edges)
    q = W.query_from_edges(k, edges, rng.integers(0, L, k).tolist(),
                           elabels=rng.integers(0, n_el, len(edges)).tolist() if n_el > 1 else None)
    # batch
    kind = ["mixed", "insert", "delete", "empty", "noisy"][seed % 5]
    E = g.edge_keys()
    present = set(E.tolist())
    lab = {}
    if n_el > 1:
        src = np.repeat(np.arange(n, dtype=np.uint64), np.diff(g.row_ptr).astype(np.int64))
        keys = (np.minimum(src, g.col) << np.uint64(32)) | np.maximum(src, g.col.astype(np.uint64))
        lab = dict(zip(keys.tolist(), g.elab.tolist()))
    n_del = 0 if kind in ("insert", "empty") else int(rng.integers(1, max(2, len(E) // 4)))
    n_ins = 0 if kind in ("delete", "empty") else int(rng.integers(1, 3 * n))
    ups = [(int(k >> 32), int(k & 0xFFFFFFFF), lab.get(int(k), 0), 0) for k in E[rng.permutation(len(E))[:n_del]]]
    used = {(a, b) for (a, b, _, _) in ups}
    tries = 0
    while len(ups) < n_del + n_ins and tries < 50 * n:
        tries += 1
        a, b = (int(x) for x in rng.integers(0, n, 2))
        key = (min(a, b) << 32) | max(a, b)
        if a == b or key in present or (min(a, b), max(a, b)) in used:
            continue
        used.add((min(a, b), max(a, b)))
        ups.append((a, b, int(rng.integers(0, n_el)), 1))
    if kind == "noisy":
        extra = []
        for (a, b, e, o) in ups[: len(ups) // 3]:
            extra.append((b, a, e, o))  # duplicate, other orientation
        for k in E[rng.permutation(len(E))[: max(1, len(E) // 20)]].tolist():
            if (k >> 32, k & 0xFFFFFFFF) not in used:
                extra.append((k >> 32, k & 0xFFFFFFFF, lab.get(k, 0), 1))  # insertion of a present edge
        ups += extra
    order = rng.permutation(len(ups)) if ups else []
    ups = [ups[i] for i in order]
    b = W.Batch(np.array([u[0] for u in ups], np.uint32), np.array([u[1] for u in ups], np.uint32),
                np.array([u[3] for u in ups], np.uint8),
                np.array([u[2] for u in ups], np.uint32) if n_el > 1 else None)
    return g, q, b


@pytest.mark.parametrize("block", range(4))
def test_random_sweep(block):
    for seed in range(block * 12, block * 12 + 12):
        g, q, b = _case(seed)
        print("[sweep] seed %d: n=%d m=%d L_e=%d k=%d |E(Q)|=%d updates=%d" % (
            seed, g.n, g.m, g.n_elabels, q.k, q.m, len(b)), flush=True)
        with make_ctx(cap=1 << 22) as ctx:
            ctx.load_graph(g.row_ptr, g.col, g.labels, elabels=g.elab, n_elabels=g.n_elabels)
            ctx.register_query(q.k, q.labels, q.edges, elabels=q.elabels)
            # counts, checksums and attribution alone (the lean search build
            # when the graph has no edge labels), as a dry run first
            lean = ctx.apply_batch(b.src, b.dst, b.op, elab=b.elab, per_update=True, dry_run=True)
            res = ctx.apply_batch(b.src, b.dst, b.op, elab=b.elab, tuples=True, seed_attr=True, per_update=True,
                                  canonical=True)
        small = int(res.counts.sum()) < 1_000_000 and not res.truncated
        ref = O2.run(g, q, b, threads=4, want_tuples=small)
        assert ref.status == 0
        for sign in (0, 1):
            assert res.count(0, sign) == ref.count[sign], (seed, sign)
            assert int(res.hash_sum[0, sign]) == ref.hsum[sign] and int(res.hash_xor[0, sign]) == ref.hxor[sign]
            if small:
                assert res.tuple_set(0, sign, q.k) == ref.tuple_set(sign), (seed, sign)
        assert np.array_equal(res.canon_lo, ref.canon_lo) and np.array_equal(res.canon_hi, ref.canon_hi)
        assert np.array_equal(res.upd_count, ref.seed_count) and np.array_equal(res.upd_hash_xor, ref.seed_hxor)
        assert np.array_equal(lean.counts, res.counts), seed
        assert np.array_equal(lean.hash_sum, res.hash_sum) and np.array_equal(lean.hash_xor, res.hash_xor), seed
        assert np.array_equal(lean.upd_count, ref.seed_count) and np.array_equal(lean.upd_hash_sum, ref.seed_hsum)
        assert np.array_equal(lean.upd_hash_xor, ref.seed_hxor), seed
