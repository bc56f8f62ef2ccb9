"""GPU parity at full size for the batched-queries workload: the mid R-MAT
graph (2^20 vertices), 64 standing queries of 4..12 vertices, one batch of
10^4 updates.

The oracle's attribution of every update of the batch for every query is
stored in tests/golden/batched_rmat20_batch0.json (written by
make_batched_golden.py, which runs the oracle only; where the oracle gave a
seed up at its match or work cap it gives a lower bound instead).  Each query then runs on the GPU on
its own (the others paused) under the per-query time limit of Sec. VI-A:
  * a solved query's sampled per-update figures equal the oracle's (above
    the cap where the oracle gave up);
  * an unsolved query (past the limit) is reported as such (open seeds),
    the batch is not committed, and every sampled update whose search work
    all finished still carries the oracle's figures.
Finally the solved queries run together in one launch, and its per-update
attribution over the whole batch equals the sum of their single runs."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from paper_2401_17018_amd import Context, GammaError, capi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LIMIT_MS = 1000  # per-query time limit on this 10^4-update batch


def _golden():
    sys.path.insert(0, GOLDEN)
    import make_batched_golden as MB
    with open(MB.PATH) as fh:
        return MB, json.load(fh)


def _run(ctx, b):
    """(solved, per-update count / sum / xor / open, per-query counts)."""
    try:
        r = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, canonical=True, dry_run=True)
        return True, r.upd_count, r.upd_hash_sum, r.upd_hash_xor, r.upd_open, r
    except GammaError as e:
        assert e.status == capi.GAMMA_ETIMEDOUT
        return False, e.upd_count, e.upd_hash_sum, e.upd_hash_xor, e.upd_open, e


def test_batched_every_query_sampled_against_the_oracle():
    MB, gold = _golden()
    w = W.batched_queries()
    b = w.batches[0]
    assert MB.input_fingerprints(w, b) == gold["inputs"], "inputs changed: rerun tests/golden/make_batched_golden.py"
    nq = len(w.queries)
    print("[batched] n=%d m=%d, %d queries, batch %d updates, limit %d ms per query" % (
        w.graph.n, w.graph.m, nq, len(b), LIMIT_MS), flush=True)
    mod, cap = gold["mod"], gold["cap"]
    compared, queries_compared, solved_ids, total, tot_s = 0, 0, [], None, None
    with Context(device=0) as ctx:
        ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels)
        for q in w.queries:
            ctx.register_query(q.k, q.labels, q.edges)
        for qi in range(nq):
            ctx.set_query_active(qi, False)
        ctx.set_tuning(query_launch=2)
        ctx.set_deadline(LIMIT_MS)
        for qi, q in enumerate(w.queries):
            ctx.set_query_active(qi, True)
            solved, cnt, hs, hx, open_, r = _run(ctx, b)
            ctx.set_query_active(qi, False)
            nc = len(cnt)
            assert nc == gold["n_canonical"]
            op = np.asarray(r.open_seeds)
            assert all(op[j] == 0 for j in range(nq) if j != qi)
            if solved:
                assert op[qi] == 0 and not open_.any()
                assert MB.canonical_fingerprint(r.canon_lo, r.canon_hi, r.canon_sign) == gold["canonical"]
                assert int(cnt.sum()) == int(np.asarray(r.counts)[qi].sum())
                solved_ids.append(qi)
                total = cnt.copy() if total is None else total + cnt
                tot_s = hs.copy() if tot_s is None else tot_s + hs  # uint64: wraps mod 2^64 like the checksum
            else:
                assert op[qi] > 0 and open_.any()
            rec = gold["queries"][qi]
            assert rec["qid"] == qi and rec["k"] == q.k
            idx = np.arange(0, nc, mod)
            want_c = np.zeros(nc, np.uint64)
            want_s = np.zeros(nc, np.uint64)
            want_x = np.zeros(nc, np.uint64)
            for o, c, s_, x_ in rec["nonzero"]:
                want_c[o], want_s[o], want_x[o] = c, int(s_), int(x_)
            over = np.zeros(nc, dtype=bool)
            over[np.asarray(rec["over_cap"], dtype=np.int64)] = True
            found = np.zeros(nc, np.uint64)
            for o, f_ in rec["work_cap"]:
                over[o] = True
                found[o] = f_
            done = np.zeros(nc, dtype=bool)
            done[idx] = open_[idx] == 0
            cmp = done & ~over
            lb = done & over
            assert np.array_equal(cnt[cmp], want_c[cmp]), qi
            assert np.array_equal(hs[cmp], want_s[cmp]) and np.array_equal(hx[cmp], want_x[cmp]), qi
            oc = np.zeros(nc, dtype=bool)
            oc[np.asarray(rec["over_cap"], dtype=np.int64)] = True
            assert np.all(cnt[lb & oc] > cap), qi
            assert np.all(cnt[lb & ~oc] >= found[lb & ~oc]), qi
            if solved:
                assert cmp.sum() + lb.sum() == len(idx)
            m = int(want_c[cmp].sum())
            compared += m
            queries_compared += int(m > 0)
            print("[batched] q%d %s k=%d: %s, %d of %d sampled updates finished, %d oracle matches compared, "
                  "%d above the oracle's cap" % (qi, q.kind, q.k, "solved" if solved else "unsolved",
                                                 int(done[idx].sum()), len(idx), m, int(lb.sum())), flush=True)
        # the solved queries in one launch: per-update sums of their single runs
        for qi in solved_ids:
            ctx.set_query_active(qi, True)
        ctx.set_tuning(query_launch=1)
        ctx.set_deadline(60000)
        r = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, dry_run=True)
    print("[batched] %d solved, %d unsolved; %d oracle matches compared over %d queries" % (
        len(solved_ids), nq - len(solved_ids), compared, queries_compared), flush=True)
    assert compared > 0 and queries_compared >= 8
    assert len(solved_ids) >= nq // 2
    assert np.array_equal(r.upd_count, total)
    assert np.array_equal(r.upd_hash_sum, tot_s)
    assert not r.upd_open.any()
