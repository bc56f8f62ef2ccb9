"""GPU parity at full size, in the launch configuration bench.py times.

Mid: a whole batch runs on the GPU with the library's default tuning (what
bench.py uses), reporting the per-update attribution: for every canonical
batch edge, the count and checksum of the incremental matches whose
minimum-ord batch edge it is.  The oracle computes the same for a
deterministic sample of the batch edges (ord % M == 0) and every sampled
entry must agree exactly.

Large (R-MAT scale 24, 2^29 CSR entries, 10^5 updates): the oracle's
attribution of the whole first batch, for each of the two queries, is
stored in tests/golden/large_rmat24_<kind>_batch0.json (written by
make_large_golden.py, which runs the oracle only).  The oracle gives up a
seed past a per-seed cap, so every update is checked: exactly where the
oracle finished it, as a lower bound (count > cap) where it gave up.  Both
queries run in bench.py's launch configuration; the sparse one (about 3·10^11
incremental matches in this batch) runs a second time under a deadline that
cuts its search short, as an unsolved query would be (Sec. VI-A): every
update whose search work all finished before the deadline (upd_open == 0)
must then carry the oracle's exact figures.

Batch-level identities that hold at any size are checked too: per-update
counts sum to the batch counts, deletions only attribute deletion results
and insertions only insertion results."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import plain as O2
from paper_2401_17018_amd import Context, GammaError, capi
from test_gpu_parity import star_and_edge_check

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,M", [("mid", 2048)])
def test_full_size_sampled_attribution(name, M):
    w = W.mid()
    q = w.queries[0]
    b = w.batches[0]
    print("[fullsize] %s: n=%d m=%d, batch %d updates, query k=%d m=%d" % (name, w.graph.n, w.graph.m, len(b),
                                                                        q.k, q.m), flush=True)
    with Context(device=0) as ctx:
        ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        res = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, canonical=True)
    nc = int(res.stats["n_canonical"])
    # identities at full size
    sign = res.canon_sign.astype(bool)
    assert int(res.upd_count.sum()) == int(res.counts.sum())
    assert int(res.upd_count[sign].sum()) == res.count(0, 1)
    assert int(res.upd_count[~sign].sum()) == res.count(0, 0)
    assert not res.upd_open.any()
    # the oracle on the sample
    ref = O2.run(w.graph, q, b, qid=0, threads=16, sample_mod=M, sample_rem=0, want_tuples=False)
    assert ref.status == 0 and ref.n_canonical == nc
    idx = np.arange(0, nc, M)
    print("[fullsize] %s: %d sampled updates, %d oracle matches in %.1f s" % (
        name, len(idx), int(ref.seed_count[idx].sum()), ref.seconds), flush=True)
    assert int(ref.seed_count[idx].sum()) > 0
    assert np.array_equal(res.upd_count[idx], ref.seed_count[idx])
    assert np.array_equal(res.upd_hash_sum[idx], ref.seed_hsum[idx])
    assert np.array_equal(res.upd_hash_xor[idx], ref.seed_hxor[idx])


@pytest.fixture(scope="module")
def large_workload():
    w = W.large()
    print("[fullsize] large: n=%d m=%d, batch %d updates" % (w.graph.n, w.graph.m, len(w.batches[0])), flush=True)
    return w


def _golden_large(kind):
    import sys
    sys.path.insert(0, GOLDEN)
    import make_large_golden as MG
    with open(MG.path_of(kind)) as fh:
        return MG, json.load(fh)


@pytest.mark.parametrize("kind,deadline_ms", [("dense", 120000), ("sparse", 120000), ("sparse", 300)])
def test_large_every_update_against_the_oracle(large_workload, kind, deadline_ms):
    w = large_workload
    MG, gold = _golden_large(kind)
    qi = [i for i, q in enumerate(w.queries) if q.kind == kind]
    assert len(qi) == 1
    q, b = w.queries[qi[0]], w.batches[0]
    assert MG.input_fingerprints(w, q, b) == gold["inputs"], "inputs changed: rerun tests/golden/make_large_golden.py"
    print("[fullsize] large %s query k=%d m=%d, deadline %d ms" % (kind, q.k, q.m, deadline_ms), flush=True)
    with Context(device=0, deadline_ms=deadline_ms) as ctx:
        ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        try:
            res = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, canonical=True, dry_run=True)
            solved = True
            cnt, hs, hx, open_ = res.upd_count, res.upd_hash_sum, res.upd_hash_xor, res.upd_open
            nc = int(res.stats["n_canonical"])
            assert MG.canonical_fingerprint(res.canon_lo, res.canon_hi, res.canon_sign) == gold["canonical"]
            assert not open_.any()
            assert int(cnt.sum()) == int(res.counts.sum())
        except GammaError as e:
            assert e.status == capi.GAMMA_ETIMEDOUT
            solved = False
            cnt, hs, hx, open_ = e.upd_count, e.upd_hash_sum, e.upd_hash_xor, e.upd_open
            nc = len(cnt)
    assert nc == gold["n_canonical"]
    exact = np.zeros(nc, dtype=bool)
    exact[:] = True
    over = np.array(gold["over_cap"], dtype=np.int64)
    exact[over] = False
    want_c = np.zeros(nc, np.uint64)
    want_s = np.zeros(nc, np.uint64)
    want_x = np.zeros(nc, np.uint64)
    for o, c, hsum, hxor in gold["nonzero"]:
        want_c[o], want_s[o], want_x[o] = c, int(hsum), int(hxor)
    done = open_ == 0
    cmp = done & exact
    print("[fullsize] large %s: %s; %d of %d updates finished, %d compared exactly (%d oracle matches), "
          "%d over the oracle's cap" % (kind, "solved" if solved else "unsolved at the deadline", int(done.sum()), nc,
                                        int(cmp.sum()), int(want_c[cmp].sum()), int((done & ~exact).sum())), flush=True)
    assert int(want_c[cmp].sum()) > 0
    assert np.array_equal(cnt[cmp], want_c[cmp])
    assert np.array_equal(hs[cmp], want_s[cmp]) and np.array_equal(hx[cmp], want_x[cmp])
    # where the oracle gave up at its cap, the finished GPU count is above it
    lb = done & ~exact
    assert np.all(cnt[lb] > gold["cap"])
    if solved:
        assert cmp.sum() + lb.sum() == nc
    else:
        assert deadline_ms < 1000 and open_.any()


def test_star_and_edge_closed_forms_on_large_graph(large_workload):
    """Full-size large R-MAT graph (2^29 CSR entries): star and single-edge
    queries against closed forms."""
    w = large_workload
    res = star_and_edge_check(w.graph, w.batches[0])
    assert res.count(0, 1) > 0


@pytest.mark.parametrize("name,M", [("elabel", 16), ("vertices", 512)])
def test_full_size_sampled_attribution_next4(name, M):
    """The edge-labelled mid workload (7 skewed edge labels) and the mid
    workload with 64 vertex deletions in its batch, at full size with the
    default tuning: per-update attribution of a 1-in-M sample of the
    canonical batch equals the oracle's; batch identities hold."""
    from oracle import vertices as OV
    if name == "elabel":
        w = W.edge_labelled()
        b, vd, ref_batch = w.batches[0], None, w.batches[0]
    else:
        w = W.mid()
        b0 = w.batches[0]
        vd = W.vertex_deletions(w.graph, 64, 1000)
        keep = ~((b0.op == 1) & (np.isin(b0.src, vd) | np.isin(b0.dst, vd)))
        b = W.Batch(b0.src[keep], b0.dst[keep], b0.op[keep])
        status, ref_batch = OV.deletion_batch(w.graph, b, vd)
        assert status == "ok"
    q = w.queries[0]
    print("[fullsize] %s: n=%d m=%d, batch %d updates" % (name, w.graph.n, w.graph.m, len(ref_batch)), flush=True)
    with Context(device=0) as ctx:
        ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels, elabels=w.graph.elab, n_elabels=w.graph.n_elabels)
        ctx.register_query(q.k, q.labels, q.edges, elabels=q.elabels)
        res = ctx.apply_batch(b.src, b.dst, b.op, elab=b.elab, delete_vertices=vd, hash=True, per_update=True,
                              canonical=True)
    nc = int(res.stats["n_canonical"])
    sign = res.canon_sign.astype(bool)
    assert int(res.upd_count.sum()) == int(res.counts.sum())
    assert int(res.upd_count[sign].sum()) == res.count(0, 1)
    assert int(res.upd_count[~sign].sum()) == res.count(0, 0)
    ref = O2.run(w.graph, q, ref_batch, qid=0, threads=16, sample_mod=M, sample_rem=0, want_tuples=False)
    assert ref.status == 0 and ref.n_canonical == nc
    assert np.array_equal(res.canon_lo, ref.canon_lo) and np.array_equal(res.canon_hi, ref.canon_hi)
    idx = np.arange(0, nc, M)
    print("[fullsize] %s: %d sampled updates, %d oracle matches in %.1f s" % (
        name, len(idx), int(ref.seed_count[idx].sum()), ref.seconds), flush=True)
    assert int(ref.seed_count[idx].sum()) > 0
    assert np.array_equal(res.upd_count[idx], ref.seed_count[idx])
    assert np.array_equal(res.upd_hash_sum[idx], ref.seed_hsum[idx])
    assert np.array_equal(res.upd_hash_xor[idx], ref.seed_hxor[idx])


@pytest.mark.parametrize("qi", range(4))
def test_full_size_core_coalescing(qi):
    """The mid graph's first batch with a query whose core is symmetric
    (the core workload's queries), in bench.py's launch configuration:
    coalescing over the core gives the same counts, checksums and
    per-update attribution as coalescing off, and the sampled attribution
    equals the oracle's."""
    w = W.core_symmetric_queries(n_batches=1)
    q = w.queries[qi]
    b = w.batches[0]
    print("[fullsize] core query %d: k=%d m=%d labels=%s" % (qi, q.k, q.m, q.labels.tolist()), flush=True)
    with Context(device=0, deadline_ms=60000) as ctx:
        ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        ctx.set_tuning(coalesced_search=1)
        off = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, canonical=True, dry_run=True)
        ctx.set_tuning(coalesced_search=3)
        on = ctx.apply_batch(b.src, b.dst, b.op, hash=True, per_update=True, canonical=True)
    assert on.stats["n_seeds"] < off.stats["n_seeds"]
    assert np.array_equal(on.counts, off.counts)
    assert np.array_equal(on.hash_sum, off.hash_sum) and np.array_equal(on.hash_xor, off.hash_xor)
    assert np.array_equal(on.upd_count, off.upd_count)
    assert np.array_equal(on.upd_hash_sum, off.upd_hash_sum) and np.array_equal(on.upd_hash_xor, off.upd_hash_xor)
    assert int(on.upd_count.sum()) == int(on.counts.sum()) > 0
    nc = int(on.stats["n_canonical"])
    M = (512, 512, 256, 2048)[qi]  # a sample that holds matches of every query, a few seconds of oracle time
    ref = O2.run(w.graph, q, b, qid=0, threads=16, sample_mod=M, sample_rem=0, want_tuples=False)
    assert ref.status == 0 and ref.n_canonical == nc
    idx = np.arange(0, nc, M)
    print("[fullsize] core query %d: %d sampled updates, %d oracle matches in %.1f s" % (
        qi, len(idx), int(ref.seed_count[idx].sum()), ref.seconds), flush=True)
    assert int(ref.seed_count[idx].sum()) > 0
    assert np.array_equal(on.upd_count[idx], ref.seed_count[idx])
    assert np.array_equal(on.upd_hash_sum[idx], ref.seed_hsum[idx])
    assert np.array_equal(on.upd_hash_xor[idx], ref.seed_hxor[idx])
