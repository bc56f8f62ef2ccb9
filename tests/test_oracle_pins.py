"""Pins for the CPU oracle (O1 brute force, O2 plain incremental enumerator).

Each test checks the oracle against something other than itself: hand-worked
examples derived from the definitions (tests/golden), closed forms, the
brute-force set difference, invariants of the problem, and planted mistakes
that the pins must catch.
"""
import glob
import itertools
import json
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import workloads as W
from oracle import brute as O1
from oracle import closed_forms as CF
from oracle import plain as O2

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "h*.json")))


def load_fixture(path):
    d = json.load(open(path))
    g = W.graph_from_edges(d["n"], [tuple(e) for e in d["edges"]], d["labels"])
    q = W.query_from_edges(d["k"], [tuple(e) for e in d["qedges"]], d["qlabels"])
    b = W.batch_from_list([tuple(u) for u in d["batch"]])
    return d, g, q, b


def as_set(rows):
    return {tuple(r) for r in rows}


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p) for p in GOLDEN])
def test_golden_o1(path):
    d, g, q, b = load_fixture(path)
    r = O1.bdsm(g, q, b)
    assert r["status"] == "ok"
    assert r["plus"] == as_set(d["plus"])
    assert r["minus"] == as_set(d["minus"])


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p) for p in GOLDEN])
def test_golden_o2(path):
    d, g, q, b = load_fixture(path)
    r = O2.run(g, q, b)
    assert r.status == 0
    assert r.tuple_set(1) == as_set(d["plus"])
    assert r.tuple_set(0) == as_set(d["minus"])
    # exactly once: no tuple is reported twice
    assert r.count[1] == len(d["plus"]) and r.count[0] == len(d["minus"])
    if "plus_ord" in d:
        assert set(r.ord[r.sign == 1].tolist()) == {d["plus_ord"]}


def test_h3_without_order_rule_duplicates():
    """The order rule is what makes H3 exactly-once: without it the 6 matches come twice."""
    d, g, q, b = load_fixture([p for p in GOLDEN if "h3_" in p][0])
    r = O2.run(g, q, b, mutant=O2.MUT_NO_ORDER_RULE)
    assert r.count[1] == 12 and r.tuple_set(1) == as_set(d["plus"])


# ---------------------------------------------------------------- O2 == O1


def _check_o2_equals_o1(g, q, b, threads=1):
    r1 = O1.bdsm(g, q, b)
    r2 = O2.run(g, q, b, threads=threads)
    if r1["status"] != "ok":
        assert r2.status == {"invalid": -1, "conflict": -2}[r1["status"]]
        return r2
    assert r2.status == 0
    assert r2.tuple_set(1) == r1["plus"]
    assert r2.tuple_set(0) == r1["minus"]
    assert r2.count == (len(r1["minus"]), len(r1["plus"]))  # no duplicates
    I2 = {(int(a), int(c)) for a, c, s in zip(r2.canon_lo, r2.canon_hi, r2.canon_sign) if s == 1}
    D2 = {(int(a), int(c)) for a, c, s in zip(r2.canon_lo, r2.canon_hi, r2.canon_sign) if s == 0}
    assert I2 == set(r1["I"]) and D2 == set(r1["D"])
    assert (r2.n_noop, r2.n_dup) == (r1["n_noop"], r1["n_dup"])
    # canonical order is ascending (lo, hi)
    keys = [(int(a), int(c)) for a, c in zip(r2.canon_lo, r2.canon_hi)]
    assert keys == sorted(keys)
    return r2


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(3, 9), k=st.integers(2, 5),
       extra=st.integers(0, 3), n_labels=st.integers(1, 3), adversarial=st.booleans())
def test_o2_equals_o1_random(seed, n, k, extra, n_labels, adversarial):
    g, q, b = W.random_small(seed, n=n, p=0.45, n_labels=n_labels, k=k, extra_q_edges=extra,
                             n_ins=3, n_del=3, adversarial=adversarial)
    _check_o2_equals_o1(g, q, b)


def test_o2_threads_agree():
    g, q, b = W.random_small(7, n=40, p=0.3, n_labels=2, k=4, extra_q_edges=2, n_ins=30, n_del=20)
    r1 = O2.run(g, q, b, threads=1)
    r8 = O2.run(g, q, b, threads=8)
    assert r1.tuple_set(1) == r8.tuple_set(1) and r1.tuple_set(0) == r8.tuple_set(0)
    assert r1.hsum == r8.hsum and r1.hxor == r8.hxor


@pytest.mark.parametrize("cap", [2, 8, 30, 100])
def test_seed_cap_keeps_completed_seeds_exact(cap):
    """The seed cap (a sampling control for huge results) gives up exactly the
    seeds whose true count exceeds it; every other seed keeps its exact
    count, checksums and tuples, and the totals are those seeds' sums."""
    g, q, b = W.random_small(11, n=40, p=0.3, n_labels=2, k=4, extra_q_edges=1, n_ins=30, n_del=20)
    full = _check_o2_equals_o1(g, q, b)
    for threads in (1, 4):
        r = O2.run(g, q, b, threads=threads, seed_cap=cap)
        assert r.status == 0 and r.n_canonical == full.n_canonical
        over = full.seed_count > cap
        assert over.any() and (~over & (full.seed_count > 0)).any()  # both kinds occur
        assert np.array_equal(r.seed_incomplete.astype(bool), over)
        assert r.n_incomplete == int(over.sum())
        done = ~over
        assert np.array_equal(r.seed_count[done], full.seed_count[done])
        assert np.array_equal(r.seed_hsum[done], full.seed_hsum[done])
        assert np.array_equal(r.seed_hxor[done], full.seed_hxor[done])
        assert np.all(r.seed_count[over] == cap + 1)  # a lower bound of the true count
        for sign in (0, 1):
            sel = done & (full.canon_sign == sign)
            assert r.count[sign] == int(full.seed_count[sel].sum())
            keep = np.isin(full.ord, np.nonzero(sel)[0]) & (full.sign == sign)
            assert r.tuple_set(sign) == {tuple(int(x) for x in t) for t in full.tuples[keep]}
    # no cap (0) and a cap above every seed change nothing
    r = O2.run(g, q, b, seed_cap=int(full.seed_count.max()))
    assert r.n_incomplete == 0 and r.count == full.count and r.hsum == full.hsum and r.hxor == full.hxor
    assert 0 < r.seconds_prep <= r.seconds


@pytest.mark.parametrize("scan_cap", [20, 200])
def test_scan_cap_keeps_completed_seeds_exact(scan_cap):
    """The scan cap gives up a seed whose search examines more than scan_cap
    neighbour-list entries (flag 2); its count is then at most the true count,
    every other seed is exact, and a cap no search reaches changes nothing."""
    g, q, b = W.random_small(11, n=40, p=0.3, n_labels=2, k=4, extra_q_edges=1, n_ins=30, n_del=20)
    full = _check_o2_equals_o1(g, q, b)
    for threads in (1, 4):
        r = O2.run(g, q, b, threads=threads, scan_cap=scan_cap, want_tuples=False)
        inc = r.seed_incomplete
        assert set(np.unique(inc).tolist()) <= {0, 2} and (inc == 2).any() and (inc == 0).any()
        done = inc == 0
        assert np.array_equal(r.seed_count[done], full.seed_count[done])
        assert np.array_equal(r.seed_hsum[done], full.seed_hsum[done])
        assert np.all(r.seed_count[~done] <= full.seed_count[~done])
        for sign in (0, 1):
            sel = done & (full.canon_sign == sign)
            assert r.count[sign] == int(full.seed_count[sel].sum())
    r = O2.run(g, q, b, scan_cap=10 ** 12, want_tuples=False)
    assert r.n_incomplete == 0 and r.count == full.count and r.hsum == full.hsum


# ---------------------------------------------------------------- closed forms


def _er(n, m, seed, L):
    lo, hi = W.er_edges(n, m, seed)
    rp, col = W.csr_from_edges(n, lo, hi)
    return W.Graph(n, rp, col, W.labels_uniform(n, L, seed + 1))


def _random_batch(g, seed, n_ins, n_del):
    rng = np.random.Generator(np.random.PCG64(seed))
    E = O1.edge_set(g)
    present = sorted(E)
    dels = [present[i] for i in rng.permutation(len(present))[:n_del]]
    ins = set()
    while len(ins) < n_ins:
        u, v = (int(x) for x in rng.integers(0, g.n, 2))
        if u != v and (min(u, v), max(u, v)) not in E:
            ins.add((min(u, v), max(u, v)))
    ups = [("+",) + e for e in sorted(ins)] + [("-",) + e for e in dels]
    return W.batch_from_list(ups), E, set(ins), set(dels)


@pytest.mark.parametrize("leaves", [(1, 1), (1, 2, 2), (0, 1, 1, 2)])
def test_star_closed_form(leaves):
    g = _er(300, 1500, 11, 3)
    k = 1 + len(leaves)
    q = W.query_from_edges(k, [(0, i) for i in range(1, k)], (0,) + leaves)
    b, E, I, D = _random_batch(g, 5, 40, 25)
    r = O2.run(g, q, b, want_tuples=False)
    E2 = (E | I) - D
    before = CF.star_matches(O1.adjacency(g.n, E), g.labels, 0, leaves)
    after = CF.star_matches(O1.adjacency(g.n, E2), g.labels, 0, leaves)
    assert r.count[1] - r.count[0] == after - before
    # insert-only batch: the + count is the whole difference
    b2 = W.batch_from_list([("+",) + e for e in sorted(I)])
    r2 = O2.run(g, q, b2, want_tuples=False)
    assert r2.count[0] == 0
    assert r2.count[1] == CF.star_matches(O1.adjacency(g.n, E | I), g.labels, 0, leaves) - before


def test_single_edge_closed_form():
    g = _er(200, 800, 3, 2)
    b, E, I, D = _random_batch(g, 9, 50, 50)
    for lx, ly in [(0, 0), (0, 1), (1, 0)]:
        q = W.query_from_edges(2, [(0, 1)], (lx, ly))
        r = O2.run(g, q, b, want_tuples=False)
        assert r.count[1] == CF.single_edge_delta(I, g.labels, lx, ly)
        assert r.count[0] == CF.single_edge_delta(D, g.labels, lx, ly)


def test_equal_label_triangle_closed_form():
    g = _er(150, 1200, 21, 2)
    q = W.query_from_edges(3, [(0, 1), (1, 2), (0, 2)], (1, 1, 1))
    b, E, I, D = _random_batch(g, 4, 60, 60)
    r = O2.run(g, q, b, want_tuples=False)
    E2 = (E | I) - D
    t0 = CF.triangles(O1.adjacency(g.n, E), label=1, labels=g.labels)
    t1 = CF.triangles(O1.adjacency(g.n, E2), label=1, labels=g.labels)
    assert r.count[1] - r.count[0] == 6 * (t1 - t0)


def test_triangle_count_textbook():
    """The node iterator itself, on graphs with known triangle counts."""
    k5 = {(a, b) for a in range(5) for b in range(a + 1, 5)}
    assert CF.triangles(O1.adjacency(5, k5)) == 10
    c4 = {(0, 1), (1, 2), (2, 3), (0, 3)}
    assert CF.triangles(O1.adjacency(4, c4)) == 0


@pytest.mark.parametrize("name,k,edges,labels,order", [
    # group orders known in closed form: S_3, S_4, S_3 on the leaves, the
    # dihedral groups D_4 and D_5, S_2 x S_3 on the two sides of K_{2,3},
    # the reflection of a path
    ("triangle", 3, [(0, 1), (1, 2), (0, 2)], (0, 0, 0), 6),
    ("K4", 4, [(a, b) for a in range(4) for b in range(a + 1, 4)], (0, 0, 0, 0), 24),
    ("star3", 4, [(0, 1), (0, 2), (0, 3)], (0, 1, 1, 1), 6),
    ("C4", 4, [(0, 1), (1, 2), (2, 3), (0, 3)], (0, 0, 0, 0), 8),
    ("C5", 5, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4)], (0,) * 5, 10),
    ("K23", 5, [(a, b) for a in (0, 1) for b in (2, 3, 4)], (0,) * 5, 12),
    ("P3", 3, [(0, 1), (1, 2)], (0, 0, 0), 2),
    # labels cut the group down: a 4-cycle labelled 0,0,1,1 keeps only the
    # reflection through the midpoints of its two one-label edges; a path
    # with different end labels keeps only the identity; a K4 with labels
    # 0,0,0,1 keeps S_3 on the three equal vertices
    ("C4_labelled", 4, [(0, 1), (1, 2), (2, 3), (0, 3)], (0, 0, 1, 1), 2),
    ("P3_ends", 3, [(0, 1), (1, 2)], (0, 1, 2), 1),
    ("K4_one_odd", 4, [(a, b) for a in range(4) for b in range(a + 1, 4)], (0, 0, 0, 1), 6),
])
def test_automorphism_counts_exact(name, k, edges, labels, order):
    """|Aut_L(Q)| against group orders known in closed form (the closure
    invariant and coalesced search rely on this enumeration)."""
    aut = CF.automorphisms(k, labels, edges)
    assert len(aut) == order, name
    assert len(set(aut)) == order and tuple(range(k)) in aut
    # a group: closed under composition
    s = set(aut)
    for p in aut:
        for r in aut:
            assert tuple(p[r[i]] for i in range(k)) in s


# ---------------------------------------------------------------- invariants


def _check_invariants(g, q, b, r, qid=0):
    E = O1.edge_set(g)
    I = {(int(a), int(c)) for a, c, s in zip(r.canon_lo, r.canon_hi, r.canon_sign) if s == 1}
    D = {(int(a), int(c)) for a, c, s in zip(r.canon_lo, r.canon_hi, r.canon_sign) if s == 0}
    E2 = (E | I) - D
    qe = [tuple(e) for e in q.edges.tolist()]
    aut = CF.automorphisms(q.k, q.labels, qe)
    for sign, H, S in [(1, E2, I), (0, E, D)]:
        res = r.tuple_set(sign)
        has = lambda u, v, H=H: (min(u, v), max(u, v)) in H
        for f in res:
            assert CF.validate_tuple(f, g.labels, q.labels, qe, has, S)
            for p in aut:  # closed under label-preserving automorphisms
                assert tuple(f[p[i]] for i in range(q.k)) in res
        assert len(res) % len(aut) == 0
        tup = r.tuples[r.sign == sign]
        assert CF.multiset_hash(tup, qid, sign) == (r.count[sign], r.hsum[sign], r.hxor[sign])


@pytest.mark.parametrize("seed", range(6))
def test_invariants_mid(seed):
    g = _er(400, 3000, 100 + seed, 2)
    qk = 3 + seed % 3
    rng = np.random.Generator(np.random.PCG64(seed))
    qe = [(i - 1, i) for i in range(1, qk)] + [(0, qk - 1)]
    q = W.query_from_edges(qk, qe, rng.integers(0, 2, qk).tolist())
    b, *_ = _random_batch(g, seed, 80, 40)
    r = O2.run(g, q, b, qid=seed, threads=4)
    _check_invariants(g, q, b, r, qid=seed)


def test_order_invariance_and_inverse():
    g = _er(300, 2400, 8, 2)
    q = W.query_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], (0, 0, 1, 0))
    b, E, I, D = _random_batch(g, 2, 60, 40)
    r = O2.run(g, q, b)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(len(b))
    sh = W.Batch(b.dst[perm].copy(), b.src[perm].copy(), b.op[perm].copy())  # reordered and reversed
    r2 = O2.run(g, q, sh)
    assert r.tuple_set(1) == r2.tuple_set(1) and r.tuple_set(0) == r2.tuple_set(0)
    rp, col = O2.updated_graph(g, b)
    g2 = W.Graph(g.n, rp, col, g.labels)
    rinv = O2.run(g2, q, b.inverse())
    assert rinv.tuple_set(1) == r.tuple_set(0) and rinv.tuple_set(0) == r.tuple_set(1)


def test_telescoping_stream():
    g = _er(250, 1200, 31, 2)
    leaves = (1, 1)
    q = W.query_from_edges(3, [(0, 1), (0, 2)], (0,) + leaves)
    start = CF.star_matches(O1.adjacency(g.n, O1.edge_set(g)), g.labels, 0, leaves)
    net = 0
    cur = g
    for t in range(4):
        b, *_ = _random_batch(cur, 50 + t, 30, 30)
        r = O2.run(cur, q, b, want_tuples=False)
        net += r.count[1] - r.count[0]
        rp, col = O2.updated_graph(cur, b)
        cur = W.Graph(g.n, rp, col, g.labels)
    end = CF.star_matches(O1.adjacency(g.n, O1.edge_set(cur)), g.labels, 0, leaves)
    assert net == end - start


def test_canonical_errors():
    g = W.graph_from_edges(4, [(0, 1), (1, 2)], [0, 0, 0, 0])
    q = W.query_from_edges(2, [(0, 1)], (0, 0))
    assert O2.run(g, q, W.batch_from_list([("+", 2, 2)])).status == -1  # self loop
    assert O2.run(g, q, W.batch_from_list([("+", 0, 9)])).status == -1  # id out of range
    assert O2.run(g, q, W.batch_from_list([("+", 0, 3), ("-", 3, 0)])).status == -2  # conflict
    r = O2.run(g, q, W.batch_from_list([("+", 0, 1), ("-", 0, 3), ("+", 2, 3), ("+", 3, 2)]))
    assert r.status == 0 and r.n_noop == 2 and r.n_dup == 1 and r.n_canonical == 1
    assert r.count == (0, 2)
    r = O2.run(g, q, W.batch_from_list([]))
    assert r.status == 0 and r.n_canonical == 0 and r.count == (0, 0)


def test_planted_match_in_mid_config():
    """The query extracted from the mid R-MAT workload maps onto its walk, which
    uses an inserted edge of the batch: that tuple satisfies every condition
    of an insertion result (checked by the per-tuple validator, not by O2)."""
    w = W.mid()
    q = w.queries[0]
    g, b = w.graph, w.batches[0]
    assert q.planted is not None and len(set(q.planted)) == q.k
    ins = {(min(int(s), int(d)), max(int(s), int(d))) for s, d, o in zip(b.src, b.dst, b.op) if o == 1}
    dels = {(min(int(s), int(d)), max(int(s), int(d))) for s, d, o in zip(b.src, b.dst, b.op) if o == 0}

    def has(u, v):
        e = (min(u, v), max(u, v))
        return (g.has_edge(u, v) or e in ins) and e not in dels

    qe = [tuple(e) for e in q.edges.tolist()]
    assert CF.validate_tuple(q.planted, g.labels, q.labels, qe, has, ins)


# ---------------------------------------------------------------- planted mistakes


def _pins_pass(mutant):
    """Run a compact set of pins against O2 with a planted mistake; True if all pass."""
    try:
        for path in GOLDEN:
            d, g, q, b = load_fixture(path)
            r = O2.run(g, q, b, mutant=mutant)
            if r.status != 0 or r.tuple_set(1) != as_set(d["plus"]) or r.tuple_set(0) != as_set(d["minus"]):
                return False
            if r.count != (len(d["minus"]), len(d["plus"])):
                return False
        for seed in range(40):
            g, q, b = W.random_small(seed, n=7, p=0.5, n_labels=2, k=3 + seed % 2, extra_q_edges=1,
                                     n_ins=3, n_del=3, adversarial=True)
            r1 = O1.bdsm(g, q, b)
            r2 = O2.run(g, q, b, mutant=mutant)
            if r1["status"] != "ok":
                continue
            if r2.tuple_set(1) != r1["plus"] or r2.tuple_set(0) != r1["minus"]:
                return False
            if r2.count != (len(r1["minus"]), len(r1["plus"])):
                return False
        return True
    except Exception:
        return False


def test_correct_oracle_passes_compact_pins():
    assert _pins_pass(O2.MUT_NONE)


@pytest.mark.parametrize("mutant", [O2.MUT_NO_INJECTIVITY, O2.MUT_ONE_ORIENTATION, O2.MUT_NO_ORDER_RULE,
                                    O2.MUT_DELETE_ON_GPRIME, O2.MUT_SKIP_FIRST_CHECK, O2.MUT_NO_LABEL_CHECK,
                                    O2.MUT_KEEP_NOOPS])
def test_planted_mistake_is_caught(mutant):
    assert not _pins_pass(mutant)


def test_ord_list_sample_keeps_full_batch_figures():
    """The ord-list sample (a sampling control) searches only the listed
    canonical updates, each with exactly its figures of the full run (the
    whole batch stays visible to the order rule)."""
    g, q, b = W.random_small(17, n=40, p=0.3, n_labels=2, k=4, extra_q_edges=1, n_ins=30, n_del=20)
    full = _check_o2_equals_o1(g, q, b)
    pick = np.nonzero(full.seed_count > 0)[0][::2]
    assert len(pick) >= 2
    for threads in (1, 4):
        r = O2.run(g, q, b, threads=threads, ords=pick.tolist())
        assert r.status == 0 and r.n_canonical == full.n_canonical
        sel = np.zeros(full.n_canonical, bool)
        sel[pick] = True
        assert np.array_equal(r.seed_count[sel], full.seed_count[sel]) and not r.seed_count[~sel].any()
        assert np.array_equal(r.seed_hsum[sel], full.seed_hsum[sel])
        assert np.array_equal(r.seed_hxor[sel], full.seed_hxor[sel])
        for sign in (0, 1):
            keep = np.isin(full.ord, pick) & (full.sign == sign)
            assert r.tuple_set(sign) == {tuple(int(x) for x in t) for t in full.tuples[keep]}
    # ords past the batch are ignored; an empty list searches nothing
    r = O2.run(g, q, b, ords=[full.n_canonical + 5])
    assert tuple(r.count) == (0, 0)


def test_checksum_definition_and_copies_agree():
    """The project's tuple checksum (not part of the method): the C oracle's
    and the Python copies agree with a direct evaluation of the definition,
    and it separates tuples that differ by a swap of positions or by a
    balanced change of two elements."""
    rng = np.random.Generator(np.random.PCG64(5))
    M = (1 << 64) - 1

    def direct(q, s, f):
        z = CF._mix_py((q << 1) | s)
        for j, v in enumerate(f):
            z = (z + (int(v) + 1) * (CF._mix_py((0x9E3779B97F4A7C15 * (j + 1)) & M) | 1)) & M
        return CF._mix_py(z)

    for _ in range(50):
        k = int(rng.integers(2, 17))
        f = [int(x) for x in rng.integers(0, 1 << 31, k)]
        q, s = int(rng.integers(0, 64)), int(rng.integers(0, 2))
        assert O2.tuple_hash(q, s, f) == CF.tuple_hash(q, s, f) == direct(q, s, f)
    t = rng.integers(0, 1 << 24, (200, 6)).astype(np.uint32)
    cnt, hs, hx = CF.multiset_hash(t, 3, 1)
    hh = [CF.tuple_hash(3, 1, row) for row in t.tolist()]
    assert cnt == 200 and hs == sum(hh) % (1 << 64)
    x = 0
    for h in hh:
        x ^= h
    assert hx == x
    assert CF.tuple_hash(0, 1, [1, 2, 3]) != CF.tuple_hash(0, 1, [2, 1, 3])
    assert CF.tuple_hash(0, 1, [10, 20]) != CF.tuple_hash(0, 1, [13, 17])
    assert CF.tuple_hash(0, 1, [5, 6]) != CF.tuple_hash(0, 0, [5, 6])
