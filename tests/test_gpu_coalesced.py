"""GPU: coalesced search (Sec. V-B) over automorphisms of the whole query.

Directed query edges that a label-preserving automorphism maps onto each
other are searched once; the matches of the others are produced by
permuting the found ones.  Results must equal the oracle's (which searches
every directed edge) and the library's own with coalescing off, exactly:
tuple sets, counts, checksums and per-update attribution."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from test_gpu_parity import _er, _mixed_batch, _skewed_graph, check_against_o2, make_ctx
from test_gpu_tuning import _same

pytestmark = pytest.mark.gpu

SYMMETRIC = {
    "edge": (2, [(0, 1)], (0, 0)),
    "triangle": (3, [(0, 1), (1, 2), (2, 0)], (0, 0, 0)),
    "path3_sym": (3, [(0, 1), (1, 2)], (1, 0, 1)),
    "star3": (4, [(0, 1), (0, 2), (0, 3)], (0, 1, 1, 1)),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)], (0, 0, 0, 0)),
    "k4": (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], (1, 1, 1, 1)),
    "k5": (5, [(a, b) for a in range(5) for b in range(a + 1, 5)], (0,) * 5),
    "house": (5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)], (0, 0, 0, 0, 1)),
}


def _run(g, qs, b, coalesced, **tuning):
    with make_ctx(cap=1 << 22) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        for q in qs:
            ctx.register_query(q.k, q.labels, q.edges)
        ctx.set_tuning(coalesced_search=2 if coalesced else 1, **tuning)
        return ctx.apply_batch(b.src, b.dst, b.op, tuples=True, seed_attr=True, per_update=True)


@pytest.mark.parametrize("name", sorted(SYMMETRIC))
def test_coalesced_symmetric_queries(name):
    k, edges, labels = SYMMETRIC[name]
    q = W.query_from_edges(k, edges, labels)
    # complete and near-complete shapes need a dense graph to occur at all
    g = _er(120, 3000, 7 + k, 2) if name in ("k4", "k5", "house") else _er(300, 2400, 7 + k, 2)
    b = _mixed_batch(g, 3 + k, 150, 60)
    on = _run(g, [q], b, True)
    off = _run(g, [q], b, False)
    _same(on, off)
    assert on.tuple_set(0, 1, k) == off.tuple_set(0, 1, k) and on.tuple_set(0, 0, k) == off.tuple_set(0, 0, k)
    check_against_o2(on, g, q, b, check_tuples=not on.truncated)
    # the automorphism group acts on the result: its size divides every count
    n_aut = len(CF.automorphisms(q.k, q.labels, q.edges.tolist()))
    assert n_aut > 1
    assert on.count(0, 1) % n_aut == 0 and on.count(0, 0) % n_aut == 0
    assert on.count(0, 1) + on.count(0, 0) > 0


def test_coalesced_many_queries_with_handover():
    """Symmetric and asymmetric queries in one launch on a skewed graph,
    with hand-over forced as often as possible."""
    g = _skewed_graph(5)
    qs = [W.query_from_edges(*SYMMETRIC[n]) for n in ("triangle", "cycle4", "star3")]
    qs.append(W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 1, 0, 1)))
    b = _mixed_batch(g, 9, 300, 100)
    tun = dict(waves_per_cu=4, poll_cycles=500, split_inner=2, split_leaf=2, handover_gate=1024)
    on = _run(g, qs, b, True, **tun)
    off = _run(g, qs, b, False)
    _same(on, off)
    assert on.stats["steals"] > 0
    for qid, q in enumerate(qs):
        check_against_o2(on, g, q, b, qid=qid, check_tuples=not on.truncated)


def test_handover_of_last_level_ranges_keeps_the_driver():
    """Regression: a wave that receives part of a last-level range rebuilds
    that level and must drive it with the donor's list.  With equal list
    lengths the choice once depended on the order the lists were gathered
    in, and K4 on label 0 of the mid graph lost matches with hand-over on."""
    from paper_2401_17018_amd import Context
    w = W.symmetric_queries()
    q, b = w.queries[2], w.batches[0]
    outs = []
    with Context(device=0) as ctx:
        ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        for tun in (dict(steal=2, coalesced_search=1), dict(steal=1, coalesced_search=1),
                    dict(steal=1, coalesced_search=2),
                    dict(steal=1, coalesced_search=1, poll_cycles=500, split_leaf=2, split_inner=2,
                         handover_gate=1024)):
            ctx.set_tuning(**tun)
            outs.append(ctx.apply_batch(b.src, b.dst, b.op, per_update=True, dry_run=True))
    assert outs[0].counts.sum() > 0
    for o in outs[1:]:
        _same(outs[0], o)
    assert outs[3].stats["steals"] > 0
