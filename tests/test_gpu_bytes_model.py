"""GPU: the search kernel's algorithmic byte count against an independent
count of the same model.

The kernel reports `bytes_alg_dfs`, the bytes a fixed model says the
search must read (per candidate examined: a 4-byte id, a 1-byte label and
one bit of the candidate table; 16 bytes per batch-hash probe of a flagged
entry; counted in eighths of a byte and rounded).  For a 3-vertex path
query x - y - z every seed (batch edge a-b mapped onto a directed query
edge) has a single last level: the neighbours of the data vertex of the
middle query vertex y with the label of the remaining vertex.  Here that
count is made in Python from the graph and the batch alone: the seeds
follow from the neighbour-label filter (Sec. IV-B) on G u I, the
candidates are the whole label subrange, and the flagged ones are the
subrange's batch edges that pass injectivity.  No kernel output enters
it.  The seed count (batch edges x directed query edges that pass the
filter) is checked the same way."""
import numpy as np
import pytest

import workloads as W
from paper_2401_17018_amd import Context
from test_gpu_parity import _er, _mixed_batch

pytestmark = pytest.mark.gpu

MB_CAND, MB_HASH_PROBE = 41, 128  # eighths of a byte


def _model_eighths(g, q, b):
    labels = np.asarray(g.labels)
    adj = {v: set(g.neighbors(v).tolist()) for v in range(g.n)}
    # canonical batch: net effect, no-ops dropped (inserts of present edges, deletes of absent ones)
    batch = set()
    for s, d, o in zip(b.src.tolist(), b.dst.tolist(), b.op.tolist()):
        key = (min(s, d), max(s, d))
        if (o == 1) != (key[1] in adj[key[0]]):
            batch.add(key)
    gi = {v: set(n) for v, n in adj.items()}  # G u I
    for a, c in batch:
        gi[a].add(c)
        gi[c].add(a)
    qadj = {u: set() for u in range(q.k)}
    for x, y in q.edges.tolist():
        qadj[x].add(y)
        qadj[y].add(x)
    ql = [int(v) for v in q.labels]

    def passes(v, u):  # neighbour-label filter on G u I
        if labels[v] != ql[u]:
            return False
        need = {}
        for w in qadj[u]:
            need[ql[w]] = need.get(ql[w], 0) + 1
        have = {}
        for w in gi[v]:
            have[int(labels[w])] = have.get(int(labels[w]), 0) + 1
        return all(have.get(l, 0) >= c for l, c in need.items())

    total, seeds = 0, 0
    for a, c in batch:
        for x in range(q.k):
            for y in qadj[x]:
                for fx, fy in ((a, c),):  # the other orientation is the reversed query edge
                    if not (passes(fx, x) and passes(fy, y)):
                        continue
                    seeds += 1
                    z = [u for u in range(q.k) if u not in (x, y)][0]
                    mid = x if z in qadj[x] else y  # the matched neighbour of z
                    f = {x: fx, y: fy}
                    sub = [w for w in gi[f[mid]] if labels[w] == ql[z]]
                    used = {f[p] for p in (x, y) if ql[p] == ql[z]}
                    flagged = [w for w in sub if w not in used and (min(f[mid], w), max(f[mid], w)) in batch]
                    total += MB_CAND * len(sub) + MB_HASH_PROBE * len(flagged)
    return total, seeds


@pytest.mark.parametrize("labels", [(0, 1, 2), (0, 1, 0), (1, 1, 1)])
def test_byte_model_of_a_path_query(labels):
    g = _er(400, 2400, 61, 3)
    b = _mixed_batch(g, 62, 120, 40)
    q = W.query_from_edges(3, [(0, 1), (1, 2)], labels)
    want, seeds = _model_eighths(g, q, b)
    assert want > 0 and seeds > 0
    with Context(device=0) as ctx:
        ctx.load_graph(g.row_ptr, g.col, g.labels)
        ctx.register_query(q.k, q.labels, q.edges)
        ctx.set_tuning(coalesced_search=1)  # every directed query edge seeds its own search
        for t in (dict(steal=1), dict(steal=2), dict(steal=1, poll_cycles=500, split_leaf=2, handover_gate=1024)):
            ctx.set_tuning(**t)
            r = ctx.apply_batch(b.src, b.dst, b.op, hash=True, dry_run=True)
            assert r.stats["n_seeds"] == seeds, (labels, t)
            assert r.stats["bytes_alg_dfs"] == (want + 4) // 8, (labels, t)
