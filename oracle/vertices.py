"""Vertex updates reduced to edge updates (Sec. II-A, the batch-dynamic
setting).  TEST INFRASTRUCTURE: see the package docstring for who may use it.

The paper treats a vertex insertion as adding the vertex and then inserting
its incident edges, and a vertex deletion as removing the vertex together
with deletions of every edge incident to it.  Vertex ids stay fixed here: a
deleted vertex remains as an isolated vertex (no query with an edge can use
it), an inserted vertex gets the next free id.

Readings (where the paper says nothing):
  * vertex deletions and the explicit edge updates of the same batch form
    one batch; the deletions contribute the edges the vertex has in G;
  * an explicit insertion that touches a deleted vertex cannot be ordered
    against the deletion and makes the batch a conflict;
  * an explicit deletion of an edge the vertex deletion also removes is a
    duplicate and collapses.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


class _Batch:
    def __init__(self, src, dst, op, elab=None):
        self.src, self.dst, self.op, self.elab = src, dst, op, elab

    def __len__(self):
        return int(self.src.shape[0])


class _Graph:
    def __init__(self, n, row_ptr, col, labels, elab=None, n_elabels=1):
        self.n, self.row_ptr, self.col, self.labels = n, row_ptr, col, labels
        self.elab, self.n_elabels = elab, n_elabels

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[int(self.row_ptr[v]):int(self.row_ptr[v + 1])]


def deletion_batch(graph, batch, vdel) -> Tuple[str, object]:
    """(status, merged batch): the explicit updates followed by one deletion
    (v, w) for every neighbour w of every v in vdel, in G (on an
    edge-labelled graph, with the label of that edge: one deletion per
    labelled edge).  status is "ok", "invalid" (an id >= n) or "conflict"
    (an explicit insertion touches a deleted vertex)."""
    vdel = [int(v) for v in np.asarray(vdel).ravel()]
    if any(v < 0 or v >= graph.n for v in vdel):
        return "invalid", None
    dead = set(vdel)
    for s, d, o in zip(batch.src.tolist(), batch.dst.tolist(), batch.op.tolist()):
        if o == 1 and (s in dead or d in dead):
            return "conflict", None
    gel = getattr(graph, "elab", None)
    src, dst, el = [], [], []
    for v in vdel:  # duplicates in vdel give duplicate deletions, which collapse
        a, b = int(graph.row_ptr[v]), int(graph.row_ptr[v + 1])
        for j in range(a, b):
            src.append(v)
            dst.append(int(graph.col[j]))
            el.append(int(gel[j]) if gel is not None else 0)
    m = len(src)
    out = _Batch(np.concatenate([np.asarray(batch.src, np.uint32), np.array(src, np.uint32)]),
                 np.concatenate([np.asarray(batch.dst, np.uint32), np.array(dst, np.uint32)]),
                 np.concatenate([np.asarray(batch.op, np.uint8), np.zeros(m, np.uint8)]))
    if gel is not None:
        bel = getattr(batch, "elab", None)
        bel = np.zeros(len(batch), np.uint32) if bel is None else np.asarray(bel, np.uint32)
        out.elab = np.concatenate([bel, np.array(el, np.uint32)])
    return "ok", out


def with_vertices(graph, labels):
    """G with isolated vertices of the given labels appended (ids n, n+1, ...)."""
    labels = np.asarray(labels, dtype=np.uint32).ravel()
    nnz = int(graph.row_ptr[-1])
    rp = np.concatenate([np.asarray(graph.row_ptr, np.uint64), np.full(len(labels), nnz, np.uint64)])
    gel = getattr(graph, "elab", None)
    return _Graph(graph.n + len(labels), rp, np.asarray(graph.col, np.uint32).copy(),
                  np.concatenate([np.asarray(graph.labels, np.uint32), labels]),
                  None if gel is None else np.asarray(gel, np.uint32).copy(), getattr(graph, "n_elabels", 1))
