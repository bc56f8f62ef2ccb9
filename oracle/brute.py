"""O1: brute-force incremental matches.  TEST INFRASTRUCTURE (see the
package docstring).

This is the problem statement of Sec. II-A taken literally:
  * Def. 2: a match of Q in a graph H is an injective map f: V(Q) -> V(H)
    with L(f(u)) = L(u) for every query vertex and {f(u), f(u')} in E(H) for
    every query edge (a non-induced embedding; automorphic images are
    distinct matches).
  * Def. 1 / problem statement: a batch is a set of edge insertions and
    deletions; G' is G after the batch, and the incremental matches are the
    difference of the match sets of G and G' (read here as the net change:
    result(+) = M(G') minus M(G), result(-) = M(G) minus M(G'); the paper's
    Example 1 reports only the net effect of a batch).
It enumerates M(G) and M(G') completely by backtracking over the query
vertices in id order (candidates: every unused data vertex with the right
label; an edge is checked once both its ends are placed) and returns the two
set differences.  No seeds, no order rule, no intersections.  The `_el`
functions at the end do the same for edge-labelled graphs.
"""
from __future__ import annotations

from typing import Dict, List, Set, Tuple


def canonical(n: int, edges: Set[Tuple[int, int]], ups):
    """Canonicalise a batch [(op, u, v)] (op 1 = insert, 0 = delete).

    Returns (status, I, D, n_noop, n_dup) with status in {"ok", "invalid",
    "conflict"}; I and D are sorted lists of (lo, hi)."""
    seen: Dict[Tuple[int, int], int] = {}
    n_dup = 0
    for (op, u, v) in ups:
        if u == v or not (0 <= u < n) or not (0 <= v < n):
            return "invalid", [], [], 0, 0
        e = (min(u, v), max(u, v))
        if e in seen:
            if seen[e] != op:
                return "conflict", [], [], 0, 0
            n_dup += 1
            continue
        seen[e] = op
    I, D, n_noop = [], [], 0
    for e, op in seen.items():
        present = e in edges
        if op == 1 and not present:
            I.append(e)
        elif op == 0 and present:
            D.append(e)
        else:
            n_noop += 1
    return "ok", sorted(I), sorted(D), n_noop, n_dup


def all_matches(n: int, labels, adj: Dict[int, Set[int]], k: int, qlabels, qedges) -> Set[tuple]:
    """Every match of Q in H (Def. 2) by plain backtracking."""
    qadj = [[False] * k for _ in range(k)]
    for (a, b) in qedges:
        qadj[a][b] = qadj[b][a] = True
    by_label: Dict[int, List[int]] = {}
    for v in range(n):
        by_label.setdefault(int(labels[v]), []).append(v)
    out: Set[tuple] = set()
    f = [-1] * k

    def rec(u: int):
        if u == k:
            out.add(tuple(f))
            return
        for c in by_label.get(int(qlabels[u]), []):
            if c in f[:u]:
                continue
            ok = True
            for w in range(u):
                if qadj[u][w] and c not in adj.get(f[w], ()):
                    ok = False
                    break
            if ok:
                f[u] = c
                rec(u + 1)
                f[u] = -1

    rec(0)
    return out


def edge_set(graph) -> Set[Tuple[int, int]]:
    s = set()
    for v in range(graph.n):
        for w in graph.neighbors(v).tolist():
            if v < w:
                s.add((v, int(w)))
    return s


def adjacency(n: int, edges: Set[Tuple[int, int]]) -> Dict[int, Set[int]]:
    adj: Dict[int, Set[int]] = {}
    for (a, b) in edges:
        adj.setdefault(a, set()).add(b)
        adj.setdefault(b, set()).add(a)
    return adj


def bdsm(graph, query, batch) -> dict:
    """O1 result for one batch: {status, plus, minus, I, D, n_noop, n_dup}."""
    E = edge_set(graph)
    ups = list(zip(batch.op.tolist(), batch.src.tolist(), batch.dst.tolist()))
    status, I, D, n_noop, n_dup = canonical(graph.n, E, ups)
    if status != "ok":
        return {"status": status}
    E2 = (E | set(I)) - set(D)
    qe = [tuple(e) for e in query.edges.tolist()]
    M1 = all_matches(graph.n, graph.labels, adjacency(graph.n, E), query.k, query.labels, qe)
    M2 = all_matches(graph.n, graph.labels, adjacency(graph.n, E2), query.k, query.labels, qe)
    return {"status": "ok", "plus": M2 - M1, "minus": M1 - M2, "I": I, "D": D, "n_noop": n_noop,
            "n_dup": n_dup, "E2": E2}


# ------------------------------------------------------------ edge labels
#
# Sec. II-A lets the labelling function cover edges too.  A data edge is then
# a triple (lo, hi, e); a query edge (a, b) with label e maps onto the data
# edge {f(a), f(b)} with label e.  The graph stays simple: one edge, with one
# label, per pair.  An update names a triple; two updates of the same pair in
# one batch must be the same triple and op (a duplicate), otherwise the
# batch is a conflict; inserting a pair present under another label is
# invalid; deleting a triple whose pair has another label is a no-op.


def edge_set_el(graph) -> Set[Tuple[int, int, int]]:
    """Undirected labelled edges (lo, hi, e) of a graph with per-entry labels."""
    el = getattr(graph, "elab", None)
    s = set()
    for v in range(graph.n):
        a, b = int(graph.row_ptr[v]), int(graph.row_ptr[v + 1])
        for j in range(a, b):
            w = int(graph.col[j])
            if v < w:
                s.add((v, w, int(el[j]) if el is not None else 0))
    return s


def canonical_el(n: int, n_el: int, edges: Set[Tuple[int, int, int]], ups):
    """Canonicalise a labelled batch [(op, u, v, e)].  Returns (status, I, D,
    n_noop, n_dup); I and D are sorted lists of (lo, hi, e)."""
    seen: Dict[Tuple[int, int], Tuple[int, int]] = {}
    n_dup = 0
    for (op, u, v, e) in ups:
        if u == v or not (0 <= u < n) or not (0 <= v < n) or not (0 <= e < n_el):
            return "invalid", [], [], 0, 0
        pair = (min(u, v), max(u, v))
        if pair in seen:
            if seen[pair] != (op, e):
                return "conflict", [], [], 0, 0
            n_dup += 1
            continue
        seen[pair] = (op, e)
    I, D, n_noop = [], [], 0
    pair_label = {(lo, hi): e for (lo, hi, e) in edges}
    for (lo, hi), (op, e) in seen.items():
        present = (lo, hi, e) in edges
        if op == 1 and not present and (lo, hi) in pair_label:
            return "invalid", [], [], 0, 0
        if op == 1 and not present:
            I.append((lo, hi, e))
        elif op == 0 and present:
            D.append((lo, hi, e))
        else:
            n_noop += 1
    return "ok", sorted(I), sorted(D), n_noop, n_dup


def all_matches_el(n: int, labels, edges: Set[Tuple[int, int, int]], k: int, qlabels, qedges, qelabels) -> Set[tuple]:
    """Every match of an edge-labelled Q in H by plain backtracking."""
    has = set()
    for (a, b, e) in edges:
        has.add((a, b, e))
        has.add((b, a, e))
    need: Dict[Tuple[int, int], int] = {}
    for (a, b), e in zip(qedges, qelabels):
        need[(a, b)] = int(e)
        need[(b, a)] = int(e)
    out: Set[tuple] = set()
    f = [-1] * k

    def rec(u: int):
        if u == k:
            out.add(tuple(f))
            return
        for c in range(n):
            if int(labels[c]) != int(qlabels[u]) or c in f[:u]:
                continue
            if all((f[w], c, need[(w, u)]) in has for w in range(u) if (w, u) in need):
                f[u] = c
                rec(u + 1)
                f[u] = -1

    rec(0)
    return out


def bdsm_el(graph, query, batch) -> dict:
    """O1 result for one batch on an edge-labelled graph."""
    n_el = int(getattr(graph, "n_elabels", 1) or 1)
    E = edge_set_el(graph)
    bel = getattr(batch, "elab", None)
    ups = [(int(o), int(s), int(d), int(bel[i]) if bel is not None else 0)
           for i, (o, s, d) in enumerate(zip(batch.op.tolist(), batch.src.tolist(), batch.dst.tolist()))]
    status, I, D, n_noop, n_dup = canonical_el(graph.n, n_el, E, ups)
    if status != "ok":
        return {"status": status}
    E2 = (E | set(I)) - set(D)
    qe = [tuple(e) for e in query.edges.tolist()]
    qel = getattr(query, "elabels", None)
    qel = [0] * len(qe) if qel is None else [int(x) for x in qel]
    M1 = all_matches_el(graph.n, graph.labels, E, query.k, query.labels, qe, qel)
    M2 = all_matches_el(graph.n, graph.labels, E2, query.k, query.labels, qe, qel)
    return {"status": "ok", "plus": M2 - M1, "minus": M1 - M2, "I": I, "D": D, "n_noop": n_noop,
            "n_dup": n_dup, "E2": E2}
