"""Closed forms, invariants and the multiset hash.  TEST INFRASTRUCTURE (see
the package docstring).

These pin the oracle with facts that do not come from running a matcher:
  * star queries: a centre of label c with m_l leaves of label l has
    prod_l (|N^l(v)|)_(m_l) matches per data centre v of label c (falling
    factorials; leaves of one label go injectively to distinct neighbours);
  * the single-edge query (k = 2): each inserted (deleted) edge contributes
    one match per orientation whose labels fit;
  * equal-label triangles: 6 matches per data triangle (3! automorphisms),
    with triangles counted by the textbook node iterator;
  * label-preserving automorphisms of Q act freely on the match set, so every
    result is closed under them and its size is a multiple of |Aut_L(Q)|.
The multiset hash (a checksum of this project, not part of the paper) sums
the tuple's elements times odd position keys (each key a SplitMix64-finaliser
value, Vigna, public domain constants) under one final finaliser; it lets
results be compared at sizes where the tuples are not materialised.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Set, Tuple

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _mix_py(z: int) -> int:
    z &= M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def _term_key(j: int) -> int:
    """K_j = mix(GOLDEN * (j + 1)) | 1: odd, so (v + 1) * K_j is a bijection of v mod 2^64."""
    return _mix_py((GOLDEN * (j + 1)) & M64) | 1


def tuple_hash(qid: int, sign: int, f) -> int:
    """h = mix(mix(qid << 1 | sign) + sum_j (f_j + 1) * K_j), sums and products mod 2^64."""
    s = _mix_py((qid << 1) | (1 if sign else 0))
    for j, v in enumerate(f):
        s = (s + (int(v) + 1) * _term_key(j)) & M64
    return _mix_py(s)


def _mix_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(0xBF58476D1CE4E5B9)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return z


def multiset_hash(tuples: np.ndarray, qid: int, sign: int) -> Tuple[int, int, int]:
    """(count, sum mod 2^64, xor) of tuple_hash over the rows of `tuples`."""
    t = np.asarray(tuples, dtype=np.uint64)
    if t.ndim != 2 or t.shape[0] == 0:
        return 0, 0, 0
    with np.errstate(over="ignore"):
        acc = np.full(t.shape[0], _mix_py((qid << 1) | (1 if sign else 0)), dtype=np.uint64)
        for j in range(t.shape[1]):
            acc = acc + (t[:, j] + np.uint64(1)) * np.uint64(_term_key(j))
        h = _mix_np(acc)
        s = int(np.sum(h, dtype=np.uint64))
    x = int(np.bitwise_xor.reduce(h))
    return int(t.shape[0]), s, x


def falling(a: int, m: int) -> int:
    out = 1
    for i in range(m):
        out *= (a - i)
    return max(out, 0) if a >= m else 0


def star_matches(adj: Dict[int, Set[int]], labels, centre_label: int, leaf_labels) -> int:
    """|M(H)| for a star with the given centre label and leaf labels."""
    need: Dict[int, int] = {}
    for l in leaf_labels:
        need[int(l)] = need.get(int(l), 0) + 1
    total = 0
    for v in range(len(labels)):
        if int(labels[v]) != centre_label:
            continue
        cnt: Dict[int, int] = {}
        for w in adj.get(v, ()):
            cnt[int(labels[w])] = cnt.get(int(labels[w]), 0) + 1
        prod = 1
        for l, m in need.items():
            prod *= falling(cnt.get(l, 0), m)
        total += prod
    return total


def single_edge_delta(edges: Iterable[Tuple[int, int]], labels, lx: int, ly: int) -> int:
    """Matches of the k = 2 query (x - y) that contain a given set of edges."""
    total = 0
    for (a, b) in edges:
        total += int(labels[a] == lx and labels[b] == ly)
        total += int(labels[b] == lx and labels[a] == ly)
    return total


def triangles(adj: Dict[int, Set[int]], vertices: Iterable[int] = None, label=None, labels=None) -> int:
    """Node-iterator triangle count (each triangle once, via its smallest vertex).
    With `label`, only triangles whose three vertices carry that label."""
    count = 0
    for v in (vertices if vertices is not None else adj.keys()):
        if label is not None and labels[v] != label:
            continue
        nb = sorted(w for w in adj.get(v, ()) if w > v and (label is None or labels[w] == label))
        for i in range(len(nb)):
            ai = adj.get(nb[i], ())
            for j in range(i + 1, len(nb)):
                if nb[j] in ai:
                    count += 1
    return count


def automorphisms(k: int, qlabels, qedges) -> list:
    """All label-preserving automorphisms of Q (brute force over k!)."""
    E = {(min(a, b), max(a, b)) for (a, b) in qedges}
    out = []
    for p in itertools.permutations(range(k)):
        if any(int(qlabels[p[i]]) != int(qlabels[i]) for i in range(k)):
            continue
        if all((min(p[a], p[b]), max(p[a], p[b])) in E for (a, b) in E):
            out.append(p)
    return out


def validate_tuple(f, labels, qlabels, qedges, has_edge, batch_edges) -> bool:
    """A tuple is a valid + (or -) result iff it is injective, label-preserving,
    every image edge is in the pass's graph (has_edge) and at least one image
    edge lies in the pass's batch edges."""
    if len(set(f)) != len(f):
        return False
    if any(int(labels[f[i]]) != int(qlabels[i]) for i in range(len(f))):
        return False
    touched = False
    for (a, b) in qedges:
        u, v = int(f[a]), int(f[b])
        if not has_edge(u, v):
            return False
        if (min(u, v), max(u, v)) in batch_edges:
            touched = True
    return touched
