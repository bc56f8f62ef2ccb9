"""Seeded synthetic workloads for batch-dynamic subgraph matching.

This module only draws inputs: data graphs (Erdos-Renyi, R-MAT), vertex
labels (uniform, Zipf), query graphs extracted from the data graph, and
update batches.  It performs no step of the matching method, and both the
oracle's tests and the GPU path consume what it returns.

Workload shapes follow the paper's experimental setup (Sec. VI-A): power-law
data graphs with skewed label alphabets (Table II) stand in for its datasets,
queries are extracted from the data graph by random walks and classed as
Dense (average degree >= 3), Sparse (< 3) or Tree, and batches mix edge
insertions with deletions.  The concrete sizes are those of tiny(), mid(),
large() and batched_queries() below.

Randomness is counter-based (SplitMix64 finaliser), so every array is a pure
function of (seed, tag, counter) and independent of thread counts.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libwlgen.so")
_lib = None

TAG_GRAPH, TAG_LABELS, TAG_PERM, TAG_QUERY, TAG_BATCH, TAG_STREAM, TAG_SHUFFLE = 1, 2, 3, 4, 5, 6, 7


def build_native(force: bool = False) -> str:
    """Compile the generator library (g++ with OpenMP) next to this file."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["g++", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c++17",
             os.path.join(_HERE, "gen.cpp"), "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        build_native(False)
        lib = ctypes.CDLL(_SO)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        lib.wl_mix64.restype = ctypes.c_uint64
        lib.wl_mix64.argtypes = [ctypes.c_uint64]
        lib.wl_draw.restype = ctypes.c_uint64
        lib.wl_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.wl_stream_key.restype = ctypes.c_uint64
        lib.wl_stream_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.wl_draws.restype = None
        lib.wl_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u64p, ctypes.c_int]
        lib.wl_er_edges.restype = ctypes.c_int64
        lib.wl_er_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p, u32p, ctypes.c_int]
        lib.wl_rmat_edges.restype = ctypes.c_int64
        lib.wl_rmat_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_uint64, u32p, u32p, ctypes.c_int]
        lib.wl_permutation.restype = None
        lib.wl_permutation.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p]
        lib.wl_apply_perm.restype = None
        lib.wl_apply_perm.argtypes = [ctypes.c_uint64, u32p, u32p, u32p, ctypes.c_int]
        lib.wl_shuffle_edges.restype = None
        lib.wl_shuffle_edges.argtypes = [ctypes.c_uint64, u32p, u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        lib.wl_build_csr.restype = ctypes.c_int
        lib.wl_build_csr.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p, u64p, u32p, ctypes.c_int]
        lib.wl_labels_uniform.restype = None
        lib.wl_labels_uniform.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                          u32p, ctypes.c_int]
        lib.wl_labels_zipf.restype = None
        lib.wl_labels_zipf.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64,
                                       ctypes.c_uint64, u32p, ctypes.c_int]
        _lib = lib
    return _lib


def _threads(threads: int) -> int:
    return int(threads) if threads and threads > 0 else 0


# --------------------------------------------------------------------------
# counter-based draws


class Draws:
    """Sequential reader over the counter-based stream (seed, tag)."""

    def __init__(self, seed: int, tag: int):
        self.key = _L().wl_stream_key(seed & (2**64 - 1), tag)
        self.ctr = 0

    def block(self, n: int) -> np.ndarray:
        out = np.empty(int(n), dtype=np.uint64)
        if n:
            _L().wl_draws(self.key, self.ctr, int(n), out, 0)
        self.ctr += int(n)
        return out

    def u64(self) -> int:
        v = _L().wl_draw(self.key, self.ctr)
        self.ctr += 1
        return int(v)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n)."""
        return (self.u64() * int(n)) >> 64

    def below_vec(self, count: int, n: int) -> np.ndarray:
        r = self.block(count)
        hi = (r >> np.uint64(32)).astype(np.uint64)
        lo = (r & np.uint64(0xFFFFFFFF)).astype(np.uint64)
        nn = np.uint64(n)
        # multiply-high of a 64-bit draw by n < 2^32, computed in two halves
        return ((hi * nn + ((lo * nn) >> np.uint64(32))) >> np.uint64(32)).astype(np.int64)


def sub_seed(seed: int, tag: int) -> int:
    """Component seed: splitmix64 finaliser of (master seed ^ tag)."""
    return int(_L().wl_mix64((seed ^ tag) & (2**64 - 1)))


# --------------------------------------------------------------------------
# data structures


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # uint64 [n+1]
    col: np.ndarray  # uint32 [2m], ascending per row
    labels: np.ndarray  # uint32 [n]
    name: str = ""
    elab: Optional[np.ndarray] = None  # uint32 [2m] edge label per CSR entry (None: unlabelled)
    n_elabels: int = 1  # edge labels are < n_elabels

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[int(self.row_ptr[v]):int(self.row_ptr[v + 1])]

    def has_edge(self, u: int, v: int) -> bool:
        r = self.neighbors(u)
        i = int(np.searchsorted(r, v))
        return i < len(r) and int(r[i]) == v

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def edge_keys(self) -> np.ndarray:
        """Canonical undirected edges as uint64 keys lo << 32 | hi, ascending."""
        src = np.repeat(np.arange(self.n, dtype=np.uint64), np.diff(self.row_ptr).astype(np.int64))
        dst = self.col.astype(np.uint64)
        keep = src < dst
        return (src[keep] << np.uint64(32)) | dst[keep]


@dataclass
class Query:
    k: int
    labels: np.ndarray  # uint32 [k]
    edges: np.ndarray  # uint32 [m, 2]
    kind: str = ""
    planted: Optional[Tuple[int, ...]] = None  # a data-vertex tuple known to be in the + result
    elabels: Optional[np.ndarray] = None  # uint32 [m] edge label per query edge (None: all 0)

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])


@dataclass
class Batch:
    src: np.ndarray  # uint32
    dst: np.ndarray  # uint32
    op: np.ndarray  # uint8, 1 = insertion, 0 = deletion
    elab: Optional[np.ndarray] = None  # uint32 edge label per update (None: all 0)

    def __len__(self):
        return int(self.src.shape[0])

    def inverse(self) -> "Batch":
        return Batch(self.src.copy(), self.dst.copy(), (1 - self.op).astype(np.uint8),
                     None if self.elab is None else self.elab.copy())


@dataclass
class Workload:
    name: str
    graph: Graph
    queries: List[Query]
    batches: List[Batch]
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# graph generators


def csr_from_edges(n: int, lo: np.ndarray, hi: np.ndarray, threads: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    lo = np.ascontiguousarray(lo, dtype=np.uint32)
    hi = np.ascontiguousarray(hi, dtype=np.uint32)
    m = int(lo.shape[0])
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    col = np.empty(2 * m, dtype=np.uint32)
    _L().wl_build_csr(n, m, lo, hi, row_ptr, col, _threads(threads))
    return row_ptr, col


def er_edges(n: int, m: int, seed: int, threads: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    lo = np.empty(m, dtype=np.uint32)
    hi = np.empty(m, dtype=np.uint32)
    r = _L().wl_er_edges(n, m, seed, lo, hi, _threads(threads))
    if r != m:
        raise ValueError("infeasible ER request")
    return lo, hi


def rmat_edges(scale: int, m: int, seed: int, abc=(0.57, 0.19, 0.19), threads: int = 0):
    lo = np.empty(m, dtype=np.uint32)
    hi = np.empty(m, dtype=np.uint32)
    r = _L().wl_rmat_edges(scale, m, abc[0], abc[1], abc[2], seed, lo, hi, _threads(threads))
    if r != m:
        raise ValueError("R-MAT generation failed")
    return lo, hi


def labels_uniform(n: int, L: int, seed: int, threads: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _L().wl_labels_uniform(n, L, seed, TAG_LABELS, out, _threads(threads))
    return out


def labels_zipf(n: int, L: int, s: float, seed: int, threads: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _L().wl_labels_zipf(n, L, s, seed, TAG_LABELS, out, _threads(threads))
    return out


def rmat_graph_with_pool(scale: int, m_graph: int, pool: int, L: int, zipf_s: float, seed: int,
                         threads: int = 0, name: str = "") -> Tuple[Graph, np.ndarray, np.ndarray]:
    """R-MAT graph with |E| = m_graph plus a disjoint pool of held-out edges.

    Steps: draw m_graph + pool distinct R-MAT pairs, permute vertex ids, shuffle
    the edge list, and hold out its first `pool` edges for insertions."""
    n = 1 << scale
    lo, hi = rmat_edges(scale, m_graph + pool, sub_seed(seed, TAG_GRAPH), threads=threads)
    perm = np.empty(n, dtype=np.uint32)
    _L().wl_permutation(n, sub_seed(seed, TAG_PERM), TAG_PERM, perm)
    _L().wl_apply_perm(lo.shape[0], lo, hi, perm, _threads(threads))
    _L().wl_shuffle_edges(lo.shape[0], lo, hi, sub_seed(seed, TAG_SHUFFLE), TAG_SHUFFLE, _threads(threads))
    pool_lo, pool_hi = lo[:pool].copy(), hi[:pool].copy()
    g_lo, g_hi = lo[pool:], hi[pool:]
    row_ptr, col = csr_from_edges(n, g_lo, g_hi, threads)
    del lo, hi, g_lo, g_hi
    labels = labels_zipf(n, L, zipf_s, sub_seed(seed, TAG_LABELS), threads)
    return Graph(n, row_ptr, col, labels, name), pool_lo, pool_hi


# --------------------------------------------------------------------------
# batches


class EdgeShadow:
    """Host copy of the current edge set, to draw valid deletions."""

    def __init__(self, graph: Graph):
        self.keys = graph.edge_keys()
        self.cnt = int(self.keys.shape[0])

    def sample_deletions(self, count: int, draws: Draws, protect: set) -> np.ndarray:
        out = []
        taken = set()
        while len(out) < count:
            need = count - len(out)
            pos = draws.below_vec(need * 2 + 16, self.cnt)
            for p in pos.tolist():
                if p in taken:
                    continue
                key = int(self.keys[p])
                if key in protect:
                    continue
                taken.add(p)
                out.append(p)
                if len(out) == count:
                    break
        pos = np.array(sorted(out, reverse=True), dtype=np.int64)
        sel = self.keys[pos].copy()
        # swap-remove, highest positions first so swaps stay valid
        for p in pos.tolist():
            self.cnt -= 1
            self.keys[p] = self.keys[self.cnt]
        self.keys = self.keys[: self.cnt]
        return sel

    def add(self, keys: np.ndarray):
        self.keys = np.concatenate([self.keys[: self.cnt], keys.astype(np.uint64)])
        self.cnt = int(self.keys.shape[0])


def make_batch(ins_keys: np.ndarray, del_keys: np.ndarray, draws: Draws) -> Batch:
    """Mix insertions and deletions, shuffle the order and orient each pair at random."""
    keys = np.concatenate([ins_keys.astype(np.uint64), del_keys.astype(np.uint64)])
    ops = np.concatenate([np.ones(len(ins_keys), np.uint8), np.zeros(len(del_keys), np.uint8)])
    n = keys.shape[0]
    order = np.argsort(draws.block(n), kind="stable")
    keys, ops = keys[order], ops[order]
    flip = (draws.block(n) & np.uint64(1)).astype(bool)
    a = (keys >> np.uint64(32)).astype(np.uint32)
    b = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    src = np.where(flip, b, a).astype(np.uint32)
    dst = np.where(flip, a, b).astype(np.uint32)
    return Batch(src, dst, ops)


def keys_of(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    a = np.minimum(lo, hi).astype(np.uint64)
    b = np.maximum(lo, hi).astype(np.uint64)
    return (a << np.uint64(32)) | b


# --------------------------------------------------------------------------
# query extraction (random walks on G u I)


class _Adj:
    """Neighbour lookup over the CSR graph plus a set of inserted edges,
    optionally restricted to vertices whose label is >= min_label."""

    def __init__(self, graph: Graph, ins_keys: np.ndarray, min_label: int = 0):
        self.g = graph
        self.min_label = min_label
        self.extra = {}
        for key in ins_keys.tolist():
            a, b = key >> 32, key & 0xFFFFFFFF
            self.extra.setdefault(a, []).append(b)
            self.extra.setdefault(b, []).append(a)

    def nbrs(self, v: int) -> np.ndarray:
        r = self.g.neighbors(v)
        e = self.extra.get(v)
        if e:
            r = np.union1d(r, np.array(e, dtype=np.uint32))
        if self.min_label:
            r = r[self.g.labels[r] >= self.min_label]
        return r

    def has(self, u: int, v: int) -> bool:
        r = self.nbrs(u)
        i = int(np.searchsorted(r, v))
        return i < len(r) and int(r[i]) == v


def _walk_vertices(adj: _Adj, a: int, b: int, k: int, draws: Draws, max_steps: int = 100000):
    order = [a, b]
    tree = [(0, 1)]
    pos = {a: 0, b: 1}
    cur = b
    steps = 0
    while len(order) < k and steps < max_steps:
        nb = adj.nbrs(cur)
        if len(nb) == 0:
            return None
        nxt = int(nb[draws.below(len(nb))])
        if nxt not in pos:
            pos[nxt] = len(order)
            tree.append((pos[cur], pos[nxt]))
            order.append(nxt)
        cur = nxt
        steps += 1
    if len(order) < k:
        return None
    return order, tree


def _induced_edges(adj: _Adj, verts: Sequence[int]) -> List[Tuple[int, int]]:
    out = []
    for i in range(len(verts)):
        for j in range(i + 1, len(verts)):
            if adj.has(verts[i], verts[j]):
                out.append((i, j))
    return out


def extract_query(graph: Graph, ins_keys: np.ndarray, k: int, kind: str, seed: int,
                  dense_ratio: float = 0.6, max_tries: int = 10000, min_label: int = 0) -> Query:
    """Extract a connected k-vertex query whose first edge maps to an inserted edge.

    kind = "induced": the walk's vertex set with every edge among them in G u I.
    kind = "sparse":  the walk's discovery tree plus one extra induced edge.
    kind = "tree":    the walk's discovery tree.
    kind = "dense":   greedy densifying growth; ceil(dense_ratio * C(k,2)) edges.
    The identity map onto the walk's vertices is a match in G' that uses an
    inserted edge, so it belongs to the insertion result (the planted match).
    With min_label > 0 the walk only visits vertices whose label is >=
    min_label (labels are ranked by frequency, so these are the rarer ones)."""
    adj = _Adj(graph, ins_keys, min_label)
    draws = Draws(seed, TAG_QUERY)
    if min_label:
        a_lab = graph.labels[(ins_keys >> np.uint64(32)).astype(np.int64)]
        b_lab = graph.labels[(ins_keys & np.uint64(0xFFFFFFFF)).astype(np.int64)]
        ins_keys = ins_keys[(a_lab >= min_label) & (b_lab >= min_label)]
        if ins_keys.shape[0] == 0:
            raise RuntimeError("no inserted edge between vertices of the allowed labels")
    n_ins = int(ins_keys.shape[0])
    best = None
    for attempt in range(max_tries):
        key = int(ins_keys[draws.below(n_ins)])
        a, b = key >> 32, key & 0xFFFFFFFF
        if draws.below(2):
            a, b = b, a
        if kind == "dense":
            verts = [a, b]
            inset = {a, b}
            tree = [(0, 1)]
            ok = True
            while len(verts) < k:
                cand = np.concatenate([adj.nbrs(v) for v in verts])
                u, cnt = np.unique(cand, return_counts=True)
                msk = ~np.isin(u, np.array(verts, dtype=np.uint32))
                u, cnt = u[msk], cnt[msk]
                if len(u) == 0:
                    ok = False
                    break
                top = cnt.max()
                best_u = u[cnt == top]
                pick = int(best_u[draws.below(len(best_u))])
                # attach to its lowest-index neighbour in the set
                par = next(i for i, v in enumerate(verts) if adj.has(v, pick))
                tree.append((par, len(verts)))
                verts.append(pick)
                inset.add(pick)
            if not ok:
                continue
            ind = _induced_edges(adj, verts)
            target = math.ceil(dense_ratio * k * (k - 1) / 2 - 1e-9)
            if len(ind) < target:
                if best is None or len(ind) > best[2]:
                    best = (verts, tree, len(ind), ind)
                continue
            edges = _pick_edges(tree, ind, target, draws)
            return _mk_query(graph, verts, edges, "dense")
        res = _walk_vertices(adj, a, b, k, draws)
        if res is None:
            continue
        verts, tree = res
        if len(set(verts)) != k:
            continue
        ind = _induced_edges(adj, verts)
        if kind == "induced":
            return _mk_query(graph, verts, ind, "induced")
        if kind == "tree":
            return _mk_query(graph, verts, tree, "tree")
        if kind == "sparse":
            tset = {tuple(sorted(e)) for e in tree}
            extra = [e for e in ind if e not in tset]
            if not extra:
                continue
            e = extra[draws.below(len(extra))]
            return _mk_query(graph, verts, sorted(tset) + [e], "sparse")
        raise ValueError(kind)
    if kind == "dense" and best is not None:
        verts, tree, _, ind = best
        return _mk_query(graph, verts, ind, "dense")
    raise RuntimeError("query extraction failed")


def _pick_edges(tree, ind, target, draws: Draws):
    tset = {tuple(sorted(e)) for e in tree}
    rest = [e for e in ind if e not in tset]
    order = np.argsort(draws.block(len(rest)), kind="stable")
    need = target - len(tset)
    return sorted(tset) + [rest[i] for i in order[:need].tolist()]


def _mk_query(graph: Graph, verts, edges, kind) -> Query:
    e = np.array(sorted({tuple(sorted(x)) for x in edges}), dtype=np.uint32).reshape(-1, 2)
    labels = graph.labels[np.array(verts, dtype=np.int64)].astype(np.uint32)
    return Query(len(verts), labels, e, kind, tuple(int(v) for v in verts))


# --------------------------------------------------------------------------
# the five configurations


def tiny(seed: int = 0) -> Workload:
    """ER G(1000, 8000), 4 uniform labels, triangle-with-pendant query whose
    labels are those of 4 uniformly drawn data vertices, 100 insertions of
    distinct non-adjacent pairs."""
    n, m = 1000, 8000
    lo, hi = er_edges(n, m, sub_seed(seed, TAG_GRAPH))
    row_ptr, col = csr_from_edges(n, lo, hi)
    labels = labels_uniform(n, 4, sub_seed(seed, TAG_LABELS))
    g = Graph(n, row_ptr, col, labels, "tiny-er")
    qd = Draws(sub_seed(seed, TAG_QUERY), TAG_QUERY)
    qv = [qd.below(n) for _ in range(4)]
    q = Query(4, labels[np.array(qv)].astype(np.uint32),
              np.array([[0, 1], [1, 2], [0, 2], [2, 3]], dtype=np.uint32), "triangle+pendant")
    bd = Draws(sub_seed(seed, TAG_BATCH), TAG_BATCH)
    existing = set(g.edge_keys().tolist())
    ins = []
    seen = set()
    while len(ins) < 100:
        u, v = bd.below(n), bd.below(n)
        if u == v:
            continue
        key = (min(u, v) << 32) | max(u, v)
        if key in existing or key in seen:
            continue
        seen.add(key)
        ins.append(key)
    b = make_batch(np.array(ins, dtype=np.uint64), np.zeros(0, np.uint64), bd)
    return Workload("tiny", g, [q], [b], {"seed": seed})


def rmat_stream(scale: int, m_graph: int, L: int, zipf_s: float, n_ins: int, n_del: int,
                n_batches: int, queries_spec: Sequence[Tuple[int, str]], seed: int = 0,
                pool_batches: Optional[int] = None, name: str = "", threads: int = 0,
                query_min_label=0) -> Workload:
    """R-MAT graph, a stream of mixed batches, and queries extracted on G u I_0.
    query_min_label: one lowest label rank for every query's walk, or a
    sequence with one per query."""
    pool_batches = pool_batches or n_batches
    if n_batches > pool_batches:
        raise ValueError("more batches than the hold-out pool covers")
    g, pl, ph = rmat_graph_with_pool(scale, m_graph, n_ins * pool_batches, L, zipf_s, seed,
                                     threads=threads, name=name)
    pool = keys_of(pl, ph)
    ins0 = pool[:n_ins]
    queries = []
    protect = set()
    for qi, (k, kind) in enumerate(queries_spec):
        ml = query_min_label[qi] if isinstance(query_min_label, (list, tuple)) else query_min_label
        q = extract_query(g, ins0, k, kind, sub_seed(seed, TAG_QUERY + 97 * (qi + 1)), min_label=ml)
        queries.append(q)
        for (x, y) in q.edges.tolist():
            a, b = q.planted[x], q.planted[y]
            protect.add((min(a, b) << 32) | max(a, b))
    shadow = EdgeShadow(g)
    bd = Draws(sub_seed(seed, TAG_BATCH), TAG_BATCH)
    batches = []
    for t in range(n_batches):
        ins = pool[t * n_ins:(t + 1) * n_ins]
        dels = shadow.sample_deletions(n_del, bd, protect) if n_del else np.zeros(0, np.uint64)
        shadow.add(ins)
        batches.append(make_batch(ins, dels, bd))
    return Workload(name, g, queries, batches, {"seed": seed, "scale": scale, "m_graph": m_graph})


def mid(seed: int = 0, n_batches: int = 1, threads: int = 0) -> Workload:
    """R-MAT scale 20 (a,b,c,d = .57,.19,.19,.05), |E| = 8 * 2^20 (average
    degree 16), 16 Zipf(1.2) labels, one 6-vertex query induced on a random
    walk, batches of 8,000 insertions and 2,000 deletions."""
    return rmat_stream(20, 8 << 20, 16, 1.2, 8000, 2000, n_batches, [(6, "induced")], seed,
                       pool_batches=max(64, n_batches), name="mid-rmat20", threads=threads)


# Zipf(1.0) over 32 labels: each label of rank >= 12 covers <= 1.9 % of the
# vertices, each of rank >= 20 <= 1.2 %
LARGE_QUERY_MIN_LABEL = 12         # the dense query's walk
LARGE_SPARSE_QUERY_MIN_LABEL = 20  # the sparse query's walk


def large(seed: int = 0, n_batches: int = 1, threads: int = 0) -> Workload:
    """R-MAT scale 24, |E| = 16 * 2^24 (average degree 32 = 2^29 CSR
    entries), 32 Zipf(1.0) labels, two 8-vertex queries (sparse: tree + one
    cycle; dense: 17 edges), batches of 90,000 insertions and 10,000 deletions.
    The query walks visit only vertices of the rarer labels: with walks
    through the most frequent labels, 100 of a batch's 10^5 updates already
    gave 1.4 * 10^12 incremental matches before a 60 s deadline.  The dense
    query's walk keeps to labels of rank >= 12; the sparse query, with 8
    edges instead of 17, has far more matches for the same labels, and its
    walk keeps to labels of rank >= 20."""
    return rmat_stream(24, 16 << 24, 32, 1.0, 90000, 10000, n_batches, [(8, "sparse"), (8, "dense")],
                       seed, pool_batches=max(16, n_batches), name="large-rmat24", threads=threads,
                       query_min_label=(LARGE_SPARSE_QUERY_MIN_LABEL, LARGE_QUERY_MIN_LABEL))


BATCHED_QUERY_MIN_LABEL = 8  # Zipf(1.2) over 16 labels: each label >= 8 covers <= 2.6% of vertices


def symmetric_queries(seed: int = 0, n_batches: int = 1, threads: int = 0) -> Workload:
    """The mid graph and its batch stream with four queries that have
    label-preserving automorphisms: triangle and K4 on label 0, a 4-cycle
    on label 1, a star with a label-2 centre and three label-1 leaves."""
    w = mid(seed, n_batches=n_batches, threads=threads)
    w.queries = [query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 0), "dense"),
                 query_from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)], (1, 1, 1, 1), "sparse"),
                 query_from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], (0, 0, 0, 0), "dense"),
                 query_from_edges(4, [(0, 1), (0, 2), (0, 3)], (2, 1, 1, 1), "tree")]
    w.name = "symmetric-rmat20"
    return w


def core_symmetric_queries(seed: int = 0, n_batches: int = 1, threads: int = 0) -> Workload:
    """The mid graph and its batch stream with four queries that have no
    automorphism of their own but whose cores (the query without its
    degree-1 vertices) have: a triangle with labels 0, 1, 1 and a label-2
    leaf on one label-1 vertex; a label-1 triangle with leaves of labels 4
    and 5 on two of its vertices; a label-2 4-cycle with leaves of labels 4
    and 5 on two adjacent vertices; two label-1 triangles on a shared edge
    with leaves of labels 4 and 5 on a shared and an unshared vertex.
    (About 10^10 matches change per batch, most of them the last two's.)"""
    w = mid(seed, n_batches=n_batches, threads=threads)
    w.queries = [
        query_from_edges(4, [(0, 1), (1, 2), (2, 0), (1, 3)], (0, 1, 1, 2), "dense"),
        query_from_edges(5, [(0, 1), (1, 2), (2, 0), (0, 3), (1, 4)], (1, 1, 1, 4, 5), "dense"),
        query_from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 5)], (2, 2, 2, 2, 4, 5), "sparse"),
        query_from_edges(6, [(0, 1), (1, 2), (2, 0), (1, 3), (3, 0), (0, 4), (2, 5)], (1, 1, 1, 1, 4, 5), "dense"),
    ]
    w.name = "core-symmetric-rmat20"
    return w


def _batched_spec(seed: int, n_queries: int, sparse_max: int = 12):
    """(k, kind) per query: odd ids dense with k ~ U{4..12}, even ids sparse
    with k = 4 + (draw mod (sparse_max - 3)) from the same draw."""
    d = Draws(sub_seed(seed, TAG_QUERY + 1000), TAG_QUERY)
    spec = []
    for i in range(n_queries):
        k = 4 + d.below(9)
        spec.append((4 + (k - 4) % (sparse_max - 3), "sparse") if i % 2 == 0 else (k, "dense"))
    return spec


def served_stream(seed: int = 0, n_requests: int = 200, n_queries: int = 32, size_lo: int = 100,
                  size_hi: int = 10000, ins_frac: float = 0.85, threads: int = 0, large: bool = False) -> Workload:
    """A request stream for the served path: the mid graph, the first
    n_queries standing queries of batched_queries() with sparse sizes
    capped at 8 (larger sparse queries are unsolved), and n_requests update
    requests valid in sequence, of log-uniform size in [size_lo, size_hi]
    with ins_frac insertions (held-out edges) and the rest deletions of
    present edges.  meta["gaps"] holds unit-mean exponential inter-arrival
    gaps (a Poisson process once scaled to the offered load).

    large=True: the large workload's graph (R-MAT scale 24, 2^28 edges, 32
    Zipf(1.0) labels) with queries of 4..10 vertices whose walks keep to the
    large workload's label ranks (sparse >= 20, dense >= 12)."""
    d = Draws(sub_seed(seed, TAG_STREAM + 11 + (500 if large else 0)), TAG_STREAM)
    lo, hi = math.log10(size_lo), math.log10(size_hi)
    u = d.block(n_requests).astype(np.float64) / 2.0 ** 64
    sizes = np.floor(10.0 ** (lo + u * (hi - lo))).astype(np.int64)
    n_ins = np.rint(sizes * ins_frac).astype(np.int64)
    n_del = sizes - n_ins
    gaps = -np.log1p(-d.block(n_requests).astype(np.float64) / 2.0 ** 64)
    name = "served-large-rmat24" if large else "served-rmat20"
    if large:
        g, pl, ph = rmat_graph_with_pool(24, 16 << 24, int(n_ins.sum()), 32, 1.0, seed, threads=threads, name=name)
    else:
        g, pl, ph = rmat_graph_with_pool(20, 8 << 20, int(n_ins.sum()), 16, 1.2, seed, threads=threads, name=name)
    pool = keys_of(pl, ph)
    # queries are extracted on G u (the first request's insertions); on the
    # large graph on G u (the first 2 * 10^4 insertions of the stream), so
    # that walks over its rare labels find an inserted edge to start from
    ins0 = pool[: max(int(n_ins[0]), min(int(n_ins.sum()), 20000))] if large else pool[: int(n_ins[0])]
    queries, protect = [], set()
    spec = _batched_spec(seed, n_queries, sparse_max=10 if large else 8)
    for qi, (k, kind) in enumerate(spec):
        if large:
            k = min(k, 10)
            ml = LARGE_SPARSE_QUERY_MIN_LABEL if kind == "sparse" else LARGE_QUERY_MIN_LABEL
        else:
            ml = BATCHED_QUERY_MIN_LABEL
        q = extract_query(g, ins0, k, kind, sub_seed(seed, TAG_QUERY + 97 * (qi + 1)), min_label=ml)
        queries.append(q)
        for (x, y) in q.edges.tolist():
            a, b = q.planted[x], q.planted[y]
            protect.add((min(a, b) << 32) | max(a, b))
    shadow = EdgeShadow(g)
    bd = Draws(sub_seed(seed, TAG_BATCH + 11), TAG_BATCH)
    reqs, at = [], 0
    for i in range(n_requests):
        ins = pool[at:at + int(n_ins[i])]
        at += int(n_ins[i])
        dels = shadow.sample_deletions(int(n_del[i]), bd, protect) if n_del[i] else np.zeros(0, np.uint64)
        shadow.add(ins)
        reqs.append(make_batch(ins, dels, bd))
    return Workload(name, g, queries, reqs, {"seed": seed, "gaps": gaps, "sizes": sizes})


def batched_queries(seed: int = 0, n_batches: int = 1, n_queries: int = 64, threads: int = 0,
                    query_min_label: int = BATCHED_QUERY_MIN_LABEL) -> Workload:
    """The mid graph with 64 standing queries (even ids sparse, odd ids
    dense, each with 4..12 vertices) and batches of 8,000 insertions and
    2,000 deletions.  The query walks visit only vertices of the rarer labels
    (>= query_min_label), as for the large workload.  Most sparse queries (a
    walk tree plus one cycle edge) of 9..12 vertices have 10^10 or more
    incremental matches per batch on this graph: under a per-query time
    limit they are the unsolved queries of Sec. VI-A."""
    spec = _batched_spec(seed, n_queries)
    return rmat_stream(20, 8 << 20, 16, 1.2, 8000, 2000, n_batches, spec, seed,
                       pool_batches=max(64, n_batches), name="batched-rmat20", threads=threads,
                       query_min_label=query_min_label)


# --------------------------------------------------------------------------
# small random instances for property tests


def random_small(seed: int, n: int = 10, p: float = 0.35, n_labels: int = 3, k: int = 3,
                 extra_q_edges: int = 1, n_ins: int = 3, n_del: int = 2, adversarial: bool = False):
    """A tiny random graph, a connected random query and a valid mixed batch.

    With adversarial=True the batch also holds duplicates, reversed
    duplicates and no-op updates (insert of a present edge, delete of an
    absent one)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = set()
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                edges.add((u, v))
    lo = np.array([e[0] for e in sorted(edges)], dtype=np.uint32)
    hi = np.array([e[1] for e in sorted(edges)], dtype=np.uint32)
    row_ptr, col = csr_from_edges(n, lo, hi, threads=1)
    labels = rng.integers(0, n_labels, size=n).astype(np.uint32)
    g = Graph(n, row_ptr, col, labels, "small")
    # connected query: random tree plus extra edges
    qe = set()
    for v in range(1, k):
        u = int(rng.integers(0, v))
        qe.add((u, v))
    tries = 0
    while len(qe) < min(k * (k - 1) // 2, k - 1 + extra_q_edges) and tries < 100:
        u, v = sorted(rng.choice(k, size=2, replace=False).tolist())
        qe.add((u, v))
        tries += 1
    qlab = rng.integers(0, n_labels, size=k).astype(np.uint32)
    q = Query(k, qlab, np.array(sorted(qe), dtype=np.uint32).reshape(-1, 2), "random")
    present = sorted(edges)
    absent = [(u, v) for u in range(n) for v in range(u + 1, n) if (u, v) not in edges]
    ins = [absent[i] for i in rng.permutation(len(absent))[: min(n_ins, len(absent))]]
    dels = [present[i] for i in rng.permutation(len(present))[: min(n_del, len(present))]]
    ups = [(u, v, 1) for (u, v) in ins] + [(u, v, 0) for (u, v) in dels]
    if adversarial:
        if ups:
            u, v, o = ups[0]
            ups.append((v, u, o))  # reversed duplicate
            ups.append((u, v, o))  # exact duplicate
        if dels:  # delete of an absent edge is a no-op only if absent: use an insert target
            pass
        rem = [e for e in absent if e not in ins]
        if rem:
            ups.append((rem[0][0], rem[0][1], 0))  # delete of absent edge: no-op
        keep = [e for e in present if e not in dels]
        if keep:
            ups.append((keep[0][1], keep[0][0], 1))  # insert of present edge: no-op
    order = rng.permutation(len(ups)) if ups else np.zeros(0, dtype=np.int64)
    ups = [ups[i] for i in order.tolist()]
    flip = rng.integers(0, 2, size=len(ups))
    src = np.array([(v if f else u) for (u, v, _), f in zip(ups, flip)], dtype=np.uint32)
    dst = np.array([(u if f else v) for (u, v, _), f in zip(ups, flip)], dtype=np.uint32)
    op = np.array([o for (_, _, o) in ups], dtype=np.uint8)
    return g, q, Batch(src, dst, op)


def graph_from_edges(n: int, edges: Sequence[Tuple[int, int]], labels: Sequence[int], name: str = "") -> Graph:
    lo = np.array([min(e) for e in edges], dtype=np.uint32)
    hi = np.array([max(e) for e in edges], dtype=np.uint32)
    row_ptr, col = csr_from_edges(n, lo, hi, threads=1)
    return Graph(n, row_ptr, col, np.array(labels, dtype=np.uint32), name)


def batch_from_list(ups: Sequence[Tuple[str, int, int]]) -> Batch:
    """[('+', u, v), ('-', u, v), ...] -> Batch."""
    src = np.array([u for (_, u, _) in ups], dtype=np.uint32)
    dst = np.array([v for (_, _, v) in ups], dtype=np.uint32)
    op = np.array([1 if s == "+" else 0 for (s, _, _) in ups], dtype=np.uint8)
    return Batch(src, dst, op)


def query_from_edges(k: int, edges: Sequence[Tuple[int, int]], labels: Sequence[int], kind: str = "",
                     elabels: Optional[Sequence[int]] = None) -> Query:
    return Query(k, np.array(labels, dtype=np.uint32), np.array(edges, dtype=np.uint32).reshape(-1, 2), kind,
                 elabels=None if elabels is None else np.array(elabels, dtype=np.uint32))


# --------------------------------------------------------------------------
# edge labels


def skewed_edge_label_draws(m: int, n_el: int, seed: int, skew: float = 1.0) -> np.ndarray:
    """m labels in [0, n_el) with P(e) proportional to 1 / (e + 1)^skew (a
    few frequent labels and a tail, as in edge-labelled graphs whose label
    counts are highly uneven)."""
    w = 1.0 / np.power(np.arange(1, n_el + 1, dtype=np.float64), skew)
    cdf = np.cumsum(w / w.sum())
    u = (Draws(seed, 0xE1AB).block(m) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return np.minimum(np.searchsorted(cdf, u, side="right"), n_el - 1).astype(np.uint32)


def with_edge_labels(g: Graph, n_el: int, seed: int, skew: float = 1.0) -> Graph:
    """g with one label per undirected edge (both CSR entries carry it)."""
    keys = g.edge_keys()
    lab = skewed_edge_label_draws(len(keys), n_el, seed, skew)
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr).astype(np.int64))
    dst = g.col.astype(np.uint64)
    ek = (np.minimum(src, dst) << np.uint64(32)) | np.maximum(src, dst)
    elab = lab[np.searchsorted(keys, ek)]
    return Graph(g.n, g.row_ptr, g.col, g.labels, g.name, elab=elab, n_elabels=n_el)


def pair_edge_labels(keys: np.ndarray, n_el: int, seed: int, skew: float = 1.0) -> np.ndarray:
    """A label for every vertex pair (key lo << 32 | hi), a function of the
    pair alone (splitmix64 of the key and seed, through the skewed
    distribution of skewed_edge_label_draws): an edge keeps its label across
    the graph, the batches that insert or delete it and a query planted on it."""
    w = 1.0 / np.power(np.arange(1, n_el + 1, dtype=np.float64), skew)
    cdf = np.cumsum(w / w.sum())
    z = np.asarray(keys, dtype=np.uint64) ^ np.uint64(sub_seed(seed, 0xE1AB))
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return np.minimum(np.searchsorted(cdf, u, side="right"), n_el - 1).astype(np.uint32)


def _pair_keys(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    return (np.minimum(a, b) << np.uint64(32)) | np.maximum(a, b)


def edge_labelled(seed: int = 0, n_batches: int = 1, n_el: int = 7, skew: float = 1.0, threads: int = 0) -> Workload:
    """The mid workload with edge labels: every pair carries one of n_el
    labels, skewed (a few frequent labels and a tail, like edge-labelled
    graphs with uneven label counts); batch updates carry their pair's
    label and the query's edges the labels of its planted match's edges."""
    w = mid(seed, n_batches=n_batches, threads=threads)
    g = w.graph
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr).astype(np.int64))
    g.elab = pair_edge_labels(_pair_keys(src, g.col), n_el, seed, skew)
    g.n_elabels = n_el
    for b in w.batches:
        b.elab = pair_edge_labels(_pair_keys(b.src, b.dst), n_el, seed, skew)
    for q in w.queries:
        pv = np.array(q.planted, dtype=np.uint64)
        q.elabels = pair_edge_labels(_pair_keys(pv[q.edges[:, 0]], pv[q.edges[:, 1]]), n_el, seed, skew)
    w.name = "elabel-rmat20"
    w.meta["n_elabels"] = n_el
    return w


def vertex_deletions(g: Graph, count: int, seed: int, exclude=(), by_degree: bool = False) -> np.ndarray:
    """`count` distinct vertices, uniformly (a removed account is a typical
    vertex) or, with by_degree, with probability proportional to degree + 1
    (on a power-law graph that picks hubs, whose deletion destroys most of
    the matches through them)."""
    d = Draws(sub_seed(seed, 0xDE1), 0xDE1)
    deg = np.diff(g.row_ptr).astype(np.float64) + 1.0 if by_degree else np.ones(g.n)
    cdf = np.cumsum(deg / deg.sum())
    out, seen = [], set(int(x) for x in exclude)
    while len(out) < count:
        u = float(d.u64() >> 11) * (1.0 / (1 << 53))
        v = int(min(np.searchsorted(cdf, u, side="right"), g.n - 1))
        if v not in seen:
            seen.add(v)
            out.append(v)
    return np.array(out, dtype=np.uint32)


def graph_from_labelled_edges(n: int, triples: Sequence[Tuple[int, int, int]], labels: Sequence[int],
                              n_el: int, name: str = "") -> Graph:
    """CSR of labelled edges (u, v, e); a pair may carry several labels.
    Rows ascend by (neighbour, label)."""
    ent = sorted({(a, b, e) for (u, v, e) in triples for (a, b) in ((u, v), (v, u))})
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    for (a, _, _) in ent:
        row_ptr[a + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.uint64)
    col = np.array([b for (_, b, _) in ent], dtype=np.uint32)
    elab = np.array([e for (_, _, e) in ent], dtype=np.uint32)
    return Graph(n, row_ptr, col, np.array(labels, dtype=np.uint32), name, elab=elab, n_elabels=n_el)


def fingerprint(arr: np.ndarray) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()
