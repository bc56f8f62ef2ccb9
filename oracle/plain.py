"""ctypes wrapper around O2 (oracle/plain.c).  TEST INFRASTRUCTURE: see the
package docstring for who may use it.

O2 follows Algorithm 1 (Sec. IV-C): seeds are the canonical batch edges, each
tried against both orientations of every query edge, extended along a BFS
matching order with label, injectivity and adjacency checks, and the order
rule (a batch edge with a lower ord than the seed is not usable) makes each
match come from exactly one seed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libo2.so")
_lib = None

MUT_NONE, MUT_NO_INJECTIVITY, MUT_ONE_ORIENTATION, MUT_NO_ORDER_RULE = 0, 1, 2, 3
MUT_DELETE_ON_GPRIME, MUT_SKIP_FIRST_CHECK, MUT_NO_LABEL_CHECK, MUT_KEEP_NOOPS = 4, 5, 6, 7
MUT_NO_EDGE_LABEL_CHECK = 8


class _Res(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("n_canonical", ctypes.c_uint32),
        ("n_insert", ctypes.c_uint32),
        ("n_delete", ctypes.c_uint32),
        ("n_noop", ctypes.c_uint32),
        ("n_dup", ctypes.c_uint32),
        ("count", ctypes.c_uint64 * 2),
        ("hsum", ctypes.c_uint64 * 2),
        ("hxor", ctypes.c_uint64 * 2),
        ("n_tuples", ctypes.c_uint64),
        ("tuples", ctypes.POINTER(ctypes.c_uint32)),
        ("tsign", ctypes.POINTER(ctypes.c_uint8)),
        ("tord", ctypes.POINTER(ctypes.c_uint32)),
        ("canon_lo", ctypes.POINTER(ctypes.c_uint32)),
        ("canon_hi", ctypes.POINTER(ctypes.c_uint32)),
        ("canon_sign", ctypes.POINTER(ctypes.c_uint8)),
        ("seed_count", ctypes.POINTER(ctypes.c_uint64)),
        ("seed_hsum", ctypes.POINTER(ctypes.c_uint64)),
        ("seed_hxor", ctypes.POINTER(ctypes.c_uint64)),
        ("seconds", ctypes.c_double),
        ("threads_used", ctypes.c_int32),
        ("canon_e", ctypes.POINTER(ctypes.c_uint32)),
        ("seed_incomplete", ctypes.POINTER(ctypes.c_uint8)),
        ("n_incomplete", ctypes.c_uint64),
        ("seconds_prep", ctypes.c_double),
    ]


def build_native(force: bool = False) -> str:
    """Compile O2 with gcc (plain C99 + pthreads)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-shared", "-fPIC",
                               os.path.join(_HERE, "plain.c"), "-o", tmp, "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        build_native(False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        u32 = ctypes.c_uint32
        lib.o2_run_el.restype = ctypes.c_int
        lib.o2_run_el.argtypes = [u32, P, P, P, u32, P, u32, u32, P, u32, P, P, u32, P, P, P, P, ctypes.c_int,
                                  u32, u32, ctypes.c_uint64, ctypes.c_uint64, P, u32, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(_Res)]
        lib.o2_free.restype = None
        lib.o2_free.argtypes = [ctypes.POINTER(_Res)]
        lib.o2_updated_graph_el.restype = ctypes.c_int
        lib.o2_updated_graph_el.argtypes = [u32, P, P, P, u32, u32, P, P, P, P,
                                            ctypes.POINTER(ctypes.POINTER(ctypes.c_uint64)),
                                            ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32)),
                                            ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32))]
        lib.o2_free_ptr.restype = None
        lib.o2_free_ptr.argtypes = [P]
        lib.o2_tuple_hash.restype = ctypes.c_uint64
        lib.o2_tuple_hash.argtypes = [ctypes.c_uint32, ctypes.c_int, P, ctypes.c_uint32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _arr(p, n, dtype):
    if n == 0 or not p:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(p, shape=(int(n),)).astype(dtype, copy=True)


@dataclass
class O2Result:
    status: int
    n_canonical: int
    n_insert: int
    n_delete: int
    n_noop: int
    n_dup: int
    count: tuple  # (deletions, insertions)
    hsum: tuple
    hxor: tuple
    tuples: Optional[np.ndarray]  # [n, k] uint32
    sign: Optional[np.ndarray]  # [n] uint8 (1 = insertion)
    ord: Optional[np.ndarray]  # [n] uint32
    canon_lo: np.ndarray
    canon_hi: np.ndarray
    canon_sign: np.ndarray
    canon_e: np.ndarray
    seed_count: np.ndarray
    seed_hsum: np.ndarray
    seed_hxor: np.ndarray
    seconds: float
    threads: int
    seed_incomplete: Optional[np.ndarray] = None  # [n_canonical] uint8: 1 = given up at the seed cap, 2 = scan cap
    n_incomplete: int = 0
    seconds_prep: float = 0.0  # the oracle's own graph update (keys, canonical batch, G')

    @property
    def seconds_search(self) -> float:
        return self.seconds - self.seconds_prep

    def tuple_set(self, sign: int) -> set:
        if self.tuples is None:
            raise ValueError("tuples were not requested")
        sel = self.tuples[self.sign == sign]
        return {tuple(int(x) for x in row) for row in sel}


def _labels_of(graph, query, batch):
    """(L, per-entry, per-query-edge, per-update edge labels or None): edge
    labels are optional attributes (elab, n_elabels; elabels; elab)."""
    ge = getattr(graph, "elab", None)
    L = int(getattr(graph, "n_elabels", 1) or 1)
    qe = getattr(query, "elabels", None) if query is not None else None
    be = getattr(batch, "elab", None)
    as32 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.uint32)
    return L, as32(ge), as32(qe), as32(be)


def _p(a):
    return None if a is None or a.size == 0 else _ptr(a)


def run(graph, query, batch, qid: int = 0, threads: int = 1, sample_mod: int = 1, sample_rem: int = 0,
        want_tuples: bool = True, mutant: int = MUT_NONE, seed_cap: int = 0, ords=None,
        scan_cap: int = 0) -> O2Result:
    """Run O2 on (graph, query, batch); graph/query/batch are workloads types
    (edge labels when they carry them).  seed_cap > 0 gives up every seed
    with more than seed_cap matches (flagged in seed_incomplete, left out of
    the totals and tuples); every other seed's figures are exact.  scan_cap
    > 0 likewise gives up a seed whose search examines more than scan_cap
    neighbour-list entries (flagged 2; its count is only a lower bound).  ords:
    only these canonical updates are searched (each with its full-batch
    figures)."""
    L = _L()
    n_el, gel, qel, bel = _labels_of(graph, query, batch)
    rp = np.ascontiguousarray(graph.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(graph.col, dtype=np.uint32)
    lab = np.ascontiguousarray(graph.labels, dtype=np.uint32)
    ql = np.ascontiguousarray(query.labels, dtype=np.uint32)
    qe = np.ascontiguousarray(query.edges, dtype=np.uint32).reshape(-1)
    src = np.ascontiguousarray(batch.src, dtype=np.uint32)
    dst = np.ascontiguousarray(batch.dst, dtype=np.uint32)
    op = np.ascontiguousarray(batch.op, dtype=np.uint8)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    if src.size == 0:
        src = np.zeros(1, np.uint32); dst = np.zeros(1, np.uint32); op = np.zeros(1, np.uint8)
        n_upd = 0
    else:
        n_upd = int(batch.src.shape[0])
    ord_arr = np.ascontiguousarray(np.asarray(ords, dtype=np.uint32)) if ords is not None else None
    r = _Res()
    rc = L.o2_run_el(graph.n, _ptr(rp), _ptr(col), _ptr(lab), n_el, _p(gel), qid, query.k, _ptr(ql), query.m,
                     _ptr(qe), _p(qel), n_upd, _ptr(src), _ptr(dst), _ptr(op), _p(bel) if n_upd else None,
                     int(threads), int(sample_mod), int(sample_rem), int(seed_cap), int(scan_cap),
                     _ptr(ord_arr) if ord_arr is not None else None, len(ord_arr) if ord_arr is not None else 0,
                     1 if want_tuples else 0, int(mutant), ctypes.byref(r))
    if rc == -3:
        raise ValueError("query rejected by the oracle (k, edges or connectivity)")
    k = query.k
    nt = int(r.n_tuples)
    out = O2Result(
        status=int(r.status), n_canonical=int(r.n_canonical), n_insert=int(r.n_insert),
        n_delete=int(r.n_delete), n_noop=int(r.n_noop), n_dup=int(r.n_dup),
        count=(int(r.count[0]), int(r.count[1])), hsum=(int(r.hsum[0]), int(r.hsum[1])),
        hxor=(int(r.hxor[0]), int(r.hxor[1])),
        tuples=(_arr(r.tuples, nt * k, np.uint32).reshape(nt, k) if want_tuples and rc == 0 else None),
        sign=(_arr(r.tsign, nt, np.uint8) if want_tuples and rc == 0 else None),
        ord=(_arr(r.tord, nt, np.uint32) if want_tuples and rc == 0 else None),
        canon_lo=_arr(r.canon_lo, r.n_canonical, np.uint32), canon_hi=_arr(r.canon_hi, r.n_canonical, np.uint32),
        canon_sign=_arr(r.canon_sign, r.n_canonical, np.uint8),
        canon_e=_arr(r.canon_e, r.n_canonical, np.uint32),
        seed_count=_arr(r.seed_count, r.n_canonical, np.uint64),
        seed_hsum=_arr(r.seed_hsum, r.n_canonical, np.uint64),
        seed_hxor=_arr(r.seed_hxor, r.n_canonical, np.uint64),
        seconds=float(r.seconds), threads=int(r.threads_used),
        seed_incomplete=_arr(r.seed_incomplete, r.n_canonical, np.uint8), n_incomplete=int(r.n_incomplete),
        seconds_prep=float(r.seconds_prep))
    if rc == 0:
        L.o2_free(ctypes.byref(r))
    return out


def updated_graph_el(graph, batch):
    """G' after applying `batch` (canonical semantics), as (row_ptr, col,
    elab); rows ascending by (neighbour, edge label)."""
    L = _L()
    n_el, gel, _, bel = _labels_of(graph, None, batch)
    rp = np.ascontiguousarray(graph.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(graph.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    src = np.ascontiguousarray(batch.src, dtype=np.uint32)
    dst = np.ascontiguousarray(batch.dst, dtype=np.uint32)
    op = np.ascontiguousarray(batch.op, dtype=np.uint8)
    n_upd = int(src.shape[0])
    if n_upd == 0:
        src = np.zeros(1, np.uint32); dst = np.zeros(1, np.uint32); op = np.zeros(1, np.uint8)
    prp = ctypes.POINTER(ctypes.c_uint64)()
    pcol = ctypes.POINTER(ctypes.c_uint32)()
    pel = ctypes.POINTER(ctypes.c_uint32)()
    rc = L.o2_updated_graph_el(graph.n, _ptr(rp), _ptr(col), _p(gel), n_el, n_upd, _ptr(src), _ptr(dst), _ptr(op),
                               _p(bel) if n_upd else None, ctypes.byref(prp), ctypes.byref(pcol), ctypes.byref(pel))
    if rc != 0:
        raise ValueError("invalid batch (status %d)" % rc)
    row_ptr = _arr(prp, graph.n + 1, np.uint64)
    nnz = int(row_ptr[-1])
    c = _arr(pcol, nnz, np.uint32)
    el = _arr(pel, nnz, np.uint32)
    for p in (prp, pcol, pel):
        L.o2_free_ptr(ctypes.cast(p, ctypes.c_void_p))
    return row_ptr, c, el


def updated_graph(graph, batch):
    """G' after applying `batch` (canonical semantics), as (row_ptr, col)."""
    rp, col, _ = updated_graph_el(graph, batch)
    return rp, col


def tuple_hash(qid: int, sign: int, f) -> int:
    a = np.ascontiguousarray(np.array(f, dtype=np.uint32))
    return int(_L().o2_tuple_hash(qid, sign, _ptr(a), len(f)))
