"""MI355X-native batch-dynamic subgraph matching (GAMMA, arXiv 2401.17018).

Python binding over the C ABI of libgamma.so (include/gamma.h).  The binding
only marshals arguments: graph loading, batch canonicalisation, the graph
update, the candidate filter, seeding, the search and the commit all run in
the library's HIP kernels on the GPU.  Inputs may be numpy arrays (host
memory) or torch tensors on the context's device; torch is used for device
memory and streams only.  To pass torch tensors, import torch (and touch
its GPU) before the first Context: torch ships its own libamdhip64.so.7,
the library then shares that runtime; loaded the other way round, torch's
GPU initialisation fails in the process.

    ctx = Context(device=0)
    ctx.load_graph(row_ptr, col, labels)
    qid = ctx.register_query(k, qlabels, qedges)
    res = ctx.apply_batch(src, dst, op, tuples=True)
    res.count(qid, +1), res.tuples
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import capi
from .capi import (F_CANONICAL, F_COUNT, F_DRY_RUN, F_HASH, F_PER_UPDATE, F_SEED_ATTR, F_TUPLES,
                   GAMMA_MEM_DEVICE, GAMMA_MEM_HOST)

__all__ = ["Context", "Server", "GammaError", "BatchOutput", "validate_graph", "validate_query", "validate_batch",
           "describe_query"]


class GammaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d)" % (message, status))
        self.status = status


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _arg(x, dtype):
    """(pointer, keepalive, where) for a numpy array or a torch tensor."""
    if x is None:
        return None, None, GAMMA_MEM_HOST
    if _is_torch(x):
        if x.is_cuda:
            t = x.contiguous()
            return ctypes.c_void_p(t.data_ptr()), t, GAMMA_MEM_DEVICE
        x = x.cpu().numpy()
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), a, GAMMA_MEM_HOST


def _check(lib, ctx_ptr, st: int, what: str):
    if st < 0:
        msg = lib.gamma_last_error(ctx_ptr) if ctx_ptr else lib.gamma_status_string(st)
        raise GammaError(st, "%s: %s" % (what, (msg or b"").decode()))
    return st


@dataclass
class BatchOutput:
    status: int
    counts: np.ndarray        # [n_queries, 2] (index 1 = insertion results, 0 = deletion results)
    hash_sum: np.ndarray      # [n_queries, 2]
    hash_xor: np.ndarray      # [n_queries, 2]
    n_tuples: int
    n_tuples_found: int
    tuples: Optional[np.ndarray] = None   # [n_tuples, width] external ids, 0xFFFFFFFF padded
    meta: Optional[np.ndarray] = None     # [n_tuples] qid << 1 | sign
    ord: Optional[np.ndarray] = None      # [n_tuples] seed ord
    canon_lo: Optional[np.ndarray] = None
    canon_hi: Optional[np.ndarray] = None
    canon_sign: Optional[np.ndarray] = None
    upd_count: Optional[np.ndarray] = None
    upd_hash_sum: Optional[np.ndarray] = None
    upd_hash_xor: Optional[np.ndarray] = None
    upd_open: Optional[np.ndarray] = None  # [n_canonical] uint8: 1 = search work of that update did not finish
    open_seeds: Optional[np.ndarray] = None  # [n_queries]: seeds left unfinished (tracked under a deadline)
    stats: dict = field(default_factory=dict)

    @property
    def truncated(self) -> bool:
        return self.status == capi.GAMMA_TRUNCATED

    def count(self, qid: int, sign: int) -> int:
        return int(self.counts[qid, 1 if sign > 0 else 0])

    def tuple_set(self, qid: int, sign: int, k: int) -> set:
        """Set of match tuples of one query and sign (requires tuples=True)."""
        if self.tuples is None:
            raise ValueError("tuples were not requested")
        sel = self.meta == ((qid << 1) | (1 if sign > 0 else 0))
        rows = self.tuples[sel][:, :k]
        return {tuple(int(v) for v in r) for r in rows}


class Context:
    """A device context holding one dynamic data graph and its standing queries."""

    def __init__(self, device: int = 0, stream=None, tuple_capacity: int = 0, waves_per_cu: int = 0,
                 steal: Optional[bool] = None, deadline_ms: int = 0):
        self._lib = capi.load_library()
        opt = capi.Options()
        opt.device = device
        if stream is not None:
            opt.stream = ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))
        opt.tuple_capacity = int(tuple_capacity)
        opt.waves_per_cu = int(waves_per_cu)
        if steal is not None:
            opt.steal = 1 if steal else 0
            opt.steal_set = 1
        opt.deadline_ms = int(deadline_ms)
        self._ptr = ctypes.c_void_p()
        st = self._lib.gamma_create(ctypes.byref(opt), ctypes.byref(self._ptr))
        if st < 0:
            raise GammaError(st, "gamma_create: %s" % self._lib.gamma_status_string(st).decode())
        self.tuple_capacity = int(tuple_capacity)
        self.query_k: List[int] = []
        self._sig = hashlib.sha256()  # graph and query shapes, for the tuning cache key

    def close(self):
        if getattr(self, "_ptr", None):
            self._lib.gamma_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ calls

    def load_graph(self, row_ptr, col, labels, elabels=None, n_elabels: int = 0):
        """Load a CSR graph; elabels (one per CSR entry, < n_elabels; default
        max + 1) makes it edge-labelled (gamma_load_graph_el)."""
        rp, k1, w1 = _arg(row_ptr, np.uint64)
        cl, k2, w2 = _arg(col, np.uint32)
        lb, k3, w3 = _arg(labels, np.uint32)
        ws = {w1, w2, w3}
        if elabels is not None:
            el, k4, w4 = _arg(elabels, np.uint32)
            ws.add(w4)
        if len(ws) != 1:
            raise ValueError("row_ptr, col, labels (and elabels) must all be host arrays or all device tensors")
        n = int(k3.shape[0])
        nnz = int(k2.shape[0])
        if elabels is None:
            _check(self._lib, self._ptr,
                   self._lib.gamma_load_graph(self._ptr, n, nnz, rp, cl if nnz else None, lb, w1), "load_graph")
        else:
            if not n_elabels:
                n_elabels = int(np.asarray(k4).max()) + 1 if nnz else 1
            _check(self._lib, self._ptr,
                   self._lib.gamma_load_graph_el(self._ptr, n, nnz, rp, cl if nnz else None, lb, el if nnz else None,
                                                 int(n_elabels), w1), "load_graph")
        self._sig = hashlib.sha256(b"graph n=%d nnz=%d el=%d" % (n, nnz, int(n_elabels or 1)))
        for q in getattr(self, "_queries", []):
            self._sig.update(q)

    def register_query(self, k: int, labels, edges, elabels=None) -> int:
        """Register a standing query; elabels: one label per edge."""
        ql = np.ascontiguousarray(np.asarray(labels), dtype=np.uint32)
        qe = np.ascontiguousarray(np.asarray(edges), dtype=np.uint32).reshape(-1)
        qel = None if elabels is None else np.ascontiguousarray(np.asarray(elabels), dtype=np.uint32)
        qid = ctypes.c_uint32()
        _check(self._lib, self._ptr,
               self._lib.gamma_register_query_el(self._ptr, int(k), ql.ctypes.data_as(ctypes.c_void_p),
                                                 int(qe.shape[0] // 2), qe.ctypes.data_as(ctypes.c_void_p),
                                                 qel.ctypes.data_as(ctypes.c_void_p) if qel is not None else None,
                                                 ctypes.byref(qid)),
               "register_query")
        self.query_k.append(int(k))
        qsig = b"query k=%d " % int(k) + ql.tobytes() + qe.tobytes() + (qel.tobytes() if qel is not None else b"")
        self._queries = getattr(self, "_queries", []) + [qsig]
        self._sig.update(qsig)
        return int(qid.value)

    def apply_batch(self, src, dst, op, hash: bool = True, tuples: bool = False, seed_attr: bool = False,
                    per_update: bool = False, canonical: bool = False, dry_run: bool = False,
                    delete_vertices=None, elab=None, noalloc: bool = False) -> BatchOutput:
        """Apply one batch (dry_run: search it without committing it).

        noalloc: through gamma_apply_batch_noalloc, which allocates no device
        memory (counts, checksums and attribution only; no edge labels or
        vertex deletions).
        delete_vertices: ids whose incident edges are all deleted in the same
        batch, appended after the explicit updates (gamma_apply_batch_vertices).
        elab: the edge label of each update (edge-labelled graphs)."""
        s, k1, w1 = _arg(src, np.uint32)
        d, k2, w2 = _arg(dst, np.uint32)
        o, k3, w3 = _arg(op, np.uint8)
        ws = {w1, w2, w3}
        el = None
        if elab is not None:
            el, k5, w5 = _arg(elab, np.uint32)
            ws.add(w5)
        if delete_vertices is not None:
            vd, k4, w4 = _arg(delete_vertices, np.uint32)
            ws.add(w4)
        if len(ws) != 1:
            raise ValueError("src, dst, op (and delete_vertices) must all be host arrays or all device tensors")
        n_upd = int(k1.shape[0])
        flags = F_COUNT
        flags |= F_HASH if hash else 0
        flags |= F_TUPLES if tuples else 0
        flags |= F_SEED_ATTR if seed_attr else 0
        flags |= F_PER_UPDATE if per_update else 0
        flags |= F_CANONICAL if canonical else 0
        flags |= F_DRY_RUN if dry_run else 0
        res = capi.BatchResult()
        if noalloc:
            if delete_vertices is not None or elab is not None:
                raise ValueError("noalloc takes plain edge updates only")
            st = self._lib.gamma_apply_batch_noalloc(self._ptr, n_upd, s if n_upd else None, d if n_upd else None,
                                                     o if n_upd else None, w1, flags, ctypes.byref(res))
        elif delete_vertices is None:
            st = self._lib.gamma_apply_batch_el(self._ptr, n_upd, s if n_upd else None, d if n_upd else None,
                                                o if n_upd else None, el if n_upd else None, w1, flags,
                                                ctypes.byref(res))
        else:
            nv = int(k4.shape[0])
            st = self._lib.gamma_apply_batch_vertices(self._ptr, n_upd, s if n_upd else None, d if n_upd else None,
                                                      o if n_upd else None, el if n_upd else None, nv,
                                                      vd if nv else None, w1, flags, ctypes.byref(res))
        if st == capi.GAMMA_ETIMEDOUT:
            err = GammaError(st, "apply_batch: %s" % (self._lib.gamma_last_error(self._ptr) or b"").decode())
            err.stats = {name: getattr(res.stats, name) for name, _ in capi.BatchStats._fields_
                         if not name.startswith("reserved")}
            err.counts = [[res.queries[i].count[sg] for sg in range(2)] for i in range(int(res.n_queries))]
            err.hash_sum = [[res.queries[i].hash_sum[sg] for sg in range(2)] for i in range(int(res.n_queries))]
            err.hash_xor = [[res.queries[i].hash_xor[sg] for sg in range(2)] for i in range(int(res.n_queries))]
            # per query: seeds left unfinished (0 = solved: its figures are exact)
            err.open_seeds = np.array([res.queries[i].open_seeds for i in range(int(res.n_queries))], dtype=np.uint64)
            nc = int(res.n_canonical)
            if per_update and nc and res.upd_count:
                # partial attribution: updates whose search finished (upd_open 0) are exact
                err.upd_count = np.ctypeslib.as_array(res.upd_count, (nc,)).copy()
                err.upd_hash_sum = np.ctypeslib.as_array(res.upd_hash_sum, (nc,)).copy()
                err.upd_hash_xor = np.ctypeslib.as_array(res.upd_hash_xor, (nc,)).copy()
                err.upd_open = np.ctypeslib.as_array(res.upd_open, (nc,)).copy()
            raise err
        _check(self._lib, self._ptr, st, "apply_batch")
        nq = int(res.n_queries)
        counts = np.zeros((nq, 2), dtype=np.uint64)
        hs = np.zeros((nq, 2), dtype=np.uint64)
        hx = np.zeros((nq, 2), dtype=np.uint64)
        op_ = np.zeros(nq, dtype=np.uint64)
        for i in range(nq):
            q = res.queries[i]
            op_[i] = q.open_seeds
            for sg in range(2):
                counts[i, sg] = q.count[sg]
                hs[i, sg] = q.hash_sum[sg]
                hx[i, sg] = q.hash_xor[sg]
        out = BatchOutput(status=int(st), counts=counts, hash_sum=hs, hash_xor=hx, n_tuples=int(res.n_tuples),
                          n_tuples_found=int(res.n_tuples_found))
        out.open_seeds = op_
        nc = int(res.n_canonical)
        if canonical and nc:
            out.canon_lo = np.ctypeslib.as_array(res.canon_lo, (nc,)).copy()
            out.canon_hi = np.ctypeslib.as_array(res.canon_hi, (nc,)).copy()
            out.canon_sign = np.ctypeslib.as_array(res.canon_sign, (nc,)).copy()
        elif canonical:
            out.canon_lo = np.zeros(0, np.uint32)
            out.canon_hi = np.zeros(0, np.uint32)
            out.canon_sign = np.zeros(0, np.uint8)
        if per_update:
            if nc:
                out.upd_count = np.ctypeslib.as_array(res.upd_count, (nc,)).copy()
                out.upd_hash_sum = np.ctypeslib.as_array(res.upd_hash_sum, (nc,)).copy()
                out.upd_hash_xor = np.ctypeslib.as_array(res.upd_hash_xor, (nc,)).copy()
                out.upd_open = np.ctypeslib.as_array(res.upd_open, (nc,)).copy()
            else:
                out.upd_count = out.upd_hash_sum = out.upd_hash_xor = np.zeros(0, np.uint64)
                out.upd_open = np.zeros(0, np.uint8)
        if tuples:
            nt, w = int(res.n_tuples), int(res.tuple_width)
            t = np.zeros((nt, w), dtype=np.uint32)
            m = np.zeros(nt, dtype=np.uint32)
            od = np.zeros(nt, dtype=np.uint32) if seed_attr else None
            if nt:
                _check(self._lib, self._ptr,
                       self._lib.gamma_copy_tuples(self._ptr, t.ctypes.data_as(ctypes.c_void_p),
                                                   m.ctypes.data_as(ctypes.c_void_p),
                                                   od.ctypes.data_as(ctypes.c_void_p) if od is not None else None,
                                                   nt, GAMMA_MEM_HOST),
                       "copy_tuples")
            out.tuples, out.meta, out.ord = t, m, od
        stt = res.stats
        out.stats = {name: getattr(stt, name) for name, _ in capi.BatchStats._fields_ if not name.startswith("reserved")}
        return out

    def add_vertices(self, labels) -> int:
        """Append isolated vertices with these labels; returns the first new id."""
        lab = np.ascontiguousarray(np.asarray(labels, dtype=np.uint32))
        first = ctypes.c_uint32(0)
        _check(self._lib, self._ptr,
               self._lib.gamma_add_vertices(self._ptr, int(lab.shape[0]),
                                            lab.ctypes.data_as(ctypes.c_void_p) if lab.size else None,
                                            ctypes.byref(first)),
               "add_vertices")
        return int(first.value)

    # ------------------------------------------------------------ tuning

    def get_tuning(self) -> dict:
        t = capi.Tuning()
        _check(self._lib, self._ptr, self._lib.gamma_get_tuning(self._ptr, ctypes.byref(t)), "get_tuning")
        return t.as_dict()

    def set_deadline(self, ms: int) -> None:
        """Search deadline of later batches in ms (0 = none).  With
        query_launch = 2 each query's search gets this time on its own; a
        query that passes it is unsolved (open_seeds > 0) and the batch
        raises GammaError(GAMMA_ETIMEDOUT) without being committed."""
        _check(self._lib, self._ptr, self._lib.gamma_set_deadline(self._ptr, int(ms)), "set_deadline")

    def set_query_active(self, qid: int, active: bool) -> None:
        """Pause or resume a standing query (a paused query is kept current
        but not searched; its results are 0)."""
        _check(self._lib, self._ptr, self._lib.gamma_set_query_active(self._ptr, int(qid), 1 if active else 0),
               "set_query_active")

    def set_tuning(self, **kw) -> dict:
        """Set search tunables (waves_per_cu, steal 1/2, poll_cycles, split_inner,
        split_leaf, query_launch 1/2, handover_gate, coalesced_search 1 off / 2
        whole-query automorphisms / 3 also symmetric cores, group_seeds 1 generation
        order / 2 sorted by first data vertex / 3 grouped by (query, directed query
        edge, first data vertex) with level 2's list built once per group);
        unnamed ones keep their value.  No tunable changes results."""
        t = capi.Tuning()
        for name, v in kw.items():
            if name not in capi.Tuning.FIELDS:
                raise ValueError("unknown tunable %r" % name)
            setattr(t, name, int(v))
        _check(self._lib, self._ptr, self._lib.gamma_set_tuning(self._ptr, ctypes.byref(t)), "set_tuning")
        return self.get_tuning()

    def tuning_key(self, n_updates: int) -> str:
        """Cache key: graph size, registered queries and the batch size's power of two."""
        return "%s:b%d" % (self._sig.hexdigest()[:24], max(int(n_updates), 1).bit_length())

    def autotune(self, src, dst, op, hash: bool = True, max_points: int = 40, reps: int = 3,
                 cache: Optional[str] = None) -> dict:
        """Tune the search on a calibration batch (dry runs, graph unchanged)
        and apply the best point.  With `cache` (a JSON file) a point stored
        for the same graph, queries and batch-size class is reused."""
        key = self.tuning_key(len(np.asarray(src)) if not _is_torch(src) else int(src.shape[0]))
        db = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
            if key in db:
                self.set_tuning(**db[key]["tuning"])
                return dict(db[key], key=key, from_cache=True)
        s, k1, w1 = _arg(src, np.uint32)
        d, k2, w2 = _arg(dst, np.uint32)
        o, k3, w3 = _arg(op, np.uint8)
        if len({w1, w2, w3}) != 1:
            raise ValueError("src, dst and op must all be host arrays or all device tensors")
        n_upd = int(k1.shape[0])
        best = capi.Tuning()
        best_ms, base_ms = ctypes.c_double(), ctypes.c_double()
        flags = F_COUNT | (F_HASH if hash else 0)
        _check(self._lib, self._ptr,
               self._lib.gamma_autotune(self._ptr, n_upd, s if n_upd else None, d if n_upd else None,
                                        o if n_upd else None, w1, flags, int(max_points), int(reps),
                                        ctypes.byref(best), ctypes.byref(best_ms), ctypes.byref(base_ms)),
               "autotune")
        entry = {"tuning": best.as_dict(), "best_ms": best_ms.value, "base_ms": base_ms.value,
                 "max_points": int(max_points), "reps": int(reps), "n_updates": n_upd}
        if cache:
            db[key] = entry
            tmp = "%s.tmp%d" % (cache, os.getpid())
            with open(tmp, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(entry, key=key, from_cache=False)

    def export_graph(self):
        n = ctypes.c_uint32()
        nnz = ctypes.c_uint64()
        _check(self._lib, self._ptr,
               self._lib.gamma_export_graph(self._ptr, ctypes.byref(n), ctypes.byref(nnz), None, None, None),
               "export_graph")
        rp = np.zeros(n.value + 1, dtype=np.uint64)
        col = np.zeros(max(nnz.value, 1), dtype=np.uint32)
        lab = np.zeros(n.value, dtype=np.uint32)
        _check(self._lib, self._ptr,
               self._lib.gamma_export_graph(self._ptr, ctypes.byref(n), ctypes.byref(nnz),
                                            rp.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p),
                                            lab.ctypes.data_as(ctypes.c_void_p)),
               "export_graph")
        return rp, col[: nnz.value], lab

    def export_graph_el(self):
        """(row_ptr, col, labels, elabels, n_elabels) of the current graph."""
        n, nnz, nel = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
        _check(self._lib, self._ptr,
               self._lib.gamma_export_graph_el(self._ptr, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(nel),
                                               None, None, None, None), "export_graph")
        rp = np.zeros(n.value + 1, dtype=np.uint64)
        col = np.zeros(max(nnz.value, 1), dtype=np.uint32)
        el = np.zeros(max(nnz.value, 1), dtype=np.uint32)
        lab = np.zeros(n.value, dtype=np.uint32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(self._lib, self._ptr,
               self._lib.gamma_export_graph_el(self._ptr, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(nel),
                                               ptr(rp), ptr(col), ptr(lab), ptr(el)), "export_graph")
        return rp, col[: nnz.value], lab, el[: nnz.value], int(nel.value)


class Server:
    """A served update stream on a Context (continuous batching by the
    library's worker thread).  While it exists, use the context only
    through it."""

    def __init__(self, ctx: Context, max_batch_updates: int = 0, hash: bool = True, per_update: bool = False,
                 coalesce: bool = True, tuples: bool = False, seed_attr: bool = False, tuple_fill_pct: int = 0,
                 max_batch_ms: int = 0):
        """tuples: keep every batch's match records (the context needs a
        tuple_capacity); admission then also bounds a batch's estimated
        records by tuple_fill_pct of that capacity.  max_batch_ms: admission
        also bounds a batch's estimated device time (0 = no bound)."""
        self._lib = ctx._lib
        self.ctx = ctx
        o = capi.ServeOptions()
        o.max_batch_updates = int(max_batch_updates)
        o.flags = (F_COUNT | (F_HASH if hash else 0) | (F_PER_UPDATE if per_update else 0) |
                   (F_TUPLES if tuples else 0) | (F_SEED_ATTR if tuples and seed_attr else 0))
        o.coalesce = 1 if coalesce else 2
        o.tuple_fill_pct = int(tuple_fill_pct)
        o.max_batch_ms = int(max_batch_ms)
        self._ptr = ctypes.c_void_p()
        _check(self._lib, ctx._ptr, self._lib.gamma_serve_create(ctx._ptr, ctypes.byref(o), ctypes.byref(self._ptr)),
               "serve_create")
        self.n_queries = len(ctx.query_k)

    def submit(self, src, dst, op, elab=None) -> int:
        """Queue one request; elab: its edge labels (edge-labelled graphs)."""
        s = np.ascontiguousarray(src, dtype=np.uint32)
        d = np.ascontiguousarray(dst, dtype=np.uint32)
        o = np.ascontiguousarray(op, dtype=np.uint8)
        e = None if elab is None else np.ascontiguousarray(elab, dtype=np.uint32)
        t = ctypes.c_uint64()
        st = self._lib.gamma_serve_submit_el(self._ptr, int(s.shape[0]), s.ctypes.data_as(ctypes.c_void_p),
                                             d.ctypes.data_as(ctypes.c_void_p), o.ctypes.data_as(ctypes.c_void_p),
                                             e.ctypes.data_as(ctypes.c_void_p) if e is not None else None,
                                             ctypes.byref(t))
        if st < 0:
            raise GammaError(st, "serve_submit: %s" % self._lib.gamma_status_string(st).decode())
        return int(t.value)

    def tuples(self, batch: int):
        """(tuples [n, width] uint32, meta [n], ord [n] or None) of a served batch."""
        n, w = ctypes.c_uint64(), ctypes.c_uint32()
        _check(self._lib, None, self._lib.gamma_serve_get_tuples(self._ptr, int(batch), None, None, None, 0,
                                                                 ctypes.byref(n), ctypes.byref(w)), "serve_get_tuples")
        t = np.zeros((n.value, w.value), np.uint32)
        m = np.zeros(n.value, np.uint32)
        o = np.zeros(n.value, np.uint32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
        _check(self._lib, None, self._lib.gamma_serve_get_tuples(self._ptr, int(batch), ptr(t), ptr(m), ptr(o), n.value,
                                                                 ctypes.byref(n), ctypes.byref(w)), "serve_get_tuples")
        return t, m, o

    def poll(self, max_results: int = 1024) -> List[dict]:
        buf = (capi.RequestResult * max_results)()
        n = ctypes.c_uint32()
        _check(self._lib, None, self._lib.gamma_serve_poll(self._ptr, buf, max_results, ctypes.byref(n)), "serve_poll")
        return [{f: getattr(buf[i], f) for f, _ in capi.RequestResult._fields_} for i in range(n.value)]

    def drain(self):
        _check(self._lib, None, self._lib.gamma_serve_drain(self._ptr), "serve_drain")

    def counts(self):
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(self._lib, None, self._lib.gamma_serve_counts(self._ptr, ctypes.byref(a), ctypes.byref(b),
                                                             ctypes.byref(c)), "serve_counts")
        return int(a.value), int(b.value), int(c.value)

    def batch(self, i: int) -> dict:
        info = capi.ServeBatch()
        qs = (capi.QueryResult * max(self.n_queries, 1))()
        _check(self._lib, None, self._lib.gamma_serve_get_batch(self._ptr, int(i), ctypes.byref(info), qs,
                                                                self.n_queries), "serve_get_batch")
        d = {f: getattr(info, f) for f, _ in capi.ServeBatch._fields_}
        d["counts"] = np.array([[qs[q].count[sg] for sg in range(2)] for q in range(info.n_queries)], np.uint64)
        d["hash_sum"] = np.array([[qs[q].hash_sum[sg] for sg in range(2)] for q in range(info.n_queries)], np.uint64)
        d["hash_xor"] = np.array([[qs[q].hash_xor[sg] for sg in range(2)] for q in range(info.n_queries)], np.uint64)
        return d

    def close(self):
        if getattr(self, "_ptr", None):
            self._lib.gamma_serve_destroy(self._ptr)
            self._ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate_graph(row_ptr, col, labels) -> int:
    lib = capi.load_library()
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    cl = np.ascontiguousarray(col, dtype=np.uint32)
    lb = np.ascontiguousarray(labels, dtype=np.uint32)
    return int(lib.gamma_validate_graph(int(lb.shape[0]), int(cl.shape[0]), rp.ctypes.data_as(ctypes.c_void_p),
                                        cl.ctypes.data_as(ctypes.c_void_p), lb.ctypes.data_as(ctypes.c_void_p)))


def describe_query(k, labels, edges, elabels=None):
    """The matching plans registration builds for a query (host only; see
    gamma_describe_query): a list of per-directed-edge dicts (x, y, order,
    n_perm, perm_first, n_core, n_cperm, cperm_first, omask) and the
    permutations as a [n, 16] array of forward maps.  Raises GammaError on an
    invalid query."""
    lib = capi.load_library()
    ql = np.ascontiguousarray(labels, dtype=np.uint32)
    qe = np.ascontiguousarray(edges, dtype=np.uint32).reshape(-1)
    m = qe.shape[0] // 2
    el = None if elabels is None else np.ascontiguousarray(elabels, dtype=np.uint32)
    cap_p, cap_g = 2 * m, 64
    while True:
        pi = (capi.PlanInfo * max(cap_p, 1))()
        perms = np.zeros((max(cap_g, 1), 16), np.uint32)
        n_p, n_g = ctypes.c_uint32(0), ctypes.c_uint32(0)
        st = lib.gamma_describe_query(int(k), ql.ctypes.data_as(ctypes.c_void_p), int(m),
                                      qe.ctypes.data_as(ctypes.c_void_p),
                                      None if el is None else el.ctypes.data_as(ctypes.c_void_p),
                                      cap_p, pi, ctypes.byref(n_p), cap_g, perms.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(n_g))
        if st == capi.GAMMA_EINVAL and (n_p.value > cap_p or n_g.value > cap_g):
            cap_p, cap_g = max(cap_p, n_p.value), max(cap_g, n_g.value)
            continue
        if st != 0:
            raise GammaError(st, "describe_query: invalid query")
        break
    plans = []
    for i in range(n_p.value):
        r = pi[i]
        plans.append(dict(x=r.x, y=r.y, n_perm=r.n_perm, perm_first=r.perm_first, n_core=r.n_core,
                          n_cperm=r.n_cperm, cperm_first=r.cperm_first, order=list(r.order)[:int(k)],
                          omask=list(r.omask)[:int(k)]))
    return plans, perms[:n_g.value].copy()


def validate_query(k, labels, edges) -> int:
    lib = capi.load_library()
    ql = np.ascontiguousarray(labels, dtype=np.uint32)
    qe = np.ascontiguousarray(edges, dtype=np.uint32).reshape(-1)
    return int(lib.gamma_validate_query(int(k), ql.ctypes.data_as(ctypes.c_void_p), int(qe.shape[0] // 2),
                                        qe.ctypes.data_as(ctypes.c_void_p)))


def validate_batch(n, src, dst, op) -> int:
    lib = capi.load_library()
    s = np.ascontiguousarray(src, dtype=np.uint32)
    d = np.ascontiguousarray(dst, dtype=np.uint32)
    o = np.ascontiguousarray(op, dtype=np.uint8)
    return int(lib.gamma_validate_batch(int(n), int(s.shape[0]), s.ctypes.data_as(ctypes.c_void_p),
                                        d.ctypes.data_as(ctypes.c_void_p), o.ctypes.data_as(ctypes.c_void_p)))
