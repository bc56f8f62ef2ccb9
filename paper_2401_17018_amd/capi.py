"""ctypes declarations of the C ABI in include/gamma.h (argument marshalling only).

The shared library is built in-tree (paper_2401_17018_amd/libgamma.so) by
``paper_2401_17018_amd.build``.  There is no fallback: if the library is
missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgamma.so")

GAMMA_OK, GAMMA_TRUNCATED = 0, 1
GAMMA_EINVAL, GAMMA_ECONFLICT, GAMMA_ENOMEM, GAMMA_EUNSUPPORTED = -1, -2, -3, -4
GAMMA_ESTATE, GAMMA_ETIMEDOUT, GAMMA_EDEVICE = -5, -6, -7

GAMMA_MEM_HOST, GAMMA_MEM_DEVICE = 0, 1

F_COUNT, F_HASH, F_TUPLES, F_SEED_ATTR, F_PER_UPDATE, F_CANONICAL, F_DRY_RUN = 1, 2, 4, 8, 16, 32, 64

# every function declared in include/gamma.h
EXPORTS = [
    "gamma_create", "gamma_destroy", "gamma_load_graph", "gamma_register_query", "gamma_apply_batch",
    "gamma_load_graph_el", "gamma_register_query_el", "gamma_apply_batch_el", "gamma_export_graph_el",
    "gamma_apply_batch_vertices", "gamma_apply_batch_noalloc", "gamma_add_vertices", "gamma_get_tuning", "gamma_set_tuning", "gamma_set_deadline", "gamma_set_query_active", "gamma_autotune",
    "gamma_serve_create", "gamma_serve_submit", "gamma_serve_submit_el", "gamma_serve_poll", "gamma_serve_drain", "gamma_serve_counts",
    "gamma_serve_get_batch", "gamma_serve_get_tuples", "gamma_serve_destroy",
    "gamma_copy_tuples", "gamma_result_release", "gamma_export_graph", "gamma_validate_graph",
    "gamma_validate_query", "gamma_validate_batch", "gamma_validate_graph_el", "gamma_validate_batch_el", "gamma_status_string", "gamma_last_error",
    "gamma_describe_query",
    "gamma_version",
]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("x", "y", "n_perm", "perm_first", "n_core", "n_cperm",
                                                 "cperm_first", "reserved")] + [
        ("order", ctypes.c_uint32 * 16), ("omask", ctypes.c_uint32 * 16)]


class Options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("tuple_capacity", ctypes.c_uint64),
        ("waves_per_cu", ctypes.c_uint32),
        ("steal", ctypes.c_uint32),
        ("steal_set", ctypes.c_uint32),
        ("deadline_ms", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 7),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("waves_per_cu", ctypes.c_uint32),
        ("steal", ctypes.c_uint32),
        ("poll_cycles", ctypes.c_uint32),
        ("split_inner", ctypes.c_uint32),
        ("split_leaf", ctypes.c_uint32),
        ("query_launch", ctypes.c_uint32),
        ("handover_gate", ctypes.c_uint32),
        ("coalesced_search", ctypes.c_uint32),
        ("group_seeds", ctypes.c_uint32),
        ("shared_leaf", ctypes.c_uint32),
    ]

    FIELDS = ("waves_per_cu", "steal", "poll_cycles", "split_inner", "split_leaf", "query_launch", "handover_gate",
              "coalesced_search", "group_seeds", "shared_leaf")

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f in self.FIELDS}


class ServeOptions(ctypes.Structure):
    _fields_ = [
        ("max_batch_updates", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("coalesce", ctypes.c_uint32),
        ("tuple_fill_pct", ctypes.c_uint32),
        ("max_batch_ms", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 3),
    ]


class RequestResult(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("batch", ctypes.c_uint64),
        ("t_submit_ms", ctypes.c_double),
        ("t_done_ms", ctypes.c_double),
        ("n_updates", ctypes.c_uint32),
        ("status", ctypes.c_int32),
    ]


class ServeBatch(ctypes.Structure):
    _fields_ = [
        ("batch", ctypes.c_uint64),
        ("first_ticket", ctypes.c_uint64),
        ("n_requests", ctypes.c_uint32),
        ("n_updates", ctypes.c_uint32),
        ("n_canonical", ctypes.c_uint32),
        ("n_queries", ctypes.c_uint32),
        ("status", ctypes.c_int32),
        ("ms_device", ctypes.c_float),
        ("t_start_ms", ctypes.c_double),
        ("t_done_ms", ctypes.c_double),
        ("n_tuples", ctypes.c_uint64),
        ("n_tuples_found", ctypes.c_uint64),
    ]


class QueryResult(ctypes.Structure):
    _fields_ = [
        ("qid", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("count", ctypes.c_uint64 * 2),
        ("hash_sum", ctypes.c_uint64 * 2),
        ("hash_xor", ctypes.c_uint64 * 2),
        ("open_seeds", ctypes.c_uint64),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("n_input", ctypes.c_uint32),
        ("n_canonical", ctypes.c_uint32),
        ("n_insert", ctypes.c_uint32),
        ("n_delete", ctypes.c_uint32),
        ("n_noop", ctypes.c_uint32),
        ("n_duplicate", ctypes.c_uint32),
        ("n_touched", ctypes.c_uint32),
        ("n_groups", ctypes.c_uint32),
        ("n_seeds", ctypes.c_uint64),
        ("dfs_nodes", ctypes.c_uint64),
        ("steals", ctypes.c_uint64),
        ("cand_scanned", ctypes.c_uint64),
        ("bytes_alg_dfs", ctypes.c_uint64),
        ("bytes_alg_update", ctypes.c_uint64),
        ("ms_canon", ctypes.c_float),
        ("ms_merge", ctypes.c_float),
        ("ms_filter", ctypes.c_float),
        ("ms_seed", ctypes.c_float),
        ("ms_dfs", ctypes.c_float),
        ("ms_commit", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("reserved1", ctypes.c_float),
        ("cyc_idle", ctypes.c_uint64),
        ("cyc_init", ctypes.c_uint64),
        ("cyc_inner", ctypes.c_uint64),
        ("cyc_leaf", ctypes.c_uint64),
        ("cyc_handover", ctypes.c_uint64),
        ("tasks_received", ctypes.c_uint64),
        ("seeds_started", ctypes.c_uint64),
    ]


class BatchResult(ctypes.Structure):
    _fields_ = [
        ("n_queries", ctypes.c_uint32),
        ("tuple_width", ctypes.c_uint32),
        ("queries", ctypes.POINTER(QueryResult)),
        ("n_tuples", ctypes.c_uint64),
        ("n_tuples_found", ctypes.c_uint64),
        ("tuples", ctypes.c_void_p),
        ("meta", ctypes.c_void_p),
        ("ord", ctypes.c_void_p),
        ("n_canonical", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("canon_lo", ctypes.POINTER(ctypes.c_uint32)),
        ("canon_hi", ctypes.POINTER(ctypes.c_uint32)),
        ("canon_sign", ctypes.POINTER(ctypes.c_uint8)),
        ("upd_count", ctypes.POINTER(ctypes.c_uint64)),
        ("upd_hash_sum", ctypes.POINTER(ctypes.c_uint64)),
        ("upd_hash_xor", ctypes.POINTER(ctypes.c_uint64)),
        ("stats", BatchStats),
        ("upd_open", ctypes.POINTER(ctypes.c_uint8)),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgamma.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgamma.so is not built (%s); run __graft_entry__.build() or "
                           "python paper_2401_17018_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    st = ctypes.c_int
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    lib.gamma_create.restype = st
    lib.gamma_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.gamma_destroy.restype = st
    lib.gamma_destroy.argtypes = [P]
    lib.gamma_load_graph.restype = st
    lib.gamma_load_graph.argtypes = [P, u32, u64, P, P, P, ctypes.c_int]
    lib.gamma_register_query.restype = st
    lib.gamma_register_query.argtypes = [P, u32, P, u32, P, ctypes.POINTER(u32)]
    lib.gamma_apply_batch.restype = st
    lib.gamma_apply_batch.argtypes = [P, u32, P, P, P, ctypes.c_int, u32, ctypes.POINTER(BatchResult)]
    lib.gamma_apply_batch_noalloc.restype = st
    lib.gamma_apply_batch_noalloc.argtypes = [P, u32, P, P, P, ctypes.c_int, u32, ctypes.POINTER(BatchResult)]
    lib.gamma_apply_batch_vertices.restype = st
    lib.gamma_apply_batch_vertices.argtypes = [P, u32, P, P, P, P, u32, P, ctypes.c_int, u32,
                                               ctypes.POINTER(BatchResult)]
    lib.gamma_load_graph_el.restype = st
    lib.gamma_load_graph_el.argtypes = [P, u32, u64, P, P, P, P, u32, ctypes.c_int]
    lib.gamma_register_query_el.restype = st
    lib.gamma_register_query_el.argtypes = [P, u32, P, u32, P, P, ctypes.POINTER(u32)]
    lib.gamma_apply_batch_el.restype = st
    lib.gamma_apply_batch_el.argtypes = [P, u32, P, P, P, P, ctypes.c_int, u32, ctypes.POINTER(BatchResult)]
    lib.gamma_export_graph_el.restype = st
    lib.gamma_export_graph_el.argtypes = [P, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u32), P, P, P,
                                          P]
    lib.gamma_add_vertices.restype = st
    lib.gamma_add_vertices.argtypes = [P, u32, P, ctypes.POINTER(u32)]
    lib.gamma_get_tuning.restype = st
    lib.gamma_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.gamma_set_tuning.restype = st
    lib.gamma_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.gamma_set_deadline.restype = st
    lib.gamma_set_deadline.argtypes = [P, ctypes.c_uint32]
    lib.gamma_set_query_active.restype = st
    lib.gamma_set_query_active.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32]
    lib.gamma_autotune.restype = st
    lib.gamma_autotune.argtypes = [P, u32, P, P, P, ctypes.c_int, u32, u32, u32, ctypes.POINTER(Tuning),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.gamma_serve_create.restype = st
    lib.gamma_serve_create.argtypes = [P, ctypes.POINTER(ServeOptions), ctypes.POINTER(P)]
    lib.gamma_serve_submit.restype = st
    lib.gamma_serve_submit.argtypes = [P, u32, P, P, P, ctypes.POINTER(u64)]
    lib.gamma_serve_submit_el.restype = st
    lib.gamma_serve_submit_el.argtypes = [P, u32, P, P, P, P, ctypes.POINTER(u64)]
    lib.gamma_serve_poll.restype = st
    lib.gamma_serve_poll.argtypes = [P, ctypes.POINTER(RequestResult), u32, ctypes.POINTER(u32)]
    lib.gamma_serve_drain.restype = st
    lib.gamma_serve_drain.argtypes = [P]
    lib.gamma_serve_counts.restype = st
    lib.gamma_serve_counts.argtypes = [P, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.gamma_serve_get_batch.restype = st
    lib.gamma_serve_get_batch.argtypes = [P, u64, ctypes.POINTER(ServeBatch), ctypes.POINTER(QueryResult), u32]
    lib.gamma_serve_destroy.restype = st
    lib.gamma_serve_destroy.argtypes = [P]
    lib.gamma_serve_get_tuples.restype = st
    lib.gamma_serve_get_tuples.argtypes = [P, u64, P, P, P, u64, ctypes.POINTER(u64), ctypes.POINTER(u32)]
    lib.gamma_copy_tuples.restype = st
    lib.gamma_copy_tuples.argtypes = [P, P, P, P, u64, ctypes.c_int]
    lib.gamma_result_release.restype = st
    lib.gamma_result_release.argtypes = [P, ctypes.POINTER(BatchResult)]
    lib.gamma_export_graph.restype = st
    lib.gamma_export_graph.argtypes = [P, ctypes.POINTER(u32), ctypes.POINTER(u64), P, P, P]
    lib.gamma_validate_graph.restype = st
    lib.gamma_validate_graph.argtypes = [u32, u64, P, P, P]
    lib.gamma_validate_query.restype = st
    lib.gamma_validate_query.argtypes = [u32, P, u32, P]
    lib.gamma_describe_query.restype = st
    lib.gamma_describe_query.argtypes = [u32, P, u32, P, P, u32, ctypes.POINTER(PlanInfo), ctypes.POINTER(u32),
                                         u32, P, ctypes.POINTER(u32)]
    lib.gamma_validate_batch.restype = st
    lib.gamma_validate_batch.argtypes = [u32, u32, P, P, P]
    lib.gamma_validate_graph_el.restype = st
    lib.gamma_validate_graph_el.argtypes = [u32, u64, P, P, P, P, u32]
    lib.gamma_validate_batch_el.restype = st
    lib.gamma_validate_batch_el.argtypes = [u32, u32, u32, P, P, P, P]
    lib.gamma_status_string.restype = ctypes.c_char_p
    lib.gamma_status_string.argtypes = [st]
    lib.gamma_last_error.restype = ctypes.c_char_p
    lib.gamma_last_error.argtypes = [P]
    lib.gamma_version.restype = u32
    lib.gamma_version.argtypes = []
    _lib = lib
    return lib
