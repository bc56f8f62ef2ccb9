"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and the host-only validators enforce the documented rules."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2401_17018_amd import capi, validate_batch, validate_graph, validate_query

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.LIB_PATH):
        from paper_2401_17018_amd import build
        build.build()
    return capi.load_library()


def header_functions():
    text = open(os.path.join(ROOT, "include", "gamma.h")).read()
    return sorted(set(re.findall(r"\b(gamma_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert header_functions() == sorted(capi.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for st in range(-7, 2):
        assert lib.gamma_status_string(st)
    assert lib.gamma_version() >= 100


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ptr = ctypes.c_void_p()
    st = lib.gamma_create(None, ctypes.byref(ptr))
    assert st == capi.GAMMA_EDEVICE and not ptr.value
    # calls on a null context are rejected, not crashed
    assert lib.gamma_destroy(None) == capi.GAMMA_OK
    t = capi.Tuning()
    assert lib.gamma_get_tuning(None, ctypes.byref(t)) == capi.GAMMA_EINVAL
    assert lib.gamma_set_tuning(None, ctypes.byref(t)) == capi.GAMMA_EINVAL
    assert lib.gamma_autotune(None, 0, None, None, None, 0, 0, 8, 1, ctypes.byref(t), None, None) == capi.GAMMA_EINVAL
    srv = ctypes.c_void_p()
    assert lib.gamma_serve_create(None, None, ctypes.byref(srv)) == capi.GAMMA_EINVAL and not srv.value
    assert lib.gamma_serve_submit(None, 0, None, None, None, None) == capi.GAMMA_EINVAL
    assert lib.gamma_serve_drain(None) == capi.GAMMA_EINVAL
    assert lib.gamma_serve_destroy(None) == capi.GAMMA_OK


def test_validate_graph(lib):
    g = W.graph_from_edges(4, [(0, 1), (1, 2), (2, 3)], [0, 1, 0, 1])
    assert validate_graph(g.row_ptr, g.col, g.labels) == 0
    # row 1 not ascending
    assert validate_graph(g.row_ptr, np.array([1, 2, 0, 1, 3, 2], np.uint32), g.labels) == capi.GAMMA_EINVAL
    # asymmetric
    rp = np.array([0, 1, 1], np.uint64)
    assert validate_graph(rp, np.array([1], np.uint32), np.zeros(2, np.uint32)) == capi.GAMMA_EINVAL
    # self loop
    rp = np.array([0, 1, 1], np.uint64)
    assert validate_graph(rp, np.array([0], np.uint32), np.zeros(2, np.uint32)) == capi.GAMMA_EINVAL
    # label out of range
    assert validate_graph(g.row_ptr, g.col, np.array([0, 1, 70000, 1], np.uint32)) == capi.GAMMA_EINVAL
    # id out of range
    rp = np.array([0, 1, 2], np.uint64)
    assert validate_graph(rp, np.array([5, 0], np.uint32), np.zeros(2, np.uint32)) == capi.GAMMA_EINVAL
    # duplicate entry in a row
    rp = np.array([0, 2, 3, 4], np.uint64)
    assert validate_graph(rp, np.array([1, 1, 0, 0], np.uint32), np.zeros(3, np.uint32)) == capi.GAMMA_EINVAL


def test_validate_query(lib):
    assert validate_query(3, [0, 0, 0], [[0, 1], [1, 2]]) == 0
    assert validate_query(3, [0, 0, 0], [[0, 1], [1, 2], [0, 2]]) == 0
    assert validate_query(1, [0], np.zeros((0, 2), np.uint32)) == capi.GAMMA_EINVAL
    assert validate_query(17, [0] * 17, [[i, i + 1] for i in range(16)]) == capi.GAMMA_EUNSUPPORTED
    assert validate_query(4, [0] * 4, [[0, 1], [2, 3], [0, 1]]) == capi.GAMMA_EINVAL  # repeated
    assert validate_query(4, [0] * 4, [[0, 1], [2, 3], [1, 0]]) == capi.GAMMA_EINVAL  # repeated (reversed)
    assert validate_query(4, [0] * 4, [[0, 1], [1, 1], [2, 3]]) == capi.GAMMA_EINVAL  # self loop
    assert validate_query(4, [0] * 4, [[0, 1], [0, 2], [1, 2]]) == capi.GAMMA_EUNSUPPORTED  # disconnected
    assert validate_query(3, [0, 70000, 0], [[0, 1], [1, 2]]) == capi.GAMMA_EINVAL
    assert validate_query(3, [0, 0, 0], [[0, 5], [1, 2]]) == capi.GAMMA_EINVAL


def test_validate_batch(lib):
    assert validate_batch(5, [0, 1], [1, 2], [1, 0]) == 0
    assert validate_batch(5, [0], [0], [1]) == capi.GAMMA_EINVAL
    assert validate_batch(5, [0], [9], [1]) == capi.GAMMA_EINVAL
    assert validate_batch(5, [0, 1], [1, 0], [1, 0]) == capi.GAMMA_ECONFLICT
    assert validate_batch(5, [0, 1], [1, 0], [1, 1]) == 0  # duplicate, not a conflict
    assert validate_batch(5, [], [], []) == 0


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def test_validate_labelled_graph_and_batch(lib):
    g = W.graph_from_labelled_edges(4, [(0, 1, 0), (1, 2, 2), (2, 3, 1)], [0, 1, 0, 1], 3)
    rp, col, lab, el = g.row_ptr, g.col, g.labels, g.elab
    v = lambda e, L: lib.gamma_validate_graph_el(4, len(col), _p(rp), _p(col), _p(lab), _p(e), L)
    assert v(el, 3) == 0
    assert v(el, 2) == capi.GAMMA_EINVAL          # a label >= n_elabels
    bad = el.copy()
    bad[0] = (bad[0] + 1) % 3                     # mirror entry disagrees
    assert v(bad, 3) == capi.GAMMA_EINVAL
    assert v(None, 1) == 0 and v(None, 3) == capi.GAMMA_EINVAL
    u32 = lambda *x: np.array(x, np.uint32)
    vb = lambda s, d, o, e, L=3: lib.gamma_validate_batch_el(4, L, len(s), _p(s), _p(d), _p(np.array(o, np.uint8)),
                                                            _p(e))
    assert vb(u32(0, 1), u32(1, 2), [1, 0], u32(0, 2)) == 0
    assert vb(u32(0, 1), u32(1, 0), [1, 1], u32(0, 1)) == capi.GAMMA_ECONFLICT  # one pair, two labels
    assert vb(u32(0, 1), u32(1, 0), [1, 1], u32(2, 2)) == 0                     # duplicate triple
    assert vb(u32(0), u32(1), [1], u32(3)) == capi.GAMMA_EINVAL                 # label out of range
    assert vb(u32(0), u32(1), [1], None) == 0
