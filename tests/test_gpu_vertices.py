"""GPU: vertex updates (Sec. II-A).  A vertex deletion is expanded on the
device into deletions of its incident edges and applied with the batch's
explicit updates; the result must equal the oracle's on the merged batch
the oracle builds on the host (counts, checksums, tuple sets, per-update
attribution over the canonical batch).  Vertex insertion appends isolated
vertices; their edges then come as ordinary insertions."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import plain as O2
from oracle import vertices as OV
from paper_2401_17018_amd import GammaError, capi
from test_gpu_parity import _er, _mixed_batch, _skewed_graph, check_against_o2, make_ctx

pytestmark = pytest.mark.gpu


def _setup(ctx, g, qs):
    ctx.load_graph(g.row_ptr, g.col, g.labels)
    for q in qs:
        ctx.register_query(q.k, q.labels, q.edges)


def _vertex_case(g, seed, n_ins, n_del, n_vdel):
    """Explicit updates with no insertion at a deleted vertex, deleted
    vertices drawn with a bias to high degree (one repeated)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = np.diff(g.row_ptr).astype(np.float64)
    p = (deg + 1) / (deg + 1).sum()
    vdel = rng.choice(g.n, n_vdel, replace=False, p=p).astype(np.uint32)
    vdel = np.concatenate([vdel, vdel[:1]])
    b = _mixed_batch(g, seed, n_ins, n_del)
    dead = set(vdel.tolist())
    keep = np.array([not (o == 1 and (int(s) in dead or int(d) in dead))
                     for s, d, o in zip(b.src, b.dst, b.op)], bool)
    b = W.Batch(b.src[keep], b.dst[keep], b.op[keep])
    status, merged = OV.deletion_batch(g, b, vdel)
    assert status == "ok"
    return b, vdel, merged


def _graph(ctx):
    rp, col, lab = ctx.export_graph()
    return W.Graph(len(lab), rp, col, lab)


@pytest.mark.parametrize("seed,n_vdel", [(1, 1), (2, 7), (3, 40)])
def test_vertex_deletion_matches_oracle(seed, n_vdel):
    g = _skewed_graph(seed) if seed != 2 else _er(1500, 9000, 23, 3)
    qs = [W.query_from_edges(4, [(0, 1), (1, 2), (2, 3)], (0, 1, 0, 1)),
          W.query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 1))]
    b, vdel, merged = _vertex_case(g, seed, 200, 60, n_vdel)
    print("[vertices] seed %d: %d explicit updates, %d deleted vertices, %d merged" % (
        seed, len(b), len(vdel), len(merged)), flush=True)
    with make_ctx(cap=1 << 22) as ctx:
        _setup(ctx, g, qs)
        res = ctx.apply_batch(b.src, b.dst, b.op, delete_vertices=vdel, tuples=True, per_update=True,
                              canonical=True)
        after = _graph(ctx)
    with make_ctx(cap=1 << 22) as ctx:
        _setup(ctx, g, qs)
        plain = ctx.apply_batch(merged.src, merged.dst, merged.op, tuples=True, per_update=True, canonical=True)
    # the same as the plain path on the oracle's merged batch, per update
    assert np.array_equal(res.canon_lo, plain.canon_lo) and np.array_equal(res.canon_hi, plain.canon_hi)
    assert np.array_equal(res.upd_count, plain.upd_count) and np.array_equal(res.upd_hash_sum, plain.upd_hash_sum)
    assert np.array_equal(res.counts, plain.counts) and np.array_equal(res.hash_xor, plain.hash_xor)
    for qid, q in enumerate(qs):
        check_against_o2(res, g, q, merged, qid=qid, check_tuples=not res.truncated)
    assert res.count(0, 0) + res.count(1, 0) > 0
    # deleted vertices are isolated; the graph is the oracle's G'
    rp, col = O2.updated_graph(g, merged)
    assert np.array_equal(after.row_ptr, rp) and np.array_equal(after.col, col)
    assert all(after.row_ptr[v + 1] == after.row_ptr[v] for v in vdel.tolist())


class _DeviceArrays:
    """Device copies of host arrays, allocated with the HIP runtime the
    library itself loaded (the soname resolves to the loaded copy)."""

    def __init__(self, *arrays):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.ptrs = []
        for a in arrays:
            a = np.ascontiguousarray(a)
            p = ctypes.c_void_p()
            assert self.hip.hipMalloc(ctypes.byref(p), max(a.nbytes, 1)) == 0
            self.ptrs.append(p)
            if a.nbytes:
                assert self.hip.hipMemcpy(p, a.ctypes.data_as(ctypes.c_void_p), a.nbytes, 1) == 0  # host to device

    def __enter__(self):
        return self.ptrs

    def __exit__(self, *exc):
        for p in self.ptrs:
            self.hip.hipFree(p)


def _c_counts(lib, ctx_ptr, n_upd, ptrs, n_vdel, flags):
    res = capi.BatchResult()
    st = lib.gamma_apply_batch_vertices(ctx_ptr, n_upd, ptrs[0], ptrs[1], ptrs[2], None, n_vdel, ptrs[3],
                                        capi.GAMMA_MEM_DEVICE, flags, ctypes.byref(res))
    assert st == capi.GAMMA_OK, st
    q = res.queries[0]
    return [int(q.count[0]), int(q.count[1])], [int(q.hash_sum[0]), int(q.hash_sum[1])]


def test_vertex_deletion_device_inputs_and_dry_run():
    """Device-resident inputs through the C-ABI (GAMMA_MEM_DEVICE), as a dry
    run and then for real; the host path gives the same."""
    g = _er(800, 5000, 31, 2)
    q = W.query_from_edges(3, [(0, 1), (1, 2)], (0, 1, 0))
    b, vdel, merged = _vertex_case(g, 5, 100, 30, 5)
    flags = capi.F_COUNT | capi.F_HASH
    with make_ctx(cap=0) as ctx:
        _setup(ctx, g, [q])
        with _DeviceArrays(b.src, b.dst, b.op, vdel) as ptrs:
            dry = _c_counts(ctx._lib, ctx._ptr, len(b), ptrs, len(vdel), flags | capi.F_DRY_RUN)
            same = _graph(ctx)
            assert np.array_equal(same.col, g.col) and np.array_equal(same.row_ptr, g.row_ptr)
            real = _c_counts(ctx._lib, ctx._ptr, len(b), ptrs, len(vdel), flags)
        after = _graph(ctx)
    with make_ctx(cap=0) as ctx:
        _setup(ctx, g, [q])
        host = ctx.apply_batch(b.src, b.dst, b.op, delete_vertices=vdel)
    assert dry == real
    assert real[0] == [int(host.counts[0, 0]), int(host.counts[0, 1])]
    assert real[1] == [int(host.hash_sum[0, 0]), int(host.hash_sum[0, 1])]
    check_against_o2(host, g, q, merged, check_tuples=False)
    rp, col = O2.updated_graph(g, merged)
    assert np.array_equal(after.row_ptr, rp) and np.array_equal(after.col, col)


def test_vertex_deletion_only_and_empty():
    g = _er(200, 3000, 37, 2)  # dense enough that the hub sits in triangles
    q = W.query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 0))
    empty = np.zeros(0, np.uint32)
    with make_ctx() as ctx:
        _setup(ctx, g, [q])
        nothing = ctx.apply_batch(empty, empty, np.zeros(0, np.uint8), delete_vertices=empty)
        assert nothing.counts.sum() == 0
        deg = np.where(g.labels == 0, np.diff(g.row_ptr).astype(np.int64), -1)
        hub = int(np.argmax(deg))  # the busiest vertex with the query's label
        res = ctx.apply_batch(empty, empty, np.zeros(0, np.uint8), delete_vertices=[hub], tuples=True)
    status, merged = OV.deletion_batch(g, W.Batch(empty, empty, np.zeros(0, np.uint8)), [hub])
    ref = check_against_o2(res, g, q, merged)
    assert ref.count[1] == 0 and ref.count[0] > 0
    assert all(hub in t for t in res.tuple_set(0, 0, 3))


def test_vertex_deletion_errors_leave_graph():
    g = _er(300, 1500, 41, 2)
    q = W.query_from_edges(2, [(0, 1)], (0, 1))
    E = g.edge_keys()
    a, c = int(E[0] >> np.uint64(32)), int(E[0] & np.uint64(0xFFFFFFFF))
    absent = next(w for w in range(g.n) if w != a and not g.has_edge(a, w))
    with make_ctx(cap=0) as ctx:
        _setup(ctx, g, [q])
        cases = [
            (([a], [absent], [1]), [a], capi.GAMMA_ECONFLICT),  # insertion at a deleted vertex (edge absent)
            (([c], [a], [1]), [a], capi.GAMMA_ECONFLICT),  # ... and present: +e with the expanded -e
            (([], [], []), [g.n], capi.GAMMA_EINVAL),  # id out of range
        ]
        for (s, d, o), vd, want in cases:
            with pytest.raises(GammaError) as ei:
                ctx.apply_batch(np.array(s, np.uint32), np.array(d, np.uint32), np.array(o, np.uint8),
                                delete_vertices=np.array(vd, np.uint32))
            assert ei.value.status == want
            now = _graph(ctx)
            assert np.array_equal(now.row_ptr, g.row_ptr) and np.array_equal(now.col, g.col)
        # an explicit deletion at a deleted vertex collapses with the expanded one
        ok = ctx.apply_batch(np.array([a], np.uint32), np.array([c], np.uint32), np.array([0], np.uint8),
                             delete_vertices=np.array([a], np.uint32))
        assert ok.stats["n_duplicate"] == 1


def test_add_vertices_then_connect():
    g = _er(600, 3500, 43, 3)
    qs = [W.query_from_edges(3, [(0, 1), (1, 2)], (0, 1, 2)), W.query_from_edges(3, [(0, 1), (1, 2), (2, 0)], (0, 0, 1))]
    rng = np.random.Generator(np.random.PCG64(7))
    new_labels = rng.integers(0, 3, 5).tolist()
    g2 = OV.with_vertices(g, new_labels)
    ups = [("+", g.n + i, int(w)) for i in range(5) for w in rng.permutation(g.n)[:12].tolist()]
    ups += [("+", g.n, g.n + 1), ("+", g.n + 2, g.n + 4)]
    E = g.edge_keys()
    ups += [("-", int(e >> np.uint64(32)), int(e & np.uint64(0xFFFFFFFF))) for e in E[rng.permutation(len(E))[:20]]]
    b = W.batch_from_list(ups)
    with make_ctx() as ctx:
        _setup(ctx, g, qs)
        first = ctx.add_vertices(new_labels)
        assert first == g.n
        grown = _graph(ctx)
        assert grown.n == g.n + 5 and np.array_equal(grown.labels, g2.labels)
        assert np.array_equal(grown.col, g.col) and np.array_equal(grown.row_ptr, g2.row_ptr)
        res = ctx.apply_batch(b.src, b.dst, b.op, tuples=True, per_update=True)
        with pytest.raises(GammaError) as ei:
            ctx.add_vertices([70000])
        assert ei.value.status == capi.GAMMA_EINVAL
    for qid, q in enumerate(qs):
        check_against_o2(res, g2, q, b, qid=qid)
    assert res.count(0, 1) + res.count(1, 1) > 0
