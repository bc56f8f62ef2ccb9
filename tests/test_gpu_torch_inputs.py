"""GPU: torch tensors as inputs.  torch ships its own HIP runtime with the
same soname as the one the library links; imported first, it is the one
the process uses, and device tensors (GAMMA_MEM_DEVICE) must give what host
arrays give.  Run in a child process so that this test's import order does
not depend on the rest of the suite."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import torch
torch.zeros(1, device="cuda")
sys.path[:0] = [ROOT, ROOT + "/tests"]
import workloads as W
from test_gpu_parity import _er, _mixed_batch
from paper_2401_17018_amd import Context
g = _er(900, 6000, 77, 2)
q = W.query_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], (0, 1, 0, 1))
b = _mixed_batch(g, 7, 300, 100)
dev = torch.device("cuda:0")
t = lambda a: torch.from_numpy(a.astype(np.int32) if a.dtype == np.uint32 else a).to(dev)
with Context(device=0) as ctx:
    ctx.load_graph(t(g.row_ptr.astype(np.int64)), t(g.col), t(g.labels))
    ctx.register_query(q.k, q.labels, q.edges)
    d = ctx.apply_batch(t(b.src), t(b.dst), t(b.op), per_update=True, dry_run=True)
    h = ctx.apply_batch(b.src, b.dst, b.op, per_update=True)
assert np.array_equal(d.counts, h.counts) and np.array_equal(d.hash_sum, h.hash_sum), (d.counts, h.counts)
assert np.array_equal(d.upd_count, h.upd_count)
assert h.counts.sum() > 0
print("torch inputs ok", h.counts.tolist(), flush=True)
"""


def test_torch_device_tensors_match_host_arrays():
    code = "ROOT = %r\n" % ROOT + CHILD
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=180)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0 and "torch inputs ok" in r.stdout
