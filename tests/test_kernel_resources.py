"""The search kernel's register budget, as the last build recorded it
(hipcc's kernel-resource-usage remarks, paper_2401_17018_amd/_build).

The lean build (no coalesced plans, edge labels or tuple output: the plain
count and checksum search that the large and mid workloads time) is held to
128 VGPRs, so that four waves per SIMD (16 per CU, the default launch) stay
resident, and must fit them without spilling to scratch; the full build,
which carries every feature, is held to three waves per SIMD and may spill
at most a few registers."""
import json
import os

import pytest

RES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2401_17018_amd", "_build",
                   "k_dfs.hip.resources.json")


@pytest.mark.skipif(not os.path.exists(RES), reason="library not built here")
def test_search_kernel_register_budgets():
    res = json.load(open(RES))
    dfs = {k: v for k, v in res.items() if "k_dfs" in k}
    lean = [v for k, v in dfs.items() if "ILb0E" in k]
    full = [v for k, v in dfs.items() if "ILb1E" in k]
    assert len(dfs) == 2 and len(lean) == 1 and len(full) == 1, sorted(res)
    assert lean[0]["occupancy"] >= 4 and lean[0]["vgprs"] <= 128, lean[0]
    assert full[0]["occupancy"] >= 3 and full[0]["vgprs"] <= 168, full[0]
    assert lean[0].get("scratch_bytes", 0) == 0 and lean[0].get("vgpr_spill", 0) == 0, lean[0]
    assert full[0].get("scratch_bytes", 0) <= 64, full[0]
