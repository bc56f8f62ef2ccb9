"""The search kernel's register budget, as the last build recorded it
(hipcc's kernel-resource-usage remarks, paper_2401_17018_amd/_build).

The default launch keeps 12 waves per CU, three per SIMD, resident; both
builds of the search kernel are held to that budget.  The lean build (no
coalesced plans, edge labels or tuple output: the plain count and checksum
search that the large and mid workloads time) must fit it without spilling
to scratch; the full build, which carries every feature, may spill at most a
few registers."""
import json
import os

import pytest

RES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2401_17018_amd", "_build",
                   "k_dfs.hip.resources.json")


@pytest.mark.skipif(not os.path.exists(RES), reason="library not built here")
def test_search_kernel_keeps_three_waves_per_simd():
    res = json.load(open(RES))
    dfs = {k: v for k, v in res.items() if "k_dfs" in k}
    lean = [v for k, v in dfs.items() if "ILb0E" in k]
    full = [v for k, v in dfs.items() if "ILb1E" in k]
    assert len(dfs) == 2 and len(lean) == 1 and len(full) == 1, sorted(res)
    for r in (lean[0], full[0]):
        assert r["occupancy"] >= 3, r
        assert r["vgprs"] <= 168, r
    assert lean[0].get("scratch_bytes", 0) == 0 and lean[0].get("vgpr_spill", 0) == 0, lean[0]
    assert full[0].get("scratch_bytes", 0) <= 64, full[0]
