"""The search kernel's register budget, as the last build recorded it
(hipcc's kernel-resource-usage remarks, paper_2401_17018_amd/_build).

The default launch keeps 12 waves per CU, three per SIMD, resident; the
kernel is built for that budget and must fit it without spilling to
scratch: at two waves per SIMD the mid search measured 5-10 % slower."""
import json
import os

import pytest

RES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2401_17018_amd", "_build",
                   "k_dfs.hip.resources.json")


@pytest.mark.skipif(not os.path.exists(RES), reason="library not built here")
def test_search_kernel_keeps_three_waves_per_simd_without_spills():
    res = json.load(open(RES))
    dfs = [v for k, v in res.items() if "k_dfs" in k]
    assert len(dfs) == 1, sorted(res)
    r = dfs[0]
    assert r["occupancy"] >= 3, r
    assert r["vgprs"] <= 168, r
    assert r.get("scratch_bytes", 0) == 0 and r.get("vgpr_spill", 0) == 0, r
