"""CPU: the pieces of bench.py's JSON line that are plain arithmetic or read
committed files (no GPU needed).

  * the roofline record: frac = achieved / 8 TB/s, the counter traffic and
    its rate beside it only when there is a traffic figure;
  * the counter traffic is taken from a committed rocprofv3 summary only
    while the search kernel's source hash equals the one recorded with the
    counters, else it is reported as null;
  * every committed counter summary parses and names the workload it
    covers;
  * percentiles."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_record_arithmetic():
    r = bench.roofline(3200.0, 3.2e12, 1.0, 2.4e10)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(0.4)
    assert r["avg_launch_ms"] == pytest.approx(1000.0)
    assert r["traffic"] == 2.4e10
    assert r["traffic_GBps"] == pytest.approx(24.0)
    assert r["hbm_frac"] == pytest.approx(0.003)
    r = bench.roofline(800.0, 4e11, 0.5, None)
    assert r["traffic"] is None and "traffic_GBps" not in r and "hbm_frac" not in r
    assert r["frac"] == pytest.approx(0.1)


def test_counter_traffic_follows_the_kernel_source(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_dfs_large-rmat24_hbm-counters.md")
    if not os.path.exists(path):
        pytest.skip("no counter summary for the large workload")
    text = open(path).read()
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["source_sha16"])
    assert bench.counter_traffic("large-rmat24") == pytest.approx(rec["traffic_bytes"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.counter_traffic("large-rmat24") is None
    assert bench.counter_traffic("no-such-workload") is None


def test_committed_counter_summaries_parse():
    pdir = os.path.join(ROOT, "profiles")
    found = 0
    for f in sorted(os.listdir(pdir)):
        if not f.endswith("_hbm-counters.md"):
            continue
        found += 1
        text = open(os.path.join(pdir, f)).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        assert rec["kernel"] == "k_dfs"
        assert f == "k_dfs_%s_hbm-counters.md" % rec["workload"]
        assert rec["traffic_bytes"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
        assert rec["fetch_bytes"] > 0 and rec["write_bytes"] >= 0 and rec["launch_ms"] > 0
        assert len(rec["source_sha16"]) == 16
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    assert found >= 1


def test_percentile():
    assert bench.percentile([], 50) == 0.0
    assert bench.percentile([3.0, 1.0, 2.0], 50) == pytest.approx(2.0)
    assert bench.percentile(list(range(101)), 99) == pytest.approx(99.0)
