"""Host-side logic of bench.py (no GPU): the one-GPU guard and the lookup of
the HBM-traffic records that the roofline object reports."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _records():
    out = []
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if name.endswith(".md"):
            for line in open(os.path.join(ROOT, "profiles", name)):
                if line.startswith("traffic-record:"):
                    out.append(json.loads(line.split(":", 1)[1]))
    return out


def test_traffic_records_are_well_formed():
    recs = _records()
    assert recs, "profiles/ holds no traffic record"
    for rec in recs:
        assert rec["kernel"] in bench.TRAFFIC_SOURCES
        assert len(rec["plan"]) == 2 and all(isinstance(v, int) for v in rec["plan"])
        assert len(rec["sources_sha256"]) == 64
        # counters and the algorithm agree to within a small factor: reads of
        # a slab panel are shared by its column tiles through L2, writes are
        # X and Y once
        assert 0.8 * rec["algorithmic_bytes"] < rec["fetch_bytes"] + rec["write_bytes"]
        assert rec["fetch_bytes"] + rec["write_bytes"] < 4.0 * rec["algorithmic_bytes"]


def test_traffic_lookup_matches_plan_and_sources(monkeypatch):
    recs = _records()
    current = [r for r in recs
               if bench.measured_traffic(r["kernel"], {"ht_tile": r["plan"][0],
                                                        "chunk_mb": r["plan"][1]}) is not None]
    for rec in current:
        plan = {"ht_tile": rec["plan"][0], "chunk_mb": rec["plan"][1]}
        assert bench.measured_traffic(rec["kernel"], plan) == pytest.approx(
            rec["fetch_bytes"] + rec["write_bytes"])
    # no record for an unknown kernel or an unmeasured plan
    assert bench.measured_traffic("exchange", {"ht_tile": 4, "chunk_mb": 1024}) is None
    assert bench.measured_traffic("half_transform", {"ht_tile": 4, "chunk_mb": 3}) is None
    # a changed source voids every record
    monkeypatch.setitem(bench.TRAFFIC_SOURCES, "half_transform",
                        bench.TRAFFIC_SOURCES["half_transform"] + ["jk_api.hip"])
    for rec in recs:
        plan = {"ht_tile": rec["plan"][0], "chunk_mb": rec["plan"][1]}
        assert bench.measured_traffic(rec["kernel"], plan) is None
