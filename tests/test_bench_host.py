"""Host checks of bench.py's bookkeeping (no GPU): the recorded HBM traffic is reported
only for the workload, variant and kernel sources it was measured on, and --gpus above 1
is refused."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("workload", sorted(bench.TRAFFIC_SOURCES))
def test_recorded_traffic_matches_its_sources(workload):
    path = os.path.join(bench.PROFILES, f"traffic_{workload}.json")
    rec = json.load(open(path))
    assert rec["workload"] == workload
    got = bench.recorded_traffic(workload, rec["variant"])
    if rec["kernel_source_sha256_16"] != bench.kernel_source_hash(workload):
        assert got is None           # sources changed since the counters were taken: reported as null
        return
    cal = rec["copy_calibration"]
    want = (rec["fetch_size_kib"] * cal["fetch_factor"] + rec["write_size_kib"] * cal["write_factor"]) * 1024
    assert got == pytest.approx(want, rel=1e-12)
    assert bench.recorded_traffic(workload, rec["variant"] + "-other") is None     # another variant
    assert bench.recorded_traffic(None, rec["variant"]) is None                   # scaled runs


def test_traffic_guard_rejects_changed_sources(monkeypatch):
    rec = json.load(open(os.path.join(bench.PROFILES, "traffic_randoms3072.json")))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda w="randoms3072": "0" * 16)
    assert bench.recorded_traffic("randoms3072", rec["variant"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
