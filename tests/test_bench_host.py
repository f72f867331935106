"""Host checks of bench.py's bookkeeping (no GPU): the recorded HBM traffic is reported
only for the workload, variant and kernel sources it was measured on, and --gpus above 1
is refused."""
import json
import time
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


def _fake_step(duration, log):
    def step():
        time.sleep(duration)
        log.append(time.monotonic())
    return step


@pytest.mark.parametrize("warmup", [0, 1, 5])
def test_steps_stay_inside_the_wall_clock_budget(warmup):
    """--steps/--warmup are upper limits: a run whose steps cannot all fit times fewer (at least
    one), reports how many, and ends inside the budget."""
    log, checks = [], []
    t0 = time.monotonic()
    budget = bench.Budget(0.0)
    budget.end = t0 + 1.6
    res = bench.run_steps(_fake_step(0.2, log), lambda: None, warmup, 20, budget, reserve_s=0.3,
                          after_first=(lambda: checks.append(len(log))) if warmup else None)
    assert 1 <= res["steps"] < 20
    assert res["warmup_done"] == (min(warmup, 1) if warmup <= 1 else res["warmup_done"])
    assert res["warmup_done"] + res["steps"] == len(log)
    assert time.monotonic() - t0 <= 1.6
    assert res["elapsed_s"] == pytest.approx(0.2 * res["steps"], abs=0.15)
    if warmup:
        assert checks == [1]            # the checks ran once, right after the first warmup step


def test_at_least_one_step_is_timed_when_nothing_fits():
    log = []
    budget = bench.Budget(0.0)
    budget.end = time.monotonic() - 10.0
    res = bench.run_steps(_fake_step(0.05, log), lambda: None, 5, 20, budget)
    assert res["warmup_done"] == 1 and res["steps"] == 1 and len(log) == 2


def test_all_requested_steps_run_when_they_fit():
    log = []
    budget = bench.Budget(0.0)
    budget.end = time.monotonic() + 60.0
    res = bench.run_steps(_fake_step(0.01, log), lambda: None, 3, 7, budget)
    assert res["warmup_done"] == 3 and res["steps"] == 7 and len(log) == 10


def test_timed_steps_come_before_extra_warmups():
    """With room for a few steps only, the steps go to timing, not to the requested warmups."""
    log = []
    budget = bench.Budget(0.0)
    budget.end = time.monotonic() + 1.0
    res = bench.run_steps(_fake_step(0.2, log), lambda: None, 5, 20, budget)
    assert res["warmup_done"] == 1 and res["steps"] >= 3


def test_long_steps_report_each_end(monkeypatch, capsys):
    """Steps of tens of seconds end with a synchronization and a progress line each, so a run
    of several such steps is never silent for more than one step; short steps stay queued
    with a single synchronization after the timed loop."""
    monkeypatch.setattr(bench, "LONG_STEP_S", 0.05)
    log, syncs = [], []
    budget = bench.Budget(0.0)
    budget.end = time.monotonic() + 60.0
    res = bench.run_steps(_fake_step(0.06, log), lambda: syncs.append(len(log)), 2, 4, budget)
    err = capsys.readouterr().err
    assert res["steps"] == 4 and res["warmup_done"] == 2
    assert [f"timed step {k} of 4 done" in err for k in (1, 2, 3, 4)] == [True] * 4
    assert all(n in syncs for n in range(2, 7))      # a synchronization after every step but the first
    monkeypatch.setattr(bench, "LONG_STEP_S", 1e9)
    log, syncs = [], []
    res = bench.run_steps(_fake_step(0.01, log), lambda: syncs.append(len(log)), 1, 5, budget)
    assert "done" not in capsys.readouterr().err.replace("0 done", "")
    assert res["steps"] == 5 and syncs.count(6) == 1   # one synchronization after the timed loop


def test_optional_run_is_kept_free_only_beside_two_timed_steps():
    log = []
    budget = bench.Budget(0.0)
    budget.end = time.monotonic() + 1.3          # first warmup 0.2 s, then room for ~5 steps
    res = bench.run_steps(_fake_step(0.2, log), lambda: None, 1, 20, budget, optional=(1.0, 0.1))
    assert res["optional"] and res["steps"] >= 2
    assert budget.left() >= 0.2                  # one more step still fits for the optional run
    log = []
    budget.end = time.monotonic() + 0.75         # first warmup 0.2 s, then room for ~2 steps
    res = bench.run_steps(_fake_step(0.2, log), lambda: None, 1, 20, budget, optional=(1.0, 0.1))
    assert not res["optional"] and res["steps"] >= 2
