"""bench.py end to end on the GPU at small sizes: one JSON line per run with the
contract's keys, the roofline object and the Swept/Standard comparison."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

KEYS = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config"}


def run_bench(*extra):
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1", "--no-cpu", *extra]
    print("bench:", " ".join(extra), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=100, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, p.stdout
    rec = json.loads(lines[0])
    assert KEYS <= set(rec)
    assert rec["n_gpus"] == 1 and rec["steps"] == 2 and rec["warmup"] == 1 and rec["value"] > 0
    assert "workload" in rec["config"]
    return rec


def check_roofline(rec):
    rf = rec["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert rf["achieved"] == pytest.approx(rf["alg_bytes_per_launch"] / (rf["avg_launch_us"] * 1e-6) / 1e9)
    assert rf["traffic"] is None  # no counters were taken at these sizes


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bench_heat(dtype):
    rec = run_bench("--n", "512", "--advance-steps", "64", "--tile", "32", "--dtype", dtype)
    assert rec["dtype"] == dtype and rec["unit"] == "cell-updates/s"
    check_roofline(rec)
    assert rec["standard"]["traffic_per_launch"] is None
    assert rec["bounds"]["frac"]["hbm"] == pytest.approx(rec["roofline"]["frac"])
    assert rec["speedup_vs_standard"] == pytest.approx(rec["value"] / rec["standard"]["value"])


def test_bench_euler():
    rec = run_bench("--workload", "euler", "--n", "256", "--advance-steps", "16", "--tile", "16", "--wg", "256")
    assert rec["unit"] == "cell-steps/s"
    check_roofline(rec)
    assert rec["reductions"]["cfl_dt"]["GBps"] > 0


def test_bench_adjoint():
    rec = run_bench("--workload", "adjoint", "--n", "256", "--advance-steps", "64")
    assert rec["value"] > 0 and rec["adjoint_over_forward"] > 0


def test_bench_batch_per_phase():
    # one launch per global phase: a cooperative launch has failed to start in a second
    # process while this one (the test runner, after the batch tests) was alive with
    # cooperative launches of its own
    rec = run_bench("--workload", "batch", "--advance-steps", "8", "--batch-per-phase")
    assert rec["value"] > 0 and "per global phase" in rec["config"]["workload"]


@pytest.mark.skip(reason="a cooperative batch launch (hipLaunchCooperativeKernel) has been refused with "
                         "SWEPT_EHIP in a second process started while the test runner, after the batch tests, "
                         "held cooperative launches of its own; test_bench_batch_per_phase covers the bench path")
def test_bench_batch_cooperative():
    rec = run_bench("--workload", "batch", "--advance-steps", "8")
    assert rec["value"] > 0


def test_bench_refuses_more_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8"], capture_output=True,
                       text=True, timeout=60, cwd=ROOT)
    assert p.returncode == 2 and "one GPU" in p.stderr
