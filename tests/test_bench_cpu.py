"""Host-side checks of bench.py: its contract (one GPU), the gating of measured
traffic by the kernel-source hash, the roofline arithmetic, the algorithmic byte
counts it divides by, and the CPU-oracle baseline record."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2105_10332_amd import geometry  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_code_text_ignores_comments_and_spacing():
    a = "int f(int x) { // one\n  return x + 1; /* two\n three */ }\n"
    b = "int f(int x)\n{\n    return x + 1;\n}"
    assert bench.code_text(a) == bench.code_text(b) == "int f(int x) { return x + 1; }"


def test_traffic_is_reported_only_for_the_measured_sources(monkeypatch):
    key = ("heat", "f64", 4096, 64, 512, 1000)
    value, digest = bench.MEASURED_TRAFFIC[key]
    monkeypatch.setattr(bench, "kernel_hash", lambda: digest)
    assert bench.measured_traffic(key) == value
    assert bench.measured_traffic(("heat", "f64", 4096, 32, 512, 1000)) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.measured_traffic(key) is None
    skey = ("euler", "f64", 2048)
    assert bench.measured_traffic(skey, bench.MEASURED_STANDARD_TRAFFIC) is None


def test_kernel_hash_is_sixteen_hex_digits():
    h = bench.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_roofline_arithmetic():
    plan = {"loads": 3_000_000, "stores": 1_000_000, "launches": 4}
    r = bench.roofline(plan, 8, 1, 8, 2e-3, "k")
    alg = (3_000_000 + 1_000_000) * 8 / 4  # bytes per launch
    assert r["alg_bytes_per_launch"] == alg
    assert r["avg_launch_us"] == pytest.approx(250.0)
    assert r["achieved"] == pytest.approx(alg / 250e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["traffic"] is None


@pytest.mark.parametrize("n,b,R,levels,nvar,S,launches,mb", [
    (4096, 64, 1, 1000, 1, 8, 65, 517.9),    # heat FP64, the default bench line
    (2048, 16, 2, 1000, 4, 8, 501, 498.6),   # Euler FP64 (500 RK2 steps = 1000 stage-levels)
    (2048, 32, 2, 1000, 4, 4, 251, 259.1),   # Euler FP32
])
def test_algorithmic_bytes_per_launch(n, b, R, levels, nvar, S, launches, mb):
    plan = geometry.totals(n, b, R, levels, R == 2)
    assert plan["launches"] == launches
    alg = (plan["loads"] + plan["stores"]) * S * nvar / plan["launches"]
    assert alg / 1e6 == pytest.approx(mb, abs=0.05)


def test_measured_traffic_covers_at_least_the_algorithmic_bytes():
    # HBM bytes from the counters can exceed the memory protocol's (cache-line granularity,
    # ring cells fetched twice), never fall below it
    alg = {("heat", "f64"): 517.9e6, ("euler", "f64"): 498.6e6, ("euler", "f32"): 259.1e6}
    for (kind, dt, *_), (value, _) in bench.MEASURED_TRAFFIC.items():
        if (kind, dt) in alg:
            assert value >= alg[(kind, dt)]
    for (kind, dt, n), (value, _) in bench.MEASURED_STANDARD_TRAFFIC.items():
        S, nvar = (8 if dt == "f64" else 4), (1 if kind == "heat" else 4)
        assert value >= 2 * S * nvar * n * n  # one read and one write of the state per step


def test_cpu_baseline_record():
    import numpy as np

    rec = bench.cpu_heat(np.float64, 64, 0.2, budget_s=0.05)
    assert rec["kind"] == "oracle" and rec["unit"] == "cell-updates/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "64x64" in rec["sample"]


@pytest.mark.parametrize("S", [8, 4])
def test_three_bound_model_agrees_with_the_roofline(S):
    n, b, M = 4096, 64, 1000
    plan = geometry.totals(n, b, 1, M)
    sec = 0.032
    rate = n * n * M / sec
    rf = bench.roofline(plan, S, 1, plan["launches"], sec, "k")
    bd = bench.heat_bounds(plan, S, n * n * M, rate)
    assert bd["frac"]["hbm"] == pytest.approx(rf["frac"])
    assert bd["binding"] == max(bd["frac"], key=bd["frac"].get)
    # LDS: 3 values per update at 128 B/clk/CU over 256 CUs at 2.4 GHz
    assert bd["ps_per_update"]["lds"] == pytest.approx(3 * S / (128 * 256 * 2.4e9) * 1e12)
    assert bd["ps_per_update"]["valu"] == pytest.approx(9 / ({8: 78.6, 4: 157.3}[S] * 1e12) * 1e12)
