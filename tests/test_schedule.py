"""Swept schedule and memory protocol, proven on the CPU (no GPU).

P5/P6: the swept decomposition (Sec. 3.3: Up-Pyramid, X/Y-Bridges,
Octahedra, Down-Pyramid) with the GPU kernels' two-buffer load/compute/store
protocol, executed by ``swept_sim`` with the oracle's stencil, equals the
oracle's one-step-at-a-time run bit for bit; every read finds its value at
the right level and no two instances of a phase conflict.
"""
import numpy as np
import pytest

import oracle
from paper_2105_10332_amd import problems
from swept_sim import Geom, SweptSim, check_partition

HEAT_CASES = [  # (N, b, L): N in {2b, 3b, 4b}; L a multiple of h and not; odd h (b = 6, 10)
    (16, 8, 1), (16, 8, 4), (16, 8, 9), (24, 8, 16), (32, 8, 13), (32, 16, 21), (48, 16, 8),
    (24, 12, 13), (18, 6, 10), (30, 10, 11), (64, 32, 20),
]
EULER_CASES = [  # stage-levels L (even = whole RK2 steps); h = b/4
    (16, 8, 2), (16, 8, 10), (32, 16, 12), (32, 16, 18), (24, 12, 14), (48, 16, 20), (40, 20, 16),
]


@pytest.mark.parametrize("N,b,L", HEAT_CASES)
def test_partition_heat(N, b, L):
    check_partition(Geom(N, b, 1, L))


@pytest.mark.parametrize("N,b,L", EULER_CASES)
def test_partition_euler(N, b, L):
    check_partition(Geom(N, b, 2, L))


@pytest.mark.parametrize("N,b,L", HEAT_CASES)
def test_swept_equals_standard_heat(N, b, L):
    T0 = problems.heat_sine_noise(N, seed=N + b + L)
    out, _ = SweptSim(Geom(N, b, 1, L), "heat", {"r": 0.2}).run(T0)
    assert np.array_equal(out, oracle.heat_run(T0, 0.2, L))


def test_swept_equals_standard_heat_fp32():
    T0 = problems.heat_sine_noise(32).astype(np.float32)
    out, _ = SweptSim(Geom(32, 16, 1, 19), "heat", {"r": 0.2}, dtype=np.float32).run(T0)
    assert out.dtype == np.float32
    assert np.array_equal(out, oracle.heat_run(T0, 0.2, 19))


@pytest.mark.parametrize("N,b,L", EULER_CASES)
def test_swept_equals_standard_euler(N, b, L):
    Q0 = problems.shu_vortex(N)
    dx = 10.0 / N
    dt = oracle.cfl_dt(Q0, dx, dx, 1.4, 0.4)
    out, _ = SweptSim(Geom(N, b, 2, L), "euler", {"gamma": 1.4, "dt": dt, "dx": dx}).run(Q0)
    assert np.array_equal(out, oracle.euler_run(Q0, dt, dx, dx, 1.4, L // 2))


def test_traffic_falls_with_tile():
    """Values moved through the buffers per (cell, level) shrink roughly as 1/b (the
    point of the method: each value crosses HBM once per ~b/(2n) levels)."""
    per = {}
    for b in (8, 16, 32):
        N, L = 2 * b if b == 32 else 4 * b, 3 * b
        T0 = np.zeros((N, N))
        _, tr = SweptSim(Geom(N, b, 1, L), "heat", {"r": 0.2}).run(T0)
        per[b] = (tr.loads + tr.stores) / (N * N * L)
    assert per[16] < 0.65 * per[8] and per[32] < 0.65 * per[16], per


def test_stale_read_is_detected():
    """Negative control: storing only each cell's top level (not top and top-1) leaves
    later shapes without values they need; the level-tag check must catch it."""
    import swept_sim

    sim = SweptSim(Geom(16, 8, 1, 9), "heat", {"r": 0.2}, store_lag=1)
    with pytest.raises(swept_sim.ProtocolError):
        sim.run(problems.heat_sine_noise(16))
