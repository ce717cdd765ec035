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
    (24, 12, 13), (18, 6, 10), (30, 10, 11), (64, 32, 20), (8, 4, 5), (12, 4, 8),  # b = 4: the smallest window, h = 2
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


@pytest.mark.parametrize("bc,bcv", [(1, 0.0), (1, 0.4), (2, 0.0)])
@pytest.mark.parametrize("N,b,L", [(16, 8, 11), (24, 8, 9), (32, 16, 21), (36, 12, 14)])
def test_swept_equals_standard_heat_walls(bc, bcv, N, b, L):
    """Dirichlet and zero-flux walls: the unchanged swept schedule, with outside neighbours
    read as ghost values, gives the walled Standard result bit for bit (every dependency of
    a walled cell is one of its periodic dependencies)."""
    T0 = problems.heat_sine_noise(N, seed=N + b + L)
    out, _ = SweptSim(Geom(N, b, 1, L), "heat", {"r": 0.2, "bc": bc, "bcv": bcv}).run(T0)
    assert np.array_equal(out, oracle.heat_run(T0, 0.2, L, bc=bc, bcv=bcv))


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


@pytest.mark.parametrize("n,b,L", [(1, 8, 30), (1, 16, 37), (1, 6, 20), (2, 16, 30), (2, 12, 25), (2, 8, 13)])
def test_kernel_ring_rule_matches_rings(n, b, L):
    """The per-cell rule the phase kernel uses to pick its up-front loads equals the union
    of the rings Box(F(l), n) minus F(l-1), per level parity, for every shape and cut."""
    from paper_2105_10332_amd import geometry

    g = Geom(3 * b, b, n, L)
    W = b + 2 * n
    C = b // 2 + n
    for p in range(g.n_phases()):
        for (wx, wy) in g.shapes(p):
            lo, hi = g.levels(wx, wy)
            want = [np.full((W, W), -1), np.full((W, W), -1)]
            ox = g.centre(wx, 0) - C
            oy = g.centre(wy, 0) - C

            def mask(f, grow):
                m = np.zeros((W, W), bool)
                if f is not None:
                    m[f[2] - oy - grow:f[3] - oy + grow, f[0] - ox - grow:f[1] - ox + grow] = True
                return m

            for lvl in range(lo, hi + 1):
                ring = mask(g.footprint(wx, wy, 0, 0, lvl), n)
                if lvl > lo:
                    ring &= ~mask(g.footprint(wx, wy, 0, 0, lvl - 1), 0)
                assert np.all(want[(lvl - 1) % 2][ring] == -1)
                want[(lvl - 1) % 2][ring] = lvl - 1
                if n == 2 and lvl == lo and lvl % 2 == 0:
                    f = mask(g.footprint(wx, wy, 0, 0, lvl), 0)
                    want[lvl % 2][f] = lvl - 2
            got = [np.full((W, W), -1), np.full((W, W), -1)]
            for ly in range(W):
                for lx in range(W):
                    for par, lev in geometry.ring_load_parities(wx, wy, lo, hi, g.h, n, b, lx, ly,
                                                                two_stage=(n == 2)).items():
                        got[par][ly, lx] = lev
            assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (p, wx, wy)


@pytest.mark.parametrize("kind,N,b,L", [("heat", 32, 16, 21), ("heat", 18, 6, 10), ("heat", 64, 32, 20),
                                        ("euler", 24, 12, 14), ("euler", 48, 16, 20)])
def test_preloaded_protocol(kind, N, b, L):
    """All of a shape's loads issued before its first level (the kernel's order) is safe."""
    if kind == "heat":
        T0 = problems.heat_sine_noise(N)
        out, _ = SweptSim(Geom(N, b, 1, L), "heat", {"r": 0.2}, preload=True).run(T0)
        assert np.array_equal(out, oracle.heat_run(T0, 0.2, L))
    else:
        Q0 = problems.shu_vortex(N)
        dx = 10.0 / N
        dt = oracle.cfl_dt(Q0, dx, dx, 1.4, 0.4)
        out, _ = SweptSim(Geom(N, b, 2, L), "euler", {"gamma": 1.4, "dt": dt, "dx": dx}, preload=True).run(Q0)
        assert np.array_equal(out, oracle.euler_run(Q0, dt, dx, dx, 1.4, L // 2))
