"""The swept adjoint schedule, proven on the CPU against the oracle's discrete adjoint.

Per cycle: forward Up-Pyramid -> P, forward Bridges -> Q, then the reverse
sweep on the shifted tiling whose shapes recompute the forward T of their own
footprints (sources chosen by owner) and pair lambda with T (adjoint_sim)."""
import numpy as np
import pytest

import oracle
from paper_2105_10332_amd import problems
from adjoint_sim import AdjointSim


@pytest.mark.parametrize("N,b,M", [(16, 8, 8), (16, 8, 12), (24, 8, 16), (32, 16, 24), (24, 12, 18), (20, 10, 15),
                                   (8, 4, 8)])
def test_swept_adjoint_equals_oracle(N, b, M):
    T0 = problems.heat_fourier_modes(N, seed=problems.SEED_ADJ_T0)
    Ts = problems.heat_fourier_modes(N, seed=problems.SEED_ADJ_TARGET)
    g = oracle.heat_run(T0, 0.2, M) - Ts
    lam, dJdr = AdjointSim(N, b, 0.2).run(T0, g, M)
    ref, rref = oracle.heat_adjoint(T0, g, 0.2, M)
    assert np.array_equal(lam, ref)
    assert abs(dJdr - rref) <= 1e-13 * abs(rref)
