"""Pins of the oracle's non-periodic heat boundaries (CPU only).

The paper's solver is periodic and notes that other conditions fit the same
decomposition.  The oracle takes two: Dirichlet (every neighbour outside the
square is a ghost cell at a fixed value) and zero flux (an outside neighbour
equals the edge cell).  Pinned by the closed-form eigenmodes of the two
walled operators, by the fixed point and the maximum principle (Dirichlet),
by conservation (zero flux), and by the independent numpy twin."""
import numpy as np
import pytest

import oracle
from oracle import numpy_ref
from paper_2105_10332_amd import problems

DIR, NEU = oracle.BC_DIRICHLET, oracle.BC_NEUMANN


def _mode(bc, N, p, q):
    i = np.arange(N)
    if bc == DIR:
        fx, fy = np.sin(np.pi * p * (i + 1) / (N + 1)), np.sin(np.pi * q * (i + 1) / (N + 1))
        lam = 4 * (np.sin(np.pi * p / (2 * (N + 1))) ** 2 + np.sin(np.pi * q / (2 * (N + 1))) ** 2)
    else:
        fx, fy = np.cos(np.pi * p * (i + 0.5) / N), np.cos(np.pi * q * (i + 0.5) / N)
        lam = 4 * (np.sin(np.pi * p / (2 * N)) ** 2 + np.sin(np.pi * q / (2 * N)) ** 2)
    return np.outer(fy, fx), lam


@pytest.mark.parametrize("bc", [DIR, NEU])
@pytest.mark.parametrize("N,p,q", [(16, 1, 1), (24, 3, 7), (33, 32, 1), (64, 5, 60)])
def test_eigenmode_decay(bc, N, p, q):
    """sin modes (Dirichlet 0) and cosine modes (zero flux) are eigenvectors of the walled
    5-point operator: each step multiplies them by 1 - r*lambda exactly (up to rounding)."""
    T0, lam = _mode(bc, N, p, q)
    r, M = 0.23, 40
    out = oracle.heat_run(T0, r, M, bc=bc)
    np.testing.assert_allclose(out, (1 - r * lam) ** M * T0, rtol=0, atol=1e-13)


def test_dirichlet_constant_is_fixed_point_and_max_principle():
    N = 40
    g = 0.625
    assert np.array_equal(oracle.heat_run(np.full((N, N), g), 0.25, 17, bc=DIR, bcv=g), np.full((N, N), g))
    T0 = problems.heat_sine_noise(N, seed=3)
    out = oracle.heat_run(T0, 0.25, 60, bc=DIR, bcv=g)
    assert out.min() >= min(g, T0.min()) - 1e-15 and out.max() <= max(g, T0.max()) + 1e-15
    # walls pull the field toward g: the distance to g shrinks in the max norm
    assert np.abs(out - g).max() < np.abs(T0 - g).max()


def test_zero_flux_conserves_sum():
    T0 = problems.heat_sine_noise(48, seed=5) + 1.0
    out = oracle.heat_run(T0, 0.2, 100, bc=NEU)
    assert abs(out.sum() - T0.sum()) < 1e-11 * abs(T0.sum())
    assert np.abs(out - out.mean()).max() < np.abs(T0 - T0.mean()).max()


@pytest.mark.parametrize("bc,bcv", [(DIR, 0.0), (DIR, -0.3), (NEU, 0.0)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_c_matches_numpy_twin(bc, bcv, dtype):
    T0 = problems.heat_sine_noise(36, seed=2).astype(dtype)
    a = oracle.heat_run(T0, 0.2, 25, bc=bc, bcv=bcv)
    b = numpy_ref.heat_run(T0, 0.2, 25, bc=bc, bcv=bcv)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, oracle.heat_run(T0, 0.2, 25))
