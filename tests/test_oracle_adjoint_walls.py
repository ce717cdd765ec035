"""Pins of the oracle's adjoint of the walled heat advance (CPU only).

The walled step is affine in T (the Dirichlet ghosts add a constant), so J is
still quadratic in T0 and exact central differences pin dJ/dT0; central
differences in r pin dJ/dr (including the ghost term of the walled
Laplacian); the dot-product identity pins the transpose of the homogeneous
walled step; the eigenmodes of the walled operators give dJ/dr and dJ/dT0 in
closed form."""
import numpy as np
import pytest

import oracle
from paper_2105_10332_amd import problems

DIR, NEU = oracle.BC_DIRICHLET, oracle.BC_NEUMANN


def _J(T0, Ts, r, M, bc, bcv):
    return oracle.l2_mismatch(oracle.heat_run(T0, r, M, bc=bc, bcv=bcv), Ts)


@pytest.mark.parametrize("bc,bcv", [(DIR, 0.0), (DIR, 0.8), (NEU, 0.0)])
def test_gradients_vs_central_differences(bc, bcv):
    N, M, r = 24, 30, 0.21
    T0 = problems.heat_fourier_modes(N, seed=problems.SEED_ADJ_T0)
    Ts = problems.heat_fourier_modes(N, seed=problems.SEED_ADJ_TARGET)
    g = oracle.heat_run(T0, r, M, bc=bc, bcv=bcv) - Ts
    gT0, dJdr = oracle.heat_adjoint(T0, g, r, M, bc=bc, bcv=bcv)
    rng = np.random.default_rng(11)
    for _ in range(4):
        v = rng.standard_normal((N, N))
        fd = (_J(T0 + v, Ts, r, M, bc, bcv) - _J(T0 - v, Ts, r, M, bc, bcv)) / 2.0
        ad = float(np.sum(gT0 * v))
        assert abs(fd - ad) <= 1e-9 * abs(ad)
    d = 1e-6
    fd = (_J(T0, Ts, r + d, M, bc, bcv) - _J(T0, Ts, r - d, M, bc, bcv)) / (2 * d)
    assert abs(fd - dJdr) <= 1e-6 * abs(dJdr), (fd, dJdr)


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_transpose_identity(bc):
    """<A0^M v, w> = <v, (A0^T)^M w> for the homogeneous walled step A0."""
    N, M = 20, 17
    rng = np.random.default_rng(3)
    v, w = rng.standard_normal((N, N)), rng.standard_normal((N, N))
    Av = oracle.heat_run(v, 0.24, M, bc=bc, bcv=0.0)
    ATw, _ = oracle.heat_adjoint(v, w, 0.24, M, bc=bc, bcv=0.0)
    lhs, rhs = float(np.sum(Av * w)), float(np.sum(v * ATw))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


@pytest.mark.parametrize("bc", [DIR, NEU])
def test_eigenmode_closed_form(bc):
    """T0 = an eigenmode phi of the walled operator (eigenvalue -lam), J = 1/2 |T^M|^2:
    T^M = G^M phi with G = 1 - r lam, so dJ/dT0 = G^(2M) phi and
    dJ/dr = -M lam G^(2M-1) |phi|^2."""
    N, M, r, p, q = 28, 25, 0.2, 3, 5
    i = np.arange(N)
    if bc == DIR:
        phi = np.outer(np.sin(np.pi * q * (i + 1) / (N + 1)), np.sin(np.pi * p * (i + 1) / (N + 1)))
        lam = 4 * (np.sin(np.pi * p / (2 * (N + 1))) ** 2 + np.sin(np.pi * q / (2 * (N + 1))) ** 2)
    else:
        phi = np.outer(np.cos(np.pi * q * (i + 0.5) / N), np.cos(np.pi * p * (i + 0.5) / N))
        lam = 4 * (np.sin(np.pi * p / (2 * N)) ** 2 + np.sin(np.pi * q / (2 * N)) ** 2)
    G = 1 - r * lam
    TM = oracle.heat_run(phi, r, M, bc=bc)
    gT0, dJdr = oracle.heat_adjoint(phi, TM, r, M, bc=bc)
    np.testing.assert_allclose(gT0, G ** (2 * M) * phi, rtol=0, atol=1e-13)
    exp = -M * lam * G ** (2 * M - 1) * float(np.sum(phi * phi))
    assert abs(dJdr - exp) <= 1e-11 * abs(exp)
