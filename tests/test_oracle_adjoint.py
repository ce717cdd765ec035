"""Pins of the heat adjoint oracle (CPU only).

J = 1/2 sum (T^M - T*)^2.  The pins use facts independent of the adjoint's
code: J is exactly quadratic in T^0 (central differences are exact up to
rounding for any step), the transpose identity <A^M v, w> = <v, (A^T)^M w>,
and the closed form dJ/dr = M <lambda^M, L T^{M-1}> that holds because A is
symmetric and commutes with L on the periodic grid.
"""
import numpy as np

import oracle
from oracle import numpy_ref
from paper_2105_10332_amd import problems


def _case(n=32, M=50, r=0.2):
    T0 = problems.heat_fourier_modes(n, seed=problems.SEED_ADJ_T0)
    Ts = problems.heat_fourier_modes(n, seed=problems.SEED_ADJ_TARGET)
    return T0, Ts, n, M, r


def _J(T0, Ts, r, M):
    return oracle.l2_mismatch(oracle.heat_run(T0, r, M), Ts)


def test_dot_product_identity():
    n, M, r = 24, 30, 0.2
    rng = np.random.default_rng(11)
    v = rng.standard_normal((n, n))
    w = rng.standard_normal((n, n))
    Av = oracle.heat_run(v, r, M)
    ATw, _ = oracle.heat_adjoint(v, w, r, M)
    lhs = float(np.sum(Av * w))
    rhs = float(np.sum(v * ATw))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_gradient_T0_exact_central_difference():
    T0, Ts, n, M, r = _case()
    g = oracle.heat_run(T0, r, M) - Ts
    gT0, _ = oracle.heat_adjoint(T0, g, r, M)
    rng = np.random.default_rng(5)
    for _ in range(4):
        v = rng.standard_normal((n, n))
        fd = (_J(T0 + v, Ts, r, M) - _J(T0 - v, Ts, r, M)) / 2.0
        ad = float(np.sum(gT0 * v))
        assert abs(fd - ad) < 1e-9 * abs(ad), (fd, ad)


def test_gradient_r_closed_form_and_fd():
    T0, Ts, n, M, r = _case()
    TM = oracle.heat_run(T0, r, M)
    g = TM - Ts
    _, dJdr = oracle.heat_adjoint(T0, g, r, M)
    TM1 = oracle.heat_run(T0, r, M - 1)
    closed = M * float(np.sum(g * numpy_ref.laplacian(TM1)))
    assert abs(dJdr - closed) < 1e-10 * abs(closed), (dJdr, closed)
    d = 1e-5
    fd = (_J(T0, Ts, r + d, M) - _J(T0, Ts, r - d, M)) / (2 * d)
    assert abs(fd - dJdr) < 1e-7 * abs(dJdr), (fd, dJdr)


def test_gradient_direction_value():
    """Value of <lambda^0, v> for the seeded direction v (seed 0) on the 32^2, M=50 case."""
    T0, Ts, n, M, r = _case()
    g = oracle.heat_run(T0, r, M) - Ts
    gT0, _ = oracle.heat_adjoint(T0, g, r, M)
    v = np.random.default_rng(0).standard_normal((n, n))
    fd = (_J(T0 + v, Ts, r, M) - _J(T0 - v, Ts, r, M)) / 2.0
    assert abs(float(np.sum(gT0 * v)) - fd) < 1e-9 * abs(fd)


def test_fp32_adjoint_close_to_fp64():
    T0, Ts, n, M, r = _case()
    g = oracle.heat_run(T0, r, M) - Ts
    a64, r64 = oracle.heat_adjoint(T0, g, r, M)
    a32, r32 = oracle.heat_adjoint(T0.astype(np.float32), g.astype(np.float32), r, M)
    assert np.abs(a32 - a64).max() / np.abs(a64).max() < 1e-5
    assert abs(r32 - r64) / abs(r64) < 1e-5
