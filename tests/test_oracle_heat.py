"""Pins of the heat oracle against what the mathematics fixes (CPU only).

The oracle is the App. A forward-Euler update; these checks tie it to facts
that do not depend on its code: the exact amplification factor of discrete
Fourier modes, the action of one step on a unit impulse, conservation and
the maximum principle, and an independent numpy implementation.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import numpy_ref
from paper_2105_10332_amd import problems


def amplification(p, q, n, r):
    """G(p,q) = 1 - 4 r [sin^2(pi p/N) + sin^2(pi q/N)] for a mode of wavenumbers (p, q)."""
    return 1.0 - 4.0 * r * (math.sin(math.pi * p / n) ** 2 + math.sin(math.pi * q / n) ** 2)


def test_impulse_response_exact():
    """One step applied to a unit impulse: 1-4r at the cell, r at its four periodic neighbours.

    r = 1/8 keeps every value exactly representable, so any dropped term,
    wrong sign or wrong neighbour index fails bit-exactly.  The impulse sits
    on the corner so the periodic wrap is exercised in both axes."""
    n, r = 8, 0.125
    for (j, i) in [(0, 0), (3, 5), (7, 7)]:
        T = np.zeros((n, n))
        T[j, i] = 1.0
        out = oracle.heat_step(T, r)
        exp = np.zeros((n, n))
        exp[j, i] = 1.0 - 4 * r
        for dj, di in [(0, 1), (0, -1), (1, 0), (-1, 0)]:
            exp[(j + dj) % n, (i + di) % n] += r
        assert np.array_equal(out, exp)


def test_anisotropic_field_orientation():
    """A field varying only along x stays x-only; along y stays y-only (no axis mix-up)."""
    n, r = 16, 0.2
    x = problems.cell_centres(n)
    fx = np.tile(np.cos(2 * math.pi * 3 * x)[None, :], (n, 1))
    out = oracle.heat_step(fx, r)
    g = 1.0 - 4 * r * math.sin(math.pi * 3 / n) ** 2
    np.testing.assert_allclose(out, g * fx, atol=1e-15)
    out_y = oracle.heat_step(fx.T.copy(), r)
    np.testing.assert_allclose(out_y, g * fx.T, atol=1e-15)


def test_sine_mode_amplification_c1():
    """P1: sin(2 pi x) sin(2 pi y) is a discrete eigenmode; T^M = G^M T^0 (64^2, r=0.2, 100 steps)."""
    n, r, M = 64, 0.2, 100
    x = problems.cell_centres(n)
    S = np.sin(2 * math.pi * x)[None, :] * np.sin(2 * math.pi * x)[:, None]
    G = amplification(1, 1, n, r)
    assert abs(G - 0.9961477813377575) < 1e-15
    out = oracle.heat_run(S, r, M)
    err = np.abs(out - G ** M * S).max()
    assert err < 1e-13, err
    assert abs(G ** M - 0.6797938036723735) < 1e-14


def test_sine_noise_max_principle_c1():
    """C1 with noise: by linearity and the maximum principle (r <= 1/4) the deviation
    from the noise-free mode never exceeds the noise amplitude 1e-3."""
    n, r, M = 64, 0.2, 100
    T0 = problems.heat_sine_noise(n)
    x = problems.cell_centres(n)
    S = np.sin(2 * math.pi * x)[None, :] * np.sin(2 * math.pi * x)[:, None]
    out = oracle.heat_run(T0, r, M)
    G = amplification(1, 1, n, r)
    assert np.abs(out - G ** M * S).max() <= 1e-3


def test_continuous_solution_weak_pin():
    """App. A analytic solution exp(-8 pi^2 alpha t) sin sin: the discrete run agrees
    to its truncation error O(dx^2) (weak pin: 64^2, alpha=1, t = M r dx^2)."""
    n, r, M = 64, 0.2, 100
    x = problems.cell_centres(n)
    S = np.sin(2 * math.pi * x)[None, :] * np.sin(2 * math.pi * x)[:, None]
    t = M * r / n ** 2
    out = oracle.heat_run(S, r, M)
    cont = math.exp(-8 * math.pi ** 2 * t)
    assert abs(cont - 0.68009) < 1e-4
    assert np.abs(out - cont * S).max() < 1e-3


@pytest.mark.parametrize("n,M", [(64, 100), (128, 300)])
def test_fourier_modes_closed_form(n, M):
    """P2: the 16-mode initial state evolves as sum a G_pq^M cos(...) exactly (up to roundoff)."""
    r = 0.2
    modes = problems.fourier_modes(problems.SEED_HEAT_MODES)
    T0 = modes.field(n)
    G = np.array([amplification(p, q, n, r) for p, q in zip(modes.p, modes.q)])
    exp = modes.field(n, amp_scale=G ** M)
    out = oracle.heat_run(T0, r, M)
    # normalised by the initial amplitude: high modes decay to ~1e-9, far below it
    err = np.abs(out - exp).max() / np.abs(T0).max()
    assert err < 1e-14, err
    assert np.abs(exp).max() > 1e3 * err


def test_c2_mode_factors():
    """Amplification factors quoted for the 4096^2 configuration (r = 0.2)."""
    assert abs(amplification(1, 1, 4096, 0.2) - 0.999999058761362) < 1e-15
    assert abs(amplification(32, 32, 4096, 0.2) - 0.999036364964138) < 1e-15


def test_invariants():
    """P3: sum T is conserved, max/min are monotone, the l2 norm does not grow."""
    n, r = 48, 0.24
    rng = np.random.default_rng(7)
    T = rng.standard_normal((n, n))
    s0 = T.sum()
    mx, mn, l2 = T.max(), T.min(), np.linalg.norm(T)
    for _ in range(50):
        T = oracle.heat_step(T, r)
        assert T.max() <= mx + 1e-15 and T.min() >= mn - 1e-15
        assert np.linalg.norm(T) <= l2 * (1 + 1e-15)
        mx, mn, l2 = T.max(), T.min(), np.linalg.norm(T)
    assert abs(T.sum() - s0) < 1e-11


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_c_matches_numpy_twin(dtype):
    """Two independent implementations of the same update agree bit for bit."""
    T0 = problems.heat_sine_noise(40).astype(dtype)
    a = oracle.heat_run(T0, 0.2, 37)
    b = numpy_ref.heat_run(T0, 0.2, 37)
    assert a.dtype == dtype
    assert np.array_equal(a, b)


def test_fp32_error_vs_fp64_stated():
    """FP32 oracle vs FP64 oracle on the C1 case: the error is of FP32 rounding size."""
    T0 = problems.heat_sine_noise(64)
    a = oracle.heat_run(T0, 0.2, 100)
    b = oracle.heat_run(T0.astype(np.float32), 0.2, 100).astype(np.float64)
    err = np.abs(a - b).max() / np.abs(a).max()
    assert 1e-9 < err < 1e-5
