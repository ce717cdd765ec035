"""The seeded input generators against what defines them: the isentropic vortex
(App. B) is a steady isentropic solution in the frame of the free stream, every
Fourier mode is an eigenvector of the periodic 5-point Laplacian, and the batch
ensemble keeps its stated ranges and seed."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2105_10332_amd import problems

GAMMA = 1.4


def primitives(Q, gamma=GAMMA):
    rho = Q[0]
    u, v = Q[1] / rho, Q[2] / rho
    p = (gamma - 1.0) * (Q[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


@pytest.mark.parametrize("eps", [1.0, 5.0])
def test_vortex_is_isentropic_with_free_stream_far_away(eps):
    Q = problems.shu_vortex(256, eps=eps)
    rho, u, v, p = primitives(Q)
    assert np.all(rho > 0) and np.all(p > 0)
    np.testing.assert_allclose(p, rho ** GAMMA, rtol=1e-12)  # p / rho^gamma = 1 everywhere
    # far from the centre (r > 4.9 at the corners) the perturbation is below exp((1 - 24)/2)
    for a in (rho[0, 0], u[0, 0], v[0, 0], p[0, 0]):
        assert abs(a - 1.0) < 1e-4
    # the density dip at the centre: T(0) = 1 - (gamma-1) eps^2 e / (8 gamma pi^2)
    T0 = 1 - (GAMMA - 1) * eps * eps * math.e / (8 * GAMMA * math.pi ** 2)
    assert rho.min() == pytest.approx(T0 ** (1 / (GAMMA - 1)), rel=2e-3)


def test_vortex_is_in_radial_equilibrium():
    # steady in the moving frame: (w . grad) w = -grad(p) / rho, w = (u - 1, v - 1)
    n, L = 1024, 10.0
    Q = problems.shu_vortex(n, eps=5.0)
    rho, u, v, p = primitives(Q)
    h = L / n
    wx, wy = u - 1.0, v - 1.0

    def ddx(f):
        return (np.roll(f, -1, axis=1) - np.roll(f, 1, axis=1)) / (2 * h)

    def ddy(f):
        return (np.roll(f, -1, axis=0) - np.roll(f, 1, axis=0)) / (2 * h)

    rx = wx * ddx(wx) + wy * ddy(wx) + ddx(p) / rho
    ry = wx * ddx(wy) + wy * ddy(wy) + ddy(p) / rho
    scale = np.abs(ddx(p) / rho).max()
    assert max(np.abs(rx).max(), np.abs(ry).max()) < 1e-3 * scale  # O(h^2) residual
    # a wrong vortex (the temperature dip halved) leaves an O(1) residual
    Qbad = problems.shu_vortex(n, eps=5.0)
    rb, ub, vb, pb = primitives(Qbad)
    pb = 1.0 + 0.5 * (pb - 1.0)
    bad = wx * ddx(wx) + wy * ddy(wx) + ddx(pb) / rb
    assert np.abs(bad).max() > 0.1 * scale


def test_fourier_modes_are_eigenvectors_of_the_discrete_laplacian():
    n = 128
    m = problems.fourier_modes()
    assert m.p.min() >= 1 and m.p.max() <= 32 and m.q.min() >= 1 and m.q.max() <= 32
    for k in range(3):
        one = problems.FourierModes(m.p[k:k + 1], m.q[k:k + 1], m.a[k:k + 1], m.phi[k:k + 1]).field(n)
        lap = (np.roll(one, 1, 0) + np.roll(one, -1, 0) + np.roll(one, 1, 1) + np.roll(one, -1, 1) - 4 * one)
        lam = -4 * (math.sin(math.pi * m.p[k] / n) ** 2 + math.sin(math.pi * m.q[k] / n) ** 2)
        np.testing.assert_allclose(lap, lam * one, atol=1e-12 * abs(m.a[k]) * 8)
    np.testing.assert_array_equal(problems.heat_fourier_modes(n), problems.heat_fourier_modes(n))
    assert not np.array_equal(problems.heat_fourier_modes(n), problems.heat_fourier_modes(n, seed=7))


def test_sine_noise_bounds():
    T = problems.heat_sine_noise(64)
    x = problems.cell_centres(64)
    base = np.sin(2 * math.pi * x)[None, :] * np.sin(2 * math.pi * x)[:, None]
    d = T - base
    assert np.abs(d).max() <= 1e-3 and np.abs(d).max() > 5e-4
    assert abs(d.mean()) < 1e-4


def test_batch_ensemble_ranges_and_seed():
    items = problems.batch_ensemble()
    heat = [it for it in items if it.kind == "heat"]
    euler = [it for it in items if it.kind == "euler"]
    assert len(heat) == 48 and len(euler) == 16
    assert all(128 <= it.n <= 1024 and it.n % 32 == 0 for it in heat)
    assert all(256 <= it.n <= 1024 and it.n % 32 == 0 for it in euler)
    assert all(0.05 <= it.r <= 0.24 for it in heat)
    assert all(1.0 <= it.eps <= 5.0 for it in euler)
    assert len({it.n for it in heat}) > 10  # uneven sizes
    again = problems.batch_ensemble()
    assert [(it.n, it.r, it.eps, it.seed) for it in again] == [(it.n, it.r, it.eps, it.seed) for it in items]
    other = problems.batch_ensemble(seed=5)
    assert [it.n for it in other] != [it.n for it in items]
