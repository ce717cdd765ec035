"""Seeded synthetic inputs shaped like the paper's two workloads.

This module only builds initial states and problem lists; it holds none of
the solver's arithmetic, so both the CPU oracle (in tests) and the GPU path
take their inputs from here.  All randomness is numpy's PCG64
(``default_rng(seed)``); every generator takes its seed explicitly.

Workloads (the paper uses no dataset; these stand in for App. A and B):

* heat on the periodic unit square, cell centres x_i = (i + 1/2)/N:
  - :func:`heat_sine_noise`: the App. A initial condition sin(2 pi x) sin(2 pi y)
    plus i.i.d. uniform noise;
  - :func:`heat_fourier_modes`: a sum of random Fourier modes
    a cos(2 pi (p x + q y) + phi), p, q in 1..kmax, a ~ N(0,1)/sqrt(p^2+q^2);
    each mode is an exact eigenvector of the discrete 5-point operator, so
    the discrete solution is known in closed form;
* Euler on the periodic square [0, 10]^2: :func:`shu_vortex`, the isentropic
  vortex of App. B (Table 1 cites Shu) superposed on the free stream
  (rho, u, v, p) = (1, 1, 1, 1), centred at (5, 5);
* :func:`batch_ensemble`: the uneven ensemble of heat and Euler problems run
  in one persistent launch.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_HEAT_NOISE = 0
SEED_HEAT_MODES = 1
SEED_ADJ_T0 = 2
SEED_ADJ_TARGET = 3
SEED_BATCH = 4


def cell_centres(n: int, length: float = 1.0) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


def heat_sine_noise(n: int, seed: int = SEED_HEAT_NOISE, amp: float = 1e-3) -> np.ndarray:
    """sin(2 pi x) sin(2 pi y) + U(-amp, amp), float64 (n, n) indexed [y, x]."""
    x = cell_centres(n)
    base = np.sin(2 * math.pi * x)[None, :] * np.sin(2 * math.pi * x)[:, None]
    rng = np.random.default_rng(seed)
    return base + rng.uniform(-amp, amp, size=(n, n))


@dataclass
class FourierModes:
    p: np.ndarray
    q: np.ndarray
    a: np.ndarray
    phi: np.ndarray

    def field(self, n: int, amp_scale=None) -> np.ndarray:
        """Sum of a_k cos(2 pi (p_k x + q_k y) + phi_k) at the cell centres (float64)."""
        x = cell_centres(n)
        out = np.zeros((n, n), dtype=np.float64)
        scale = np.ones_like(self.a) if amp_scale is None else amp_scale
        for p, q, a, ph, s in zip(self.p, self.q, self.a, self.phi, scale):
            out += (a * s) * np.cos(2 * math.pi * (p * x[None, :] + q * x[:, None]) + ph)
        return out


def fourier_modes(seed: int = SEED_HEAT_MODES, n_modes: int = 16, kmax: int = 32) -> FourierModes:
    rng = np.random.default_rng(seed)
    p = rng.integers(1, kmax + 1, size=n_modes)
    q = rng.integers(1, kmax + 1, size=n_modes)
    k = np.sqrt(p.astype(np.float64) ** 2 + q.astype(np.float64) ** 2)
    a = rng.standard_normal(n_modes) / k
    phi = rng.uniform(0.0, 2 * math.pi, size=n_modes)
    return FourierModes(p, q, a, phi)


def heat_fourier_modes(n: int, seed: int = SEED_HEAT_MODES, n_modes: int = 16, kmax: int = 32) -> np.ndarray:
    return fourier_modes(seed, n_modes, kmax).field(n)


def shu_vortex(n: int, eps: float = 5.0, gamma: float = 1.4, length: float = 10.0,
               centre=(5.0, 5.0), u_inf: float = 1.0, v_inf: float = 1.0) -> np.ndarray:
    """Conserved state (rho, rho u, rho v, E) of the isentropic vortex, (4, n, n) float64.

    T = 1 - (gamma-1) eps^2/(8 gamma pi^2) exp(1 - r^2), rho = T^(1/(gamma-1)),
    p = rho T, (u, v) = (u_inf, v_inf) + eps/(2 pi) exp((1 - r^2)/2) (-(y-yc), x-xc).
    """
    x = cell_centres(n, length)
    X = x[None, :] - centre[0]
    Y = x[:, None] - centre[1]
    r2 = X * X + Y * Y
    e = np.exp(0.5 * (1.0 - r2))
    du = -eps / (2 * math.pi) * Y * e
    dv = eps / (2 * math.pi) * X * e
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    u = u_inf + du
    v = v_inf + dv
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


def uniform_state(n: int, rho=1.0, u=1.0, v=1.0, p=1.0, gamma=1.4) -> np.ndarray:
    """Constant free stream as conserved variables, (4, n, n) float64."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([np.full((n, n), rho), np.full((n, n), rho * u), np.full((n, n), rho * v),
                     np.full((n, n), E)])


@dataclass
class BatchItem:
    kind: str          # "heat" or "euler"
    n: int
    r: float = 0.0     # heat: alpha dt / dx^2
    eps: float = 0.0   # euler: vortex strength
    seed: int = 0
    extra: dict = field(default_factory=dict)


def batch_ensemble(seed: int = SEED_BATCH, n_heat: int = 48, n_euler: int = 16,
                   heat_edges=(128, 1024), euler_edges=(256, 1024), step: int = 32):
    """Uneven ensemble: heat edges U{128..1024 step 32}, r ~ U[0.05, 0.24];
    Euler edges U{256..1024 step 32}, eps ~ U[1, 5]."""
    rng = np.random.default_rng(seed)
    items = []
    for k in range(n_heat):
        n = int(rng.integers(heat_edges[0] // step, heat_edges[1] // step + 1)) * step
        r = float(rng.uniform(0.05, 0.24))
        items.append(BatchItem("heat", n, r=r, seed=1000 + k))
    for k in range(n_euler):
        n = int(rng.integers(euler_edges[0] // step, euler_edges[1] // step + 1)) * step
        eps = float(rng.uniform(1.0, 5.0))
        items.append(BatchItem("euler", n, eps=eps, seed=2000 + k))
    return items
