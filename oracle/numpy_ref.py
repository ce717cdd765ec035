"""Whole-field numpy twin of the C oracle (TEST INFRASTRUCTURE ONLY).

Written independently of ``oracle.c`` with ``np.roll`` shifts instead of
index loops, so that a transposed operand or a wrong neighbour in either
implementation shows up as a disagreement on small grids.  Same readings of
the paper as the C code (heat update of App. A; Euler scheme of App. B with
the limiter, flux and RK2 readings listed in ``oracle.c``).

Arrays are indexed [y, x] (row j, column i), x fastest in memory.
"""
from __future__ import annotations

import numpy as np


def _sh(a, dx=0, dy=0):
    """Value of the neighbour at (i+dx, j+dy) for every cell (periodic)."""
    return np.roll(np.roll(a, -dy, axis=-2), -dx, axis=-1)


def _ghosted(T, bc, bcv):
    """T padded by one ghost cell per side: periodic copy (bc 0), the constant bcv
    (Dirichlet, bc 1) or the edge cell itself (zero flux, bc 2)."""
    if bc == 0:
        return np.pad(T, 1, mode="wrap")
    if bc == 1:
        return np.pad(T, 1, mode="constant", constant_values=T.dtype.type(bcv))
    return np.pad(T, 1, mode="edge")


def heat_step(T: np.ndarray, r: float, bc: int = 0, bcv: float = 0.0) -> np.ndarray:
    """App. A update, evaluated as (T + r*dxx) + r*dyy with dxx = (T_E - 2T) + T_W."""
    r = T.dtype.type(r)
    two = T + T
    if bc == 0:
        dxx = (_sh(T, 1, 0) - two) + _sh(T, -1, 0)
        dyy = (_sh(T, 0, 1) - two) + _sh(T, 0, -1)
    else:
        G = _ghosted(T, bc, bcv)
        dxx = (G[1:-1, 2:] - two) + G[1:-1, :-2]
        dyy = (G[2:, 1:-1] - two) + G[:-2, 1:-1]
    return (T + r * dxx) + r * dyy


def heat_run(T0: np.ndarray, r: float, steps: int, bc: int = 0, bcv: float = 0.0) -> np.ndarray:
    T = np.array(T0, copy=True)
    for _ in range(steps):
        T = heat_step(T, r, bc, bcv)
    return T


def laplacian(T: np.ndarray) -> np.ndarray:
    """L T without 1/dx^2, in float64."""
    T = T.astype(np.float64)
    return (_sh(T, 1, 0) - 2.0 * T + _sh(T, -1, 0)) + (_sh(T, 0, 1) - 2.0 * T + _sh(T, 0, -1))


# ----------------------------------------------------------------- Euler


def _pressure(Q, gm1):
    u = Q[1] / Q[0]
    v = Q[2] / Q[0]
    return gm1 * (Q[3] - Q.dtype.type(0.5) * (Q[1] * u + Q[2] * v))


def _phys_flux(Q, a, gamma, gm1):
    """Physical flux along the axis whose momentum is Q[a]; returns (F, |u_a| + c)."""
    b = 2 if a == 1 else 1
    rho = Q[0]
    ua = Q[a] / rho
    ub = Q[b] / rho
    p = gm1 * (Q[3] - Q.dtype.type(0.5) * (Q[a] * ua + Q[b] * ub))
    F = np.empty_like(Q)
    F[0] = Q[a]
    F[a] = Q[a] * ua + p
    F[b] = Q[a] * ub
    F[3] = (Q[3] + p) * ua
    c = np.sqrt(gamma * p / rho)
    return F, np.abs(ua) + c


def _roe_speed(L, R, a, gm1):
    """|u~_a| + c~ at the sqrt(rho)-weighted (Roe) average of the face states L and R."""
    b = 2 if a == 1 else 1
    t = L.dtype.type
    wl, wr = np.sqrt(L[0]), np.sqrt(R[0])
    ual, ubl = L[a] / L[0], L[b] / L[0]
    uar, ubr = R[a] / R[0], R[b] / R[0]
    hl = (L[3] + _pressure(L, gm1)) / L[0]
    hr = (R[3] + _pressure(R, gm1)) / R[0]
    ua = (wl * ual + wr * uar) / (wl + wr)
    ub = (wl * ubl + wr * ubr) / (wl + wr)
    H = (wl * hl + wr * hr) / (wl + wr)
    return np.abs(ua) + np.sqrt(gm1 * (H - t(0.5) * (ua * ua + ub * ub)))


def _run_flux(A, B, C, D, a, gamma, scheme):
    """Numerical flux through the face between B and C of the runs A, B, C, D (arrays of
    conserved states, elementwise): pressure-ratio reconstruction, then the Rusanov form
    (scheme: variant bits, 1 = limiter exponents as printed, 2 = Roe-averaged speed)."""
    t = B.dtype.type
    gm1 = gamma - t(1)
    pA, pB, pC, pD = (_pressure(X, gm1) for X in (A, B, C, D))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        rB = (pC - pB) / (pB - pA)  # pressure ratio of the left cell
        rC = (pD - pC) / (pC - pB)  # pressure ratio of the right cell
        okB = (rB > 0) & (rB < np.inf)
        okC = (rC > 0) & (rC < np.inf)
        if scheme & 1:
            phiL = t(0.5) * np.minimum(rB, t(1))
            phiR = t(0.5) * np.minimum(t(1) / rC, t(1))
        else:
            phiL = t(0.5) * np.minimum(t(1) / rB, t(1))
            phiR = t(0.5) * np.minimum(rC, t(1))
        L = np.where(okB[None], B + phiL[None] * (C - B), B)
        R = np.where(okC[None], C + phiR[None] * (B - C), C)
    fL, sL = _phys_flux(L, a, gamma, gm1)
    fR, sR = _phys_flux(R, a, gamma, gm1)
    s = _roe_speed(L, R, a, gm1) if scheme & 2 else np.maximum(sL, sR)
    return t(0.5) * ((fR + fL) + s[None] * (L - R))


def _face_flux(Q, axis, gamma, scheme=0):
    """Flux through the face between each cell and its +axis neighbour (periodic)."""
    a = 1 if axis == "x" else 2
    shift = (lambda A, k: _sh(A, k, 0)) if axis == "x" else (lambda A, k: _sh(A, 0, k))
    return _run_flux(shift(Q, -1), Q, shift(Q, 1), shift(Q, 2), a, gamma, scheme)


def _wall_faces(Q, axis, gamma, scheme, bc):
    """The N + 1 faces along axis (face f between cells f - 1 and f; faces 0 and N are the
    walls) with two ghost cells per side: the edge cell (bc 2, zero gradient) or the mirrored
    cells with the normal momentum negated (bc 3, slip wall)."""
    a = 1 if axis == "x" else 2
    ax = -1 if axis == "x" else -2
    width = [(0, 0)] * Q.ndim
    width[ax] = (2, 2)
    P = np.pad(Q, width, mode="edge" if bc == 2 else "symmetric")
    if bc == 3:
        n = Q.shape[ax]
        idx = [slice(None)] * Q.ndim
        for sl in (slice(0, 2), slice(n + 2, n + 4)):
            idx[0] = a
            idx[ax] = sl
            P[tuple(idx)] = -P[tuple(idx)]
    n = Q.shape[ax]

    def cut(k):
        idx = [slice(None)] * Q.ndim
        idx[ax] = slice(k, k + n + 1)
        return P[tuple(idx)]

    return _run_flux(cut(0), cut(1), cut(2), cut(3), a, gamma, scheme)


def euler_stage(Qbase, Qflux, hx, hy, gamma, scheme=0, bc=0):
    if bc == 0:
        fx = _face_flux(Qflux, "x", gamma, scheme)
        gy = _face_flux(Qflux, "y", gamma, scheme)
        dF = fx - _sh(fx, -1, 0)
        dG = gy - _sh(gy, 0, -1)
    else:
        fx = _wall_faces(Qflux, "x", gamma, scheme, bc)
        gy = _wall_faces(Qflux, "y", gamma, scheme, bc)
        dF = fx[..., 1:] - fx[..., :-1]
        dG = gy[..., 1:, :] - gy[..., :-1, :]
    return (Qbase - hx * dF) - hy * dG


def euler_run(Q0, dt, dx, dy, gamma, steps, scheme=0, bc=0):
    Q = np.array(Q0, copy=True)
    t = Q.dtype.type
    g = t(gamma)
    hx, hy = t(0.5 * dt / dx), t(0.5 * dt / dy)
    kx, ky = t(dt / dx), t(dt / dy)
    for _ in range(steps):
        Qs = euler_stage(Q, Q, hx, hy, g, scheme, bc)
        Q = euler_stage(Q, Qs, kx, ky, g, scheme, bc)
    return Q
