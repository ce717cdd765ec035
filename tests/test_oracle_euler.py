"""Pins of the Euler oracle (App. B scheme) against what the mathematics fixes (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import numpy_ref
from paper_2105_10332_amd import problems

GAMMA = 1.4


def prim_flux(rho, u, v, p, axis):
    """Textbook physical flux from primitive variables (App. B, F and G)."""
    E = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)
    if axis == 1:
        return np.array([rho * u, rho * u * u + p, rho * u * v, (E + p) * u])
    return np.array([rho * v, rho * u * v, rho * v * v + p, (E + p) * v])


def cons(rho, u, v, p):
    E = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)
    return np.array([rho, rho * u, rho * v, E])


def minmod(a, b):
    if a * b <= 0:
        return 0.0
    return a if abs(a) < abs(b) else b


def test_free_stream_preserved_exactly():
    """A uniform state is a fixed point of the scheme (all flux differences are zero)."""
    Q0 = problems.uniform_state(24, rho=1.3, u=0.7, v=-0.4, p=2.1)
    out = oracle.euler_run(Q0, 1e-2, 10 / 24, 10 / 24, GAMMA, 10)
    assert np.array_equal(out, Q0)


@pytest.mark.parametrize("axis", [1, 2])
def test_consistent_flux(axis):
    """Equal states on both sides: the numerical flux equals the physical flux."""
    q = cons(1.2, 0.3, -0.8, 0.9)
    L, R, F = oracle.face(q, q, q, q, axis, GAMMA)
    np.testing.assert_allclose(F, prim_flux(1.2, 0.3, -0.8, 0.9, axis), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("axis", [1, 2])
def test_rusanov_dissipation(axis):
    """First-order states (non-monotone pressure): flux = (F_L+F_R)/2 - s/2 (Q_R-Q_L),
    s = max(|u_n|+c) over the two cells."""
    a, b, c, d = [(1.0, 0.2, 0.1, 1.0), (1.1, 0.3, -0.1, 1.5), (0.9, -0.1, 0.2, 0.8), (1.0, 0.0, 0.0, 1.6)]
    qa, qb, qc, qd = [cons(*s) for s in (a, b, c, d)]
    L, R, F = oracle.face(qa, qb, qc, qd, axis, GAMMA)
    # pressures 1.0, 1.5, 0.8, 1.6: ratio at B = (0.8-1.5)/(1.5-1.0) < 0, at C = (1.6-0.8)/(0.8-1.5) < 0
    np.testing.assert_array_equal(L, qb)
    np.testing.assert_array_equal(R, qc)
    un_b = b[1] if axis == 1 else b[2]
    un_c = c[1] if axis == 1 else c[2]
    s = max(abs(un_b) + math.sqrt(GAMMA * b[3] / b[0]), abs(un_c) + math.sqrt(GAMMA * c[3] / c[0]))
    exp = 0.5 * (prim_flux(*b, axis) + prim_flux(*c, axis)) - 0.5 * s * (qc - qb)
    np.testing.assert_allclose(F, exp, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("seed", range(20))
def test_limiter_is_minmod_on_pressure(seed):
    """For a fluid at rest, E = p/(gamma-1) is reconstructed linearly, so the face
    pressures must be the textbook minmod MUSCL values
    p_L = p_i + minmod(dp_-, dp_+)/2,  p_R = p_{i+1} - minmod(dp_+, dp_++)/2."""
    rng = np.random.default_rng(seed)
    ps = rng.uniform(0.5, 2.0, size=4)
    qs = [cons(1.0, 0.0, 0.0, p) for p in ps]
    L, R, F = oracle.face(*qs, 1, GAMMA)
    pL = (GAMMA - 1) * L[3]
    pR = (GAMMA - 1) * R[3]
    dm, d0, dp = ps[1] - ps[0], ps[2] - ps[1], ps[3] - ps[2]
    assert abs(pL - (ps[1] + 0.5 * minmod(dm, d0))) < 1e-14
    assert abs(pR - (ps[2] - 0.5 * minmod(d0, dp))) < 1e-14


def test_c_matches_numpy_twin_fp64():
    Q0 = problems.shu_vortex(32)
    dx = 10 / 32
    dt = oracle.cfl_dt(Q0, dx, dx, GAMMA, 0.4)
    a = oracle.euler_run(Q0, dt, dx, dx, GAMMA, 12)
    b = numpy_ref.euler_run(Q0, dt, dx, dx, GAMMA, 12)
    assert np.array_equal(a, b)


def test_c_matches_numpy_twin_fp32():
    Q0 = problems.shu_vortex(32).astype(np.float32)
    dx = 10 / 32
    a = oracle.euler_run(Q0, 0.02, dx, dx, GAMMA, 8)
    b = numpy_ref.euler_run(Q0, 0.02, dx, dx, GAMMA, 8)
    assert np.array_equal(a, b)


def test_conservation_to_roundoff():
    """P4: sum rho, rho u, rho v, E stay constant on the periodic grid (face fluxes telescope)."""
    n = 48
    Q0 = problems.shu_vortex(n)
    dx = 10 / n
    dt = oracle.cfl_dt(Q0, dx, dx, GAMMA, 0.4)
    out = oracle.euler_run(Q0, dt, dx, dx, GAMMA, 40)
    s0 = oracle.plane_sums(Q0)
    s1 = oracle.plane_sums(out)
    scale = np.abs(Q0).reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) / scale < 1e-13), (s1 - s0) / scale


def _swap_axes(Q):
    return np.stack([Q[0].T, Q[2].T, Q[1].T, Q[3].T]).copy()


def test_transpose_symmetry_exact_1d():
    """A state varying only along x (with both velocity components nonzero) has zero
    y-flux differences, so swapping x with y (transpose, exchange rho u and rho v)
    must commute with the scheme bit for bit: pins the G flux against the F flux."""
    n = 32
    x = problems.cell_centres(n, 10.0)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x / 10) + 0.1 * np.cos(6 * np.pi * x / 10)
    u = 0.5 + 0.2 * np.cos(2 * np.pi * x / 10)
    v = -0.7 + 0.1 * np.sin(4 * np.pi * x / 10)
    p = 1.0 + 0.4 * np.cos(2 * np.pi * x / 10 + 0.3)
    Q0 = np.stack([np.tile(c[None, :], (n, 1)) for c in cons(rho, u, v, p)])
    dx = 10 / n
    a = oracle.euler_run(Q0, 0.01, dx, dx, GAMMA, 6)
    b = oracle.euler_run(_swap_axes(Q0), 0.01, dx, dx, GAMMA, 6)
    assert np.array_equal(a, _swap_axes(b))
    assert np.abs(a - Q0).max() > 1e-3
    assert np.array_equal(a, a[:, :1, :].repeat(n, axis=1))  # still independent of y


def test_transpose_symmetry_2d_one_step():
    """The same symmetry for a genuinely 2D state, one step, up to rounding (a pressure-ratio
    limiter switch can flip on a rounding difference, so longer runs diverge slowly)."""
    n = 32
    Q0 = problems.shu_vortex(n, centre=(4.3, 5.6), u_inf=0.7, v_inf=-0.2)
    dx = 10 / n
    a = oracle.euler_run(Q0, 0.01, dx, dx, GAMMA, 1)
    b = oracle.euler_run(_swap_axes(Q0), 0.01, dx, dx, GAMMA, 1)
    assert np.abs(a - _swap_axes(b)).max() < 1e-12
    assert np.abs(a - Q0).max() > 1e-4


def test_vortex_translates_at_45_degrees():
    """E2 / P4: the vortex is advected by the free stream (1, 1).  The L1 density error
    against the exact vortex translated by (t, t) falls with N at about first order
    (the pressure-ratio limiter acts on all four variables, so velocities are limited
    near pressure extrema; a per-variable minmod would reach ~1.5) and is far below
    the error against the vortex moved the wrong way."""
    t_end = 1.0
    errs = []
    for n in (32, 64, 128):
        Q0 = problems.shu_vortex(n)
        dx = 10 / n
        dt0 = oracle.cfl_dt(Q0, dx, dx, GAMMA, 0.4)
        steps = int(math.ceil(t_end / dt0))
        dt = t_end / steps
        out = oracle.euler_run(Q0, dt, dx, dx, GAMMA, steps)
        exact = problems.shu_vortex(n, centre=(5.0 + t_end, 5.0 + t_end))
        wrong = problems.shu_vortex(n, centre=(5.0 + t_end, 5.0 - t_end))
        errs.append(np.abs(out[0] - exact[0]).mean())
        assert np.abs(out[0] - wrong[0]).mean() > 5 * errs[-1]
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[2] < 1.5e-3
    assert min(orders) > 0.9, (errs, orders)


def _density_wave_at_rest(n):
    """Fluid at rest at constant pressure (E = 2.5, so p = 1) with a density wave that
    depends on the integer cell index, so every density extremum sits on a cell centre and
    no two neighbours are equal.  The momenta stay exactly zero and E exactly constant, so
    every pressure jump is exactly zero, every pressure ratio is 0/0 and the spatial operator
    is the first-order Rusanov form at every stage: the density diffuses with the speed
    s = max(c_L, c_R) and only the time rule changes with dt."""
    i = np.arange(n)
    rho = 1 + 0.3 * np.cos(2 * np.pi * (i[None, :] - 3) / n) + 0.2 * np.cos(4 * np.pi * (i[:, None] - 5) / n)
    return np.stack([rho, 0 * rho, 0 * rho, np.full_like(rho, 2.5)])


def _time_self_convergence(run, n=32, t_end=1.0):
    """Density at t_end from runs of 20, 40, 80 and 160 steps; returns the ratios of
    successive differences (about 4 for a second-order time rule, 2 for a first-order one)."""
    outs = [run(t_end / m, m) for m in (20, 40, 80, 160)]
    d = [np.abs(outs[k][0] - outs[k + 1][0]).max() for k in range(3)]
    assert np.all(outs[-1][1] == 0) and np.all(outs[-1][3] == outs[-1][3][0, 0])  # at rest, p constant
    return [d[k] / d[k + 1] for k in range(2)]


@pytest.mark.parametrize("impl", ["c", "numpy"])
def test_rk2_is_second_order_in_time(impl):
    """App. B time integration (explicit midpoint): with the spatial operator fixed (every
    pressure ratio 0/0), successive halvings of dt shrink the differences about 4x."""
    n = 32
    dx = 10 / n
    Q0 = _density_wave_at_rest(n)
    run = oracle.euler_run if impl == "c" else numpy_ref.euler_run
    ratios = _time_self_convergence(lambda dt, m: run(Q0, dt, dx, dx, GAMMA, m))
    assert min(ratios) > 3.5, ratios


def test_time_order_check_rejects_forward_euler_stages():
    """Negative control: two forward-Euler half steps per step (a first-order rule built
    from the twin's own stage) shrink the differences only 2x and fail the check above."""
    n = 32
    dx = 10 / n
    Q0 = _density_wave_at_rest(n)

    def fe_run(dt, m):
        Q = Q0.copy()
        h = 0.5 * dt / dx
        for _ in range(m):
            Qs = numpy_ref.euler_stage(Q, Q, h, h, np.float64(GAMMA))
            Q = numpy_ref.euler_stage(Qs, Qs, h, h, np.float64(GAMMA))
        return Q

    ratios = _time_self_convergence(fe_run)
    assert max(ratios) < 2.5, ratios


def _velocities_by_reciprocal(monkeypatch):
    """Plants, in the numpy twin only, the other rounding of the same equation of state and
    flux: velocities as momentum times fl(1/rho) instead of the plain quotient m/rho."""

    def pressure(Q, gm1):
        inv = Q.dtype.type(1) / Q[0]
        return gm1 * (Q[3] - Q.dtype.type(0.5) * (Q[1] * (Q[1] * inv) + Q[2] * (Q[2] * inv)))

    def phys_flux(Q, a, gamma, gm1):
        b = 2 if a == 1 else 1
        inv = Q.dtype.type(1) / Q[0]
        ua, ub = Q[a] * inv, Q[b] * inv
        p = gm1 * (Q[3] - Q.dtype.type(0.5) * (Q[a] * ua + Q[b] * ub))
        F = np.empty_like(Q)
        F[0], F[a], F[b], F[3] = Q[a], Q[a] * ua + p, Q[a] * ub, (Q[3] + p) * ua
        return F, np.abs(ua) + np.sqrt(gamma * p * inv)

    monkeypatch.setattr(numpy_ref, "_pressure", pressure)
    monkeypatch.setattr(numpy_ref, "_phys_flux", phys_flux)


def test_pressure_rounding_flips_the_limiter_on_the_vortex_centre_lines(monkeypatch):
    """The vortex's pressure is mirror-symmetric about x = 5 and y = 5, which are faces for
    even N: across them the pressure jump is zero up to rounding, so its sign -- and with it
    whether the limiter is on -- is decided by how p is rounded, and the face state moves by
    half the momentum jump.  One step with velocities rounded as m*fl(1/rho) instead of m/rho
    therefore moves the result by far more than the 1e-10 parity tolerance, and the largest
    changes sit next to the centre lines.  Pins the plain quotients of the equation of state:
    any re-rounding of the oracle fails this test."""
    n = 256
    dx = 10 / n
    Q0 = problems.shu_vortex(n)
    dt = oracle.cfl_dt(Q0, dx, dx, GAMMA, 0.4)
    plain = oracle.euler_run(Q0, dt, dx, dx, GAMMA, 1)
    assert np.array_equal(plain, numpy_ref.euler_run(Q0, dt, dx, dx, GAMMA, 1))
    _velocities_by_reciprocal(monkeypatch)
    other = numpy_ref.euler_run(Q0, dt, dx, dx, GAMMA, 1)
    rel = np.abs(plain - other) / np.abs(plain).max(axis=(1, 2))[:, None, None]
    assert rel.max() > 1e-6, rel.max()
    centre = {n // 2 - 1, n // 2}
    for k in range(4):
        j, i = np.unravel_index(np.argmax(rel[k]), rel[k].shape)
        assert j in centre or i in centre, (k, j, i)


def test_cfl_uniform_closed_form():
    Q = problems.uniform_state(8, rho=1.0, u=1.0, v=1.0, p=1.0)
    c = math.sqrt(GAMMA)
    dx, dy = 0.1, 0.2
    exp = 0.4 / ((1 + c) / dx + (1 + c) / dy)
    assert abs(oracle.cfl_dt(Q, dx, dy, GAMMA, 0.4) - exp) < 1e-17


def test_vortex_c4_facts():
    """Initial-state facts of the 2048^2 vortex: min rho, min p and the CFL-0.4 time step."""
    Q = problems.shu_vortex(2048)
    rho = Q[0]
    p = (GAMMA - 1) * (Q[3] - 0.5 * (Q[1] ** 2 + Q[2] ** 2) / rho)
    assert abs(rho.min() - 0.493812) < 1e-6
    assert abs(p.min() - 0.372380) < 1e-6
    dt = oracle.cfl_dt(Q, 10 / 2048, 10 / 2048, GAMMA, 0.4)
    assert abs(dt - 3.621859e-4) < 1e-9


def test_plane_sums_vs_fsum():
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((4, 64, 64))
    s = oracle.plane_sums(Q)
    for c in range(4):
        exact = math.fsum(Q[c].ravel())
        assert abs(s[c] - exact) <= 64 * 64 * 2.3e-16 * np.abs(Q[c]).sum()
