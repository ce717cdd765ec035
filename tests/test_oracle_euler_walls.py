"""Pins of the oracle's Euler walls (CPU only).

Slip walls (BC_REFLECT: ghost cells mirror the inside cells with the normal
momentum negated) and zero-gradient boundaries (BC_NEUMANN: ghost cells hold
the edge cell).  Pinned by what the walls must do exactly: a slip wall passes
no mass and no energy, so the mass and energy totals stay constant to
roundoff while the momentum normal to the walls does not; a fluid at rest
stays at rest; a uniform stream passes a zero-gradient boundary unchanged; a
state symmetric about the centre stays symmetric; and the independent numpy
twin agrees bit for bit."""
import numpy as np
import pytest

import oracle
from oracle import numpy_ref
from paper_2105_10332_amd import problems

GAMMA = 1.4
REF, ZG = oracle.BC_REFLECT, oracle.BC_NEUMANN


def _pulse(n, amp=0.4):
    """Fluid at rest with a Gaussian pressure and density bump at the centre of [0,10]^2."""
    x = (np.arange(n) + 0.5) * 10 / n
    r2 = (x[None, :] - 5) ** 2 + (x[:, None] - 5) ** 2
    bump = np.exp(-r2)
    rho = 1 + amp * bump
    p = 1 + amp * bump
    return np.stack([rho, 0 * rho, 0 * rho, p / (GAMMA - 1)])


def test_fluid_at_rest_stays_at_rest():
    Q0 = problems.uniform_state(24, rho=1.3, u=0.0, v=0.0, p=2.1)
    assert np.array_equal(oracle.euler_run(Q0, 1e-2, 10 / 24, 10 / 24, GAMMA, 8, bc=REF), Q0)
    assert np.array_equal(oracle.euler_run(Q0, 1e-2, 10 / 24, 10 / 24, GAMMA, 8, bc=ZG), Q0)


def test_uniform_stream_passes_zero_gradient_boundary():
    Q0 = problems.uniform_state(24, rho=1.3, u=0.7, v=-0.4, p=2.1)
    assert np.array_equal(oracle.euler_run(Q0, 1e-2, 10 / 24, 10 / 24, GAMMA, 8, bc=ZG), Q0)


@pytest.mark.parametrize("scheme", [0, 3])
def test_slip_walls_conserve_mass_and_energy(scheme):
    """The vortex pushed against slip walls: sum rho and sum E constant to roundoff, while
    the momenta change (the walls exert a force)."""
    n = 40
    Q0 = problems.shu_vortex(n)
    dx = 10 / n
    dt = oracle.cfl_dt(Q0, dx, dx, GAMMA, 0.4)
    out = oracle.euler_run(Q0, dt, dx, dx, GAMMA, 60, scheme=scheme, bc=REF)
    s0, s1 = oracle.plane_sums(Q0), oracle.plane_sums(out)
    scale = np.abs(Q0).reshape(4, -1).sum(axis=1)
    assert abs(s1[0] - s0[0]) / scale[0] < 1e-13 and abs(s1[3] - s0[3]) / scale[3] < 1e-13
    assert abs(s1[1] - s0[1]) / scale[1] > 1e-6  # the walls push back on the stream


def test_slip_walls_keep_mirror_symmetry():
    """A pressure bump at rest in the centre: the solution stays symmetric under
    x -> 10 - x (with rho u -> -rho u) and under y -> 10 - y (rho v -> -rho v).
    N is odd so that the mirror lines run through cell centres: with even N they are
    faces, where the mirrored pressure jump is zero up to rounding, and the left factor
    fl(1/fl(d+/d-)) and its mirror image fl(d-/d+) round differently, so the limiter
    branch there follows the rounding and the two halves drift apart at O(1e-2)."""
    n = 33
    Q0 = _pulse(n)
    dx = 10 / n
    out = oracle.euler_run(Q0, 0.02, dx, dx, GAMMA, 40, bc=REF)
    mx = out[:, :, ::-1].copy()
    mx[1] = -mx[1]
    my = out[:, ::-1, :].copy()
    my[2] = -my[2]
    scale = np.abs(out).max(axis=(1, 2))[:, None, None]
    assert np.abs(mx - out).max() / scale.max() < 1e-12
    assert np.abs(my - out).max() / scale.max() < 1e-12
    assert np.abs(out[1]).max() > 1e-3  # the bump did spread


@pytest.mark.parametrize("bc", [REF, ZG])
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_walls_c_matches_numpy_twin(bc, scheme, dtype):
    Q0 = problems.shu_vortex(32).astype(dtype)
    dx = 10 / 32
    a = oracle.euler_run(Q0, 0.02, dx, dx, GAMMA, 8, scheme=scheme, bc=bc)
    b = numpy_ref.euler_run(Q0, 0.02, dx, dx, GAMMA, 8, scheme=scheme, bc=bc)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, oracle.euler_run(Q0, 0.02, dx, dx, GAMMA, 8, scheme=scheme))
