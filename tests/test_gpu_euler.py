"""GPU parity of the Euler path (through the C ABI)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2105_10332_amd import problems
from paper_2105_10332_amd.solver import EULER, SweptSolver, swept_cfl_dt

from gpu_helpers import DEV, euler_gpu, rel_err

pytestmark = pytest.mark.gpu
GAMMA = 1.4


def _dt(Q0, n, length=10.0):
    dx = length / n
    return oracle.cfl_dt(Q0, dx, dx, GAMMA, 0.4)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile,N", [(8, 16), (8, 24), (16, 32), (16, 48), (32, 64), (12, 36)])
def test_swept_equals_standard_and_oracle(dtype, tile, N):
    Q0 = problems.shu_vortex(N)
    dt = _dt(Q0, N)
    Q0 = Q0.astype(dtype)
    h = tile // 4
    for steps in sorted({1, max(1, h // 2), h, h + 1, 2 * h + 3}):
        sw = euler_gpu(Q0, dt, steps, tile, "swept")
        st = euler_gpu(Q0, dt, steps, tile, "standard")
        assert np.array_equal(sw, st), (tile, N, steps)
        ref = oracle.euler_run(Q0, dt, 10.0 / N, 10.0 / N, GAMMA, steps)
        err = rel_err(sw, ref)
        assert err <= (1e-10 if dtype == np.float64 else 1e-5), err


@pytest.mark.parametrize("wg", [128, 512, 1024])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile,N", [(16, 48), (32, 96)])
def test_workgroup_sizes(wg, dtype, tile, N):
    """Every workgroup size up to the 1024-thread launch bound gives the Standard result."""
    Q0 = problems.shu_vortex(N)
    dt = _dt(Q0, N)
    Q0 = Q0.astype(dtype)
    steps = 2 * (tile // 4) + 3
    sw = euler_gpu(Q0, dt, steps, tile, "swept", wg=wg)
    st = euler_gpu(Q0, dt, steps, tile, "standard")
    assert np.array_equal(sw, st), (wg, tile, N)


@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile,N", [(8, 24), (16, 48), (32, 64)])
def test_scheme_variants_swept_equals_standard_and_oracle(scheme, dtype, tile, N):
    """The limiter-as-printed and Roe-speed variants: Swept == Standard bit for bit and
    both match the oracle run with the same variant bits."""
    Q0 = problems.shu_vortex(N)
    dt = _dt(Q0, N)
    Q0 = Q0.astype(dtype)
    h = tile // 4
    for steps in sorted({1, h + 1, 2 * h + 3}):
        sw = euler_gpu(Q0, dt, steps, tile, "swept", scheme=scheme)
        st = euler_gpu(Q0, dt, steps, tile, "standard", scheme=scheme)
        assert np.array_equal(sw, st), (scheme, tile, N, steps)
        ref = oracle.euler_run(Q0, dt, 10.0 / N, 10.0 / N, GAMMA, steps, scheme=scheme)
        err = rel_err(sw, ref)
        assert err <= (1e-10 if dtype == np.float64 else 1e-5), err
        if dtype == np.float64 and steps > 1:
            assert rel_err(ref, oracle.euler_run(Q0, dt, 10.0 / N, 10.0 / N, GAMMA, steps)) > 1e-12


@pytest.mark.parametrize("bc", [2, 3])
@pytest.mark.parametrize("scheme", [0, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile,N", [(8, 16), (8, 24), (16, 48), (32, 64), (12, 36)])
def test_walls_swept_equals_standard_and_oracle(bc, scheme, dtype, tile, N):
    """Zero-gradient (2) and slip (3) walls on the vortex: Swept == Standard bit for bit and
    both equal the walled oracle (FP64 within 1e-10, FP32 within 1e-5)."""
    Q0 = problems.shu_vortex(N)
    dt = _dt(Q0, N)
    Q0 = Q0.astype(dtype)
    h = tile // 4
    for steps in sorted({1, h + 1, 2 * h + 3, 9}):
        sw = euler_gpu(Q0, dt, steps, tile, "swept", scheme=scheme, bc=bc)
        st = euler_gpu(Q0, dt, steps, tile, "standard", scheme=scheme, bc=bc)
        assert np.array_equal(sw, st), (bc, scheme, tile, N, steps)
        ref = oracle.euler_run(Q0, dt, 10.0 / N, 10.0 / N, GAMMA, steps, scheme=scheme, bc=bc)
        err = rel_err(sw, ref)
        assert err <= (1e-10 if dtype == np.float64 else 1e-5), (err, steps)


@pytest.mark.parametrize("bc", [2, 3])
@pytest.mark.parametrize("scheme", [0, 3])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_walls_with_1024_thread_workgroups(bc, scheme, dtype):
    """The walled instantiations at the 1024-thread launch bound (tile 32, 96^2, 19 steps):
    Swept == Standard bit for bit and both equal the walled oracle."""
    N, tile, steps = 96, 32, 19
    Q0 = problems.shu_vortex(N)
    dt = _dt(Q0, N)
    Q0 = Q0.astype(dtype)
    sw = euler_gpu(Q0, dt, steps, tile, "swept", scheme=scheme, bc=bc, wg=1024)
    st = euler_gpu(Q0, dt, steps, tile, "standard", scheme=scheme, bc=bc)
    assert np.array_equal(sw, st), (bc, scheme)
    ref = oracle.euler_run(Q0, dt, 10.0 / N, 10.0 / N, GAMMA, steps, scheme=scheme, bc=bc)
    assert rel_err(sw, ref) <= (1e-10 if dtype == np.float64 else 1e-5)


def test_slip_walls_conserve_mass_and_energy_on_gpu():
    """128^2 vortex against slip walls, 60 steps: the FP64 sums of rho and E stay constant
    to roundoff (a slip wall passes neither), the x momentum does not."""
    Q0 = problems.shu_vortex(128)
    dt = _dt(Q0, 128)
    Q = torch.tensor(Q0, device=DEV)
    s = SweptSolver(EULER, Q, dt=dt, length=10.0, gamma=GAMMA, tile=16, boundary=3)
    s0 = np.array(s.swept_conserved())
    s.swept_advance(60)
    s1 = np.array(s.swept_conserved())
    s.close()
    scale = np.abs(Q0).reshape(4, -1).sum(axis=1)
    assert abs(s1[0] - s0[0]) / scale[0] < 1e-12 and abs(s1[3] - s0[3]) / scale[3] < 1e-12
    assert abs(s1[1] - s0[1]) / scale[1] > 1e-6


def test_poisoned_workspace_and_determinism():
    Q0 = problems.shu_vortex(64)
    dt = _dt(Q0, 64)
    a = euler_gpu(Q0, dt, 13, 16, "swept", poison=True)
    b = euler_gpu(Q0, dt, 13, 16, "swept", poison=True)
    st = euler_gpu(Q0, dt, 13, 16, "standard")
    assert np.isfinite(a).all() and np.array_equal(a, b) and np.array_equal(a, st)


def test_conservation_on_gpu():
    Q0 = problems.shu_vortex(128)
    dt = _dt(Q0, 128)
    Q = torch.tensor(Q0, device=DEV)
    s = SweptSolver(EULER, Q, dt=dt, length=10.0, gamma=GAMMA, tile=16)
    s0 = np.array(s.swept_conserved())
    assert np.allclose(s0, oracle.plane_sums(Q0), rtol=1e-13, atol=0)
    s.swept_advance(60)
    s1 = np.array(s.swept_conserved())
    scale = np.abs(Q0).reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(s1 - s0) / scale < 1e-12)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_cfl_dt_matches_oracle_bitwise(dtype):
    Q0 = problems.shu_vortex(256).astype(dtype)
    dt_gpu = swept_cfl_dt(torch.tensor(Q0, device=DEV), 10.0, 0.4)
    dt_cpu = oracle.cfl_dt(Q0, 10 / 256, 10 / 256, GAMMA, 0.4)
    assert dt_gpu == dt_cpu


def test_c4_full_size_short_run_vs_oracle():
    """2048^2 vortex, FP64, CFL 0.4: 3 steps against the oracle, Swept == Standard."""
    n = 2048
    Q0 = problems.shu_vortex(n)
    dt = swept_cfl_dt(torch.tensor(Q0, device=DEV), 10.0, 0.4)
    assert abs(dt - 3.621859e-4) < 1e-9
    sw = euler_gpu(Q0, dt, 3, 16, "swept")
    st = euler_gpu(Q0, dt, 3, 16, "standard")
    assert np.array_equal(sw, st)
    ref = oracle.euler_run(Q0, dt, 10 / n, 10 / n, GAMMA, 3)
    assert rel_err(sw, ref) <= 1e-10


def _vortex_gpu(n, dtype, length=10.0, eps=5.0, gamma=GAMMA, rows=4096):
    """The isentropic vortex of problems.shu_vortex built on the GPU in row blocks (input only)."""
    import math

    x = (torch.arange(n, device=DEV, dtype=torch.float64) + 0.5) * (length / n) - 5.0
    Q = torch.empty((4, n, n), dtype=dtype, device=DEV)
    for j0 in range(0, n, rows):
        Y = x[j0:j0 + rows, None]
        X = x[None, :]
        r2 = X * X + Y * Y
        e = torch.exp(0.5 * (1.0 - r2))
        u = 1.0 - eps / (2 * math.pi) * Y * e
        v = 1.0 + eps / (2 * math.pi) * X * e
        T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * torch.exp(1.0 - r2)
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        Q[0, j0:j0 + rows] = rho
        Q[1, j0:j0 + rows] = rho * u
        Q[2, j0:j0 + rows] = rho * v
        Q[3, j0:j0 + rows] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return Q


@pytest.mark.parametrize("scheme", [0, 3])
def test_largest_grid_sampled_cells(scheme):
    """The largest grid the library accepts (32768^2, FP32: 2^32 values over the four
    planes), in the FP32 launch configuration (b = 32, 512 threads), three steps, default
    scheme and both variant bits: Swept equals Standard bit for bit, and sampled cells in and
    around the vortex core equal the oracle run on a 40 x 40 periodic patch around each (a cell
    after three RK2 steps depends only on cells within 12 of it, so the patch's own wrap cannot
    reach the centre)."""
    n, M, tile, wg = 32768, 3, 32, 512
    dx = 10.0 / n
    dt = 0.4 * dx / 6.5  # below the CFL limit: (|u|+c) + (|v|+c) < 6.5 everywhere on this vortex
    Q0 = _vortex_gpu(n, torch.float32)
    Q = Q0.clone()
    s = SweptSolver(EULER, Q, dt=dt, length=10.0, gamma=GAMMA, tile=tile, wg=wg, scheme=scheme)
    s.swept_advance(M)
    s.close()
    del s
    Qs = Q0.clone()
    s = SweptSolver(EULER, Qs, dt=dt, length=10.0, gamma=GAMMA, tile=tile, wg=wg, scheme=scheme)
    s.standard_advance(M)
    torch.cuda.synchronize()
    s.close()
    del s
    assert torch.equal(Q, Qs)
    del Qs
    rng = np.random.default_rng(5)
    core = rng.integers(int(3.5 / dx), int(6.5 / dx), size=(6, 2))
    anywhere = rng.integers(0, n, size=(2, 2))
    scale = Q0.abs().amax(dim=(1, 2)).double().cpu().numpy()
    worst = 0.0
    for cy, cx in np.concatenate([core, anywhere]):
        iy = torch.tensor((np.arange(-20, 20) + cy) % n, device=DEV)
        ix = torch.tensor((np.arange(-20, 20) + cx) % n, device=DEV)
        patch = Q0[:, iy][:, :, ix].cpu().numpy()
        ref = oracle.euler_run(patch, dt, dx, dx, GAMMA, M, scheme=scheme)[:, 20, 20]
        got = Q[:, int(cy), int(cx)].cpu().numpy()
        worst = max(worst, float(np.max(np.abs(got.astype(np.float64) - ref) / scale)))
    print(f"Euler {n}^2 fp32 scheme {scheme} sampled cells vs oracle patches: {worst:.3e}")
    assert worst <= 1e-6


def test_cfl_rejects_nonphysical_state():
    """A state with negative pressure has no sound speed: swept_cfl_dt reports
    SWEPT_ENONFINITE rather than a time step."""
    from paper_2105_10332_amd._lib import SweptError

    Q = torch.tensor(problems.shu_vortex(32), device=DEV)
    Q[3, 10, 10] = 0.0  # E = 0 with nonzero momentum: p < 0
    with pytest.raises(SweptError) as ei:
        swept_cfl_dt(Q, 10.0, 0.4)
    assert ei.value.name == "SWEPT_ENONFINITE"
