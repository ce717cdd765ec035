"""GPU parity of the heat path (through the C ABI): Swept == Standard bit for bit,
both against the oracle (FP64 within 1e-10 normwise; FP32 against the FP32
oracle and, as a stated error, against the FP64 one)."""
import math

import numpy as np
import pytest

import oracle
from paper_2105_10332_amd import problems

from gpu_helpers import DEV, heat_gpu, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile,N", [(8, 16), (8, 40), (16, 32), (16, 48), (32, 64), (32, 96), (64, 128), (6, 18),
                                    (12, 36), (4, 8), (4, 12)])
def test_swept_equals_standard_and_oracle(dtype, tile, N):
    h = tile // 2
    T0 = problems.heat_sine_noise(N, seed=tile + N).astype(dtype)
    for steps in sorted({1, h - 1, h, h + 1, 3 * h + 5}):
        sw, r = heat_gpu(T0, 0.2, steps, tile, "swept")
        st, _ = heat_gpu(T0, 0.2, steps, tile, "standard")
        assert np.array_equal(sw, st), (tile, N, steps)
        ref = oracle.heat_run(T0, r, steps)
        if dtype == np.float64:
            assert rel_err(sw, ref) <= 1e-10
        else:
            assert rel_err(sw, ref) <= 1e-6


@pytest.mark.parametrize("bc,bcv", [(1, 0.0), (1, 0.75), (2, 0.0)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile,N", [(8, 16), (16, 48), (32, 64), (64, 128), (12, 36), (4, 12)])
def test_boundaries_swept_equals_standard_and_oracle(bc, bcv, dtype, tile, N):
    """Dirichlet (ghost cells at bcv) and zero-flux walls: Swept == Standard bit for bit and
    both equal to the oracle with the same boundary, over partial and several windows."""
    h = tile // 2
    T0 = problems.heat_sine_noise(N, seed=tile + N).astype(dtype)
    for steps in sorted({1, h, h + 1, 3 * h + 5}):
        sw, r = heat_gpu(T0, 0.2, steps, tile, "swept", bc=bc, bcv=bcv)
        st, _ = heat_gpu(T0, 0.2, steps, tile, "standard", bc=bc, bcv=bcv)
        assert np.array_equal(sw, st), (bc, tile, N, steps)
        ref = oracle.heat_run(T0, r, steps, bc=bc, bcv=bcv)
        assert rel_err(sw, ref) <= (1e-10 if dtype == np.float64 else 1e-6)
        if steps > 1:
            assert rel_err(ref, oracle.heat_run(T0, r, steps)) > 1e-6  # the walls matter


@pytest.mark.parametrize("bc", [1, 2])
def test_boundaries_closed_form_4096(bc):
    """4096^2 FP64, tile 64, 1000 steps: the discrete eigenmode of the walled operator
    (Dirichlet 0: sin(pi p (i+1)/(N+1)); zero flux: cos(pi p (i+1/2)/N)) decays by its
    closed-form factor G^M, sampled over the whole grid."""
    N, M, p, q = 4096, 1000, 3, 5
    i = np.arange(N)
    if bc == 1:
        fx, fy = np.sin(np.pi * p * (i + 1) / (N + 1)), np.sin(np.pi * q * (i + 1) / (N + 1))
        lam = 4 * (np.sin(np.pi * p / (2 * (N + 1))) ** 2 + np.sin(np.pi * q / (2 * (N + 1))) ** 2)
    else:
        fx, fy = np.cos(np.pi * p * (i + 0.5) / N), np.cos(np.pi * q * (i + 0.5) / N)
        lam = 4 * (np.sin(np.pi * p / (2 * N)) ** 2 + np.sin(np.pi * q / (2 * N)) ** 2)
    T0 = np.outer(fy, fx)
    sw, r = heat_gpu(T0, 0.2, M, 64, "swept", bc=bc)
    exp = (1 - r * lam) ** M * T0
    err = rel_err(sw, exp)
    print(f"walls bc={bc} 4096^2 closed form: {err:.2e}")
    assert err <= 1e-12


def test_c1_config_fp64():
    """64^2, FP64, r = 0.2, 100 steps, sin sin + noise, 16x16 tiles (both solvers)."""
    T0 = problems.heat_sine_noise(64)
    sw, r = heat_gpu(T0, 0.2, 100, 16, "swept")
    st, _ = heat_gpu(T0, 0.2, 100, 16, "standard")
    ref = oracle.heat_run(T0, r, 100)
    assert np.array_equal(sw, st)
    err = rel_err(sw, ref)
    print(f"C1 fp64 swept vs oracle: {err:.3e}")
    assert err <= 1e-10


def test_fp32_matches_fp32_oracle_and_states_fp64_error():
    """FP32 swept vs the FP32 oracle (same operation order), and the stated FP32 error
    against the FP64 oracle on the C1 initial state (a slowly decaying mode + noise)."""
    T0 = problems.heat_sine_noise(128)
    sw, r = heat_gpu(T0.astype(np.float32), 0.2, 300, 32, "swept")
    o32 = oracle.heat_run(T0.astype(np.float32), r, 300)
    o64 = oracle.heat_run(T0, r, 300)
    assert rel_err(sw, o32) <= 1e-6
    e64 = rel_err(sw, o64)
    print(f"FP32 GPU vs FP64 oracle (128^2, 300 steps): {e64:.3e}")
    assert e64 < 1e-5


def test_zero_steps_is_identity():
    T0 = problems.heat_sine_noise(32)
    sw, _ = heat_gpu(T0, 0.2, 0, 16, "swept")
    assert np.array_equal(sw, T0)


def test_poisoned_workspace_and_determinism():
    """All-NaN workspace: a stale read would surface as NaN; two runs agree bitwise."""
    T0 = problems.heat_sine_noise(96, seed=5)
    a, _ = heat_gpu(T0, 0.24, 77, 32, "swept", poison=True)
    b, _ = heat_gpu(T0, 0.24, 77, 32, "swept", poison=True)
    st, _ = heat_gpu(T0, 0.24, 77, 32, "standard")
    assert np.isfinite(a).all()
    assert np.array_equal(a, b) and np.array_equal(a, st)


@pytest.mark.parametrize("wg", [64, 512, 1024])
def test_workgroup_sizes(wg):
    T0 = problems.heat_sine_noise(128, seed=wg)
    a, _ = heat_gpu(T0, 0.2, 41, 64, "swept", wg=wg)
    st, _ = heat_gpu(T0, 0.2, 41, 64, "standard")
    assert np.array_equal(a, st)


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_state_not_16_byte_aligned_is_rejected(dtype_name):
    """swept_init requires a 16-byte aligned state (and workspace): a state that starts one
    value into its allocation is rejected with SWEPT_EINVAL, one at its start is taken."""
    import torch

    from paper_2105_10332_amd._lib import SweptError
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    n = 256
    store = torch.zeros(n * n + 2, dtype=getattr(torch, dtype_name), device=DEV)
    with pytest.raises(SweptError, match="16-byte aligned"):
        SweptSolver(HEAT, store[1:1 + n * n].view(n, n), dt=0.2 / n / n, length=1.0, alpha=1.0, tile=64)
    s = SweptSolver(HEAT, store[:n * n].view(n, n), dt=0.2 / n / n, length=1.0, alpha=1.0, tile=64)
    s.close()


@pytest.mark.parametrize("wg", [256, 512, 1024])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("tile", [16, 32, 64])
def test_tiles_and_workgroups_equal_standard(tile, dtype, wg):
    """Every fixed-tile heat instantiation at 256, 512 and 1024 threads on 4 x 4 tiles (windows
    inside the domain and across its edge): runs that end inside the first window, after one
    and over several cycles equal the Standard path bit for bit."""
    n, h = 4 * tile, tile // 2
    T0 = problems.heat_sine_noise(n, seed=tile + wg).astype(dtype)
    for steps in sorted({1, h // 4, h // 4 + 1, h - 1, h + 1, 2 * h + 5, 4 * h + 3}):
        sw, _ = heat_gpu(T0, 0.2, steps, tile, "swept", wg=wg)
        st, _ = heat_gpu(T0, 0.2, steps, tile, "standard")
        assert np.array_equal(sw, st), (tile, wg, steps)


@pytest.mark.parametrize("dtype,tile", [(np.float64, 16), (np.float64, 32), (np.float64, 64), (np.float32, 32)])
def test_c2_full_size_closed_form(dtype, tile):
    """4096^2, r = 0.2, 1000 steps, 16 Fourier modes: Swept equals Standard, and sampled
    cells equal the exact discrete solution sum a G^M cos(...) (P2)."""
    n, M = 4096, 1000
    modes = problems.fourier_modes(problems.SEED_HEAT_MODES)
    T0 = modes.field(n).astype(dtype)
    sw, r = heat_gpu(T0, 0.2, M, tile, "swept")
    if tile == 32:
        st, _ = heat_gpu(T0, 0.2, M, tile, "standard")
        assert np.array_equal(sw, st)
    G = np.array([1 - 4 * r * (math.sin(math.pi * p / n) ** 2 + math.sin(math.pi * q / n) ** 2)
                  for p, q in zip(modes.p, modes.q)])
    rng = np.random.default_rng(9)
    js, is_ = rng.integers(0, n, 400), rng.integers(0, n, 400)
    x = (np.arange(n) + 0.5) / n
    exact = np.zeros(400)
    for p, q, a, ph, g in zip(modes.p, modes.q, modes.a, modes.phi, G):
        exact += a * g ** M * np.cos(2 * math.pi * (p * x[is_] + q * x[js]) + ph)
    err = np.abs(sw[js, is_] - exact).max() / np.abs(T0).max()
    print(f"C2 {np.dtype(dtype).name} b={tile}: closed-form error {err:.3e}")
    assert err < (1e-12 if dtype == np.float64 else 2e-5)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_largest_grid_closed_form(dtype):
    """The largest grid the library accepts (32768^2: 2^30 cells, 8 GiB of FP64 state, byte
    offsets past 2^32), tile 64, a step count that ends mid-window: Swept equals Standard
    and sampled cells equal the exact discrete solution of one Fourier mode (P1), which holds
    at any size."""
    import torch

    from gpu_helpers import DEV, TDT
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    n, M, r, tile = 32768, 37, 0.2, 64
    p, q, phase = 3, 5, 0.25
    x = (torch.arange(n, device=DEV, dtype=torch.float64) + 0.5) / n
    T0 = torch.cos(2 * math.pi * (p * x[None, :] + q * x[:, None]) + phase).to(TDT[dtype])
    T = T0.clone()
    dx = 1.0 / n
    s = SweptSolver(HEAT, T, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile)
    s.swept_advance(M)
    r_used = s.info.r
    s.close()
    del s
    Ts = T0.clone()
    s = SweptSolver(HEAT, Ts, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile)
    s.standard_advance(M)
    torch.cuda.synchronize()
    s.close()
    del s
    assert torch.equal(T, Ts)
    del Ts
    rng = np.random.default_rng(11)
    js, is_ = rng.integers(0, n, 400), rng.integers(0, n, 400)
    got = T[torch.tensor(js, device=DEV), torch.tensor(is_, device=DEV)].double().cpu().numpy()
    g = 1 - 4 * r_used * (math.sin(math.pi * p / n) ** 2 + math.sin(math.pi * q / n) ** 2)
    xs = (np.arange(n) + 0.5) / n
    exact = g ** M * np.cos(2 * math.pi * (p * xs[is_] + q * xs[js]) + phase)
    err = np.abs(got - exact).max()
    print(f"{n}^2 {np.dtype(dtype).name}: closed-form error {err:.3e}")
    assert err < (1e-13 if dtype == np.float64 else 1e-5)


@pytest.mark.parametrize("bc", [1, 2])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_largest_grid_walls_closed_form(bc, dtype):
    """Walls at the largest grid (32768^2, tile 64, 37 steps ending mid-window): Swept equals
    Standard, and sampled cells (including the four edges) equal the walled operator's
    eigenmode decay G^M: sin(pi p (i+1)/(N+1)) for Dirichlet 0, cos(pi p (i+1/2)/N) for zero
    flux."""
    import torch

    from gpu_helpers import DEV, TDT
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    n, M, r, tile, p, q = 32768, 37, 0.2, 64, 3, 5
    i = torch.arange(n, device=DEV, dtype=torch.float64)
    if bc == 1:
        fx, fy = torch.sin(math.pi * p * (i + 1) / (n + 1)), torch.sin(math.pi * q * (i + 1) / (n + 1))
    else:
        fx, fy = torch.cos(math.pi * p * (i + 0.5) / n), torch.cos(math.pi * q * (i + 0.5) / n)
    T0 = (fy[:, None] * fx[None, :]).to(TDT[dtype])
    del i, fx, fy
    T = T0.clone()
    dx = 1.0 / n
    s = SweptSolver(HEAT, T, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile, boundary=bc)
    s.swept_advance(M)
    r_used = s.info.r
    s.close()
    del s
    Ts = T0.clone()
    s = SweptSolver(HEAT, Ts, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile, boundary=bc)
    s.standard_advance(M)
    torch.cuda.synchronize()
    s.close()
    del s
    assert torch.equal(T, Ts)
    del Ts, T0
    rng = np.random.default_rng(12)
    js = np.concatenate([rng.integers(0, n, 300), [0, n - 1, 0, n - 1, 7, n - 3]])
    is_ = np.concatenate([rng.integers(0, n, 300), [0, n - 1, n - 1, 0, n - 1, 0]])
    got = T[torch.tensor(js, device=DEV), torch.tensor(is_, device=DEV)].double().cpu().numpy()
    if bc == 1:
        lam = 4 * (math.sin(math.pi * p / (2 * (n + 1))) ** 2 + math.sin(math.pi * q / (2 * (n + 1))) ** 2)
        mode = np.sin(np.pi * q * (js + 1) / (n + 1)) * np.sin(np.pi * p * (is_ + 1) / (n + 1))
    else:
        lam = 4 * (math.sin(math.pi * p / (2 * n)) ** 2 + math.sin(math.pi * q / (2 * n)) ** 2)
        mode = np.cos(np.pi * q * (js + 0.5) / n) * np.cos(np.pi * p * (is_ + 0.5) / n)
    err = np.abs(got - (1 - r_used * lam) ** M * mode).max()
    print(f"walls bc={bc} {n}^2 {np.dtype(dtype).name}: closed-form error {err:.3e}")
    assert err < (1e-13 if dtype == np.float64 else 1e-5)


def test_nonfinite_state_is_reported():
    """swept_conserved reports a non-finite plane sum as SWEPT_ENONFINITE (after a swept
    advance has spread a NaN), instead of returning it as a number."""
    import torch

    from gpu_helpers import DEV
    from paper_2105_10332_amd._lib import SweptError
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    T = torch.tensor(problems.heat_sine_noise(32), device=DEV)
    s = SweptSolver(HEAT, T, dt=0.2 / 32 / 32, length=1.0, alpha=1.0, tile=8)
    assert math.isfinite(s.swept_conserved()[0])
    T[5, 7] = float("nan")
    s.swept_advance(3)
    with pytest.raises(SweptError) as ei:
        s.swept_conserved()
    assert ei.value.name == "SWEPT_ENONFINITE"
    s.close()


@pytest.mark.parametrize("method", ["swept", "standard"])
def test_advance_replays_from_a_hip_graph(method):
    """An advance captured once in a graph (torch.cuda.CUDAGraph on the library's stream) and
    replayed three times, with eager work in between, equals the eager advance each time."""
    import torch

    from gpu_helpers import DEV
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    N, M, tile = 96, 37, 32
    T0 = problems.heat_sine_noise(N, seed=9)
    x = torch.tensor(T0, device=DEV)
    y = torch.empty_like(x)
    dt = 0.2 / N / N
    a = SweptSolver(HEAT, x, dt=dt, length=1.0, alpha=1.0, tile=tile)
    b = SweptSolver(HEAT, y, dt=dt, length=1.0, alpha=1.0, tile=tile)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm the kernels before capture
        getattr(a, method + "_advance")(1)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        getattr(a, method + "_advance")(M)
    for _ in range(3):
        y.copy_(x)
        g.replay()
        getattr(b, method + "_advance")(M)
        torch.cuda.synchronize()
        assert torch.equal(x, y)
    a.close()
    b.close()
