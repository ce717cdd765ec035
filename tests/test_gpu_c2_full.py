"""The heat workload at its full size and length (4096^2 periodic, r = 0.2, 1000 steps,
16 seeded Fourier modes) in the launch configurations the benchmark times: FP64 tile 64
with 512 threads, FP32 tile 64 with 256.  Swept equals Standard bit for bit, each
precision equals the oracle run in that precision over the whole field (0 measured in
both), and the FP32 error against the FP64 oracle is stated (2.0e-6 measured)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2105_10332_amd import problems

from gpu_helpers import heat_gpu, rel_err

pytestmark = pytest.mark.gpu
N, STEPS, R = 4096, 1000, 0.2


@pytest.fixture(scope="module")
def c2():
    T0 = problems.heat_fourier_modes(N)
    print(f"C2 oracle: {N}^2, {STEPS} steps", flush=True)
    return T0, oracle.heat_run(T0, R, STEPS)


@pytest.mark.parametrize("dtype,tile,wg", [(np.float64, 64, 512), (np.float32, 64, 256)])
def test_c2_full_length_equals_oracle(c2, dtype, tile, wg):
    T0, ref64 = c2
    x0 = T0.astype(dtype)
    sw, r = heat_gpu(x0, R, STEPS, tile, "swept", wg=wg)
    if dtype == np.float64:
        assert r == R  # the r the kernels used is the oracle's
    st, _ = heat_gpu(x0, R, STEPS, tile, "standard", wg=wg)
    assert np.isfinite(sw).all()
    assert np.array_equal(sw, st)
    ref = ref64 if dtype == np.float64 else oracle.heat_run(x0, r, STEPS)
    err = rel_err(sw, ref)
    err64 = rel_err(sw, ref64)
    print(f"C2 {np.dtype(dtype).name} b={tile} wg={wg}: vs oracle of its precision {err:.3e}, "
          f"vs FP64 oracle {err64:.3e}")
    assert err <= (1e-10 if dtype == np.float64 else 1e-6)
    assert err64 <= (1e-10 if dtype == np.float64 else 1e-5)
