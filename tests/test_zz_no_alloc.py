"""swept_cfl_dt_noalloc: the CFL time step with the library's static device
scratch, against swept_cfl_dt with a caller-provided workspace.

Both run the same reduction kernels in the same order, so the time steps must
be equal bit for bit; two calls in a row (the second on a smaller grid) check
that the shared scratch carries nothing from one call to the next."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_2105_10332_amd import problems
from paper_2105_10332_amd._lib import CODES, EULER, F32, F64, Problem, lib


def _problem(n: int, dtype: int) -> Problem:
    return Problem(EULER, dtype, n, n, 10.0, 10.0, 1.0, 1.0, 1.4, 0, 0, 0.0)


def test_noalloc_rejects_oversized_grid_before_any_hip_call():
    p = _problem(65536, F64)
    out = ctypes.c_double(0.0)
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib().swept_cfl_dt_noalloc(ctypes.byref(p), fake, 0.4, None, ctypes.byref(out)) == CODES["SWEPT_ESHAPE"]
    assert lib().swept_cfl_dt_noalloc(None, fake, 0.4, None, ctypes.byref(out)) == CODES["SWEPT_EINVAL"]


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [F64, F32])
def test_noalloc_cfl_equals_workspace_cfl_twice(dtype):
    import torch

    dev = torch.device("cuda", 0)
    tdt = torch.float64 if dtype == F64 else torch.float32
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, eps in ((512, 5.0), (128, 3.0)):  # the second call on a smaller grid
        q = torch.tensor(problems.shu_vortex(n, eps=eps), device=dev, dtype=tdt)
        p = _problem(n, dtype)
        need = ctypes.c_size_t(0)
        assert lib().swept_workspace_bytes(ctypes.byref(p), None, ctypes.byref(need)) == 0
        work = torch.empty(need.value, dtype=torch.uint8, device=dev)
        ref = ctypes.c_double(0.0)
        rc = lib().swept_cfl_dt(ctypes.byref(p), ctypes.c_void_p(q.data_ptr()), 0.4, ctypes.c_void_p(work.data_ptr()),
                                need.value, stream, ctypes.byref(ref))
        assert rc == 0, lib().swept_last_error()
        del work
        got = ctypes.c_double(0.0)
        rc = lib().swept_cfl_dt_noalloc(ctypes.byref(p), ctypes.c_void_p(q.data_ptr()), 0.4, stream,
                                        ctypes.byref(got))
        assert rc == 0, lib().swept_last_error()
        print(f"cfl n={n} dtype={dtype}: workspace {ref.value!r} static {got.value!r}", flush=True)
        assert np.float64(got.value).tobytes() == np.float64(ref.value).tobytes()
        assert got.value > 0
