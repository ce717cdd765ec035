"""Python face of libswept: device memory from PyTorch, everything else in HIP.

``SweptSolver`` owns a caller-visible state tensor and the workspace tensor
and forwards to the C ABI with the same names (``swept_advance``,
``standard_advance``, ``swept_conserved`` ...).  The kernels run on the
current torch stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import EULER, F32, F64, HEAT, Info, Problem, Tuning, check, lib

_DT = {torch.float64: F64, torch.float32: F32}


def make_problem(kind: int, n: int, dtype: torch.dtype, dt: float, length: float, alpha: float = 1.0,
                 gamma: float = 1.4) -> Problem:
    return Problem(kind, _DT[dtype], n, n, float(length), float(length), float(dt), float(alpha), float(gamma))


def swept_workspace_bytes(prob: Problem, tile: int = 0, wg: int = 0) -> int:
    out = ctypes.c_size_t(0)
    check(lib().swept_workspace_bytes(ctypes.byref(prob), ctypes.byref(Tuning(tile, wg)), ctypes.byref(out)))
    return out.value


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("libswept takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("state must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class SweptSolver:
    """A swept/standard solver bound to one device state tensor (advanced in place).

    state: heat (N, N) or Euler (4, N, N) tensor on the GPU, float64 or float32.
    """

    def __init__(self, kind: int, state: torch.Tensor, dt: float, length: float = 1.0, alpha: float = 1.0,
                 gamma: float = 1.4, tile: int = 0, wg: int = 0):
        n = state.shape[-1]
        expect = (n, n) if kind == HEAT else (4, n, n)
        if tuple(state.shape) != expect:
            raise ValueError(f"state shape {tuple(state.shape)} != {expect}")
        self.kind = kind
        self.state = state
        self.prob = make_problem(kind, n, state.dtype, dt, length, alpha, gamma)
        nbytes = swept_workspace_bytes(self.prob, tile, wg)
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=state.device)
        self._ctx = ctypes.c_void_p(0)
        check(lib().swept_init(ctypes.byref(self._ctx), ctypes.byref(self.prob), ctypes.byref(Tuning(tile, wg)),
                               _dev_ptr(state), _dev_ptr(self.work), nbytes, _stream_ptr()))

    @property
    def info(self) -> Info:
        inf = Info()
        check(lib().swept_query(self._ctx, ctypes.byref(inf)))
        return inf

    def swept_advance(self, n_steps: int):
        check(lib().swept_set_stream(self._ctx, _stream_ptr()))
        check(lib().swept_advance(self._ctx, int(n_steps)))
        return self.state

    def standard_advance(self, n_steps: int):
        check(lib().swept_set_stream(self._ctx, _stream_ptr()))
        check(lib().standard_advance(self._ctx, int(n_steps)))
        return self.state

    def swept_conserved(self):
        nvar = 1 if self.kind == HEAT else 4
        out = (ctypes.c_double * nvar)()
        check(lib().swept_set_stream(self._ctx, _stream_ptr()))
        check(lib().swept_conserved(self._ctx, out))
        return list(out)

    def close(self):
        if self._ctx:
            lib().swept_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def swept_cfl_dt(state: torch.Tensor, length: float, cfl: float, gamma: float = 1.4) -> float:
    """Euler time step for a CFL number, reduced on the GPU (see swept.h)."""
    n = state.shape[-1]
    prob = make_problem(EULER, n, state.dtype, 1.0, length, gamma=gamma)
    nbytes = swept_workspace_bytes(prob)
    work = torch.empty(nbytes, dtype=torch.uint8, device=state.device)
    out = ctypes.c_double(0.0)
    check(lib().swept_cfl_dt(ctypes.byref(prob), _dev_ptr(state), float(cfl), _dev_ptr(work), nbytes,
                             _stream_ptr(), ctypes.byref(out)))
    return out.value


__all__ = ["SweptSolver", "swept_cfl_dt", "swept_workspace_bytes", "make_problem", "HEAT", "EULER", "_lib"]
