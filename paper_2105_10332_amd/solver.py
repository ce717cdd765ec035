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
from ._lib import (BATCH_COOPERATIVE, BATCH_PER_PHASE, BC_DIRICHLET, BC_NEUMANN, BC_PERIODIC, BC_REFLECT, EULER, F32,
                   F64, HEAT, LIMITER_LITERAL, SPEED_ROE, Info, Problem, Tuning, check, lib)

_DT = {torch.float64: F64, torch.float32: F32}


def make_problem(kind: int, n: int, dtype: torch.dtype, dt: float, length: float, alpha: float = 1.0,
                 gamma: float = 1.4, scheme: int = 0, boundary: int = 0, boundary_value: float = 0.0) -> Problem:
    """scheme: Euler variant bits, LIMITER_LITERAL | SPEED_ROE (0 = minmod + Rusanov).
    boundary: BC_PERIODIC; heat BC_DIRICHLET (ghost cells hold boundary_value) or BC_NEUMANN (zero
    flux); Euler BC_NEUMANN (zero gradient) or BC_REFLECT (slip walls)."""
    return Problem(kind, _DT[dtype], n, n, float(length), float(length), float(dt), float(alpha), float(gamma),
                   int(scheme), int(boundary), float(boundary_value))


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
                 gamma: float = 1.4, tile: int = 0, wg: int = 0, scheme: int = 0, boundary: int = 0,
                 boundary_value: float = 0.0):
        n = state.shape[-1]
        expect = (n, n) if kind == HEAT else (4, n, n)
        if tuple(state.shape) != expect:
            raise ValueError(f"state shape {tuple(state.shape)} != {expect}")
        self.kind = kind
        self.state = state
        self.prob = make_problem(kind, n, state.dtype, dt, length, alpha, gamma, scheme, boundary, boundary_value)
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

    # ---- adjoint (heat) ----
    def swept_tape_bytes(self, n_steps: int) -> int:
        out = ctypes.c_size_t(0)
        check(lib().swept_tape_bytes(self._ctx, int(n_steps), ctypes.byref(out)))
        return out.value

    def new_tape(self, n_steps: int) -> torch.Tensor:
        return torch.empty(self.swept_tape_bytes(n_steps), dtype=torch.uint8, device=self.state.device)

    def swept_advance_checkpointed(self, n_steps: int, tape: torch.Tensor):
        check(lib().swept_set_stream(self._ctx, _stream_ptr()))
        check(lib().swept_advance_checkpointed(self._ctx, int(n_steps), _dev_ptr(tape), tape.numel()))
        return self.state

    def swept_adjoint(self, n_steps: int, tape: torch.Tensor, gTM: torch.Tensor, gT0: torch.Tensor) -> float:
        """Writes dJ/dT^0 into gT0 for dJ/dT^M = gTM; returns dJ/dalpha."""
        for t in (gTM, gT0):
            if t.dtype != self.state.dtype or t.shape != self.state.shape:
                raise ValueError("gradients must match the state's shape and dtype")
        out = ctypes.c_double(0.0)
        check(lib().swept_set_stream(self._ctx, _stream_ptr()))
        check(lib().swept_adjoint(self._ctx, int(n_steps), _dev_ptr(tape), tape.numel(), _dev_ptr(gTM),
                                  _dev_ptr(gT0), ctypes.byref(out)))
        return out.value

    def close(self):
        if self._ctx:
            lib().swept_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SweptHetero:
    """The GPU share of Eq. 2: a SweptSolver's advance split between the GPU (tile rows
    below the share) and host worker threads (the rest), see swept.h.  The solver must
    outlive this object."""

    def __init__(self, solver: SweptSolver, gpu_share: float, cpu_threads: int = 0):
        self.solver = solver
        self._h = ctypes.c_void_p(0)
        check(lib().swept_hetero_init(ctypes.byref(self._h), solver._ctx, float(gpu_share), int(cpu_threads)))

    def swept_hetero_advance(self, n_steps: int):
        check(lib().swept_set_stream(self.solver._ctx, _stream_ptr()))
        check(lib().swept_hetero_advance(self._h, int(n_steps)))
        return self.solver.state

    def query(self):
        """(GPU tile rows, host tile rows, host threads)."""
        g, c, t = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        check(lib().swept_hetero_query(self._h, ctypes.byref(g), ctypes.byref(c), ctypes.byref(t)))
        return g.value, c.value, t.value

    def close(self):
        if self._h:
            lib().swept_hetero_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SweptBatch:
    """Many problems (heat (N, N) and Euler (4, N, N) tensors, one dtype) advanced
    together by one persistent launch per swept_batch_advance (see swept.h).

    items: list of (kind, state, dt, length, alpha, gamma, tile), optionally followed by
    (scheme, boundary, boundary_value) as for SweptSolver."""

    def __init__(self, items):
        n = len(items)
        self.states = [it[1] for it in items]
        probs = (Problem * n)()
        tunes = (Tuning * n)()
        for q, (kind, st, dt, length, alpha, gamma, tile, *extra) in enumerate(items):
            scheme, boundary, boundary_value = (list(extra) + [0, 0, 0.0][len(extra):])[:3]
            probs[q] = make_problem(kind, st.shape[-1], st.dtype, dt, length, alpha, gamma, scheme, boundary,
                                    boundary_value)
            tunes[q] = Tuning(int(tile), 0)
        out = ctypes.c_size_t(0)
        check(lib().swept_batch_workspace_bytes(probs, tunes, n, ctypes.byref(out)))
        self.work = torch.empty(out.value, dtype=torch.uint8, device=self.states[0].device)
        ptrs = (ctypes.c_void_p * n)(*[_dev_ptr(st).value for st in self.states])
        self._ctx = ctypes.c_void_p(0)
        check(lib().swept_batch_init(ctypes.byref(self._ctx), probs, tunes, ptrs, n, _dev_ptr(self.work),
                                     out.value, _stream_ptr()))
        self.count = n

    def swept_batch_advance(self, n_steps: int):
        check(lib().swept_batch_set_stream(self._ctx, _stream_ptr()))
        check(lib().swept_batch_advance(self._ctx, int(n_steps)))

    def swept_batch_set_mode(self, mode: int):
        """BATCH_COOPERATIVE (one persistent launch, the default) or BATCH_PER_PHASE (one
        launch per global phase, for processes that cannot make cooperative launches)."""
        check(lib().swept_batch_set_mode(self._ctx, int(mode)))

    def info(self, q: int) -> Info:
        inf = Info()
        check(lib().swept_batch_query(self._ctx, q, ctypes.byref(inf)))
        return inf

    @property
    def grid(self) -> int:
        g = ctypes.c_int32(0)
        check(lib().swept_batch_grid(self._ctx, ctypes.byref(g)))
        return g.value

    def close(self):
        if self._ctx:
            lib().swept_batch_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SweptHeatAdvance(torch.autograd.Function):
    """T^M = swept heat advance of T^0 by n_steps with diffusivity alpha, differentiable
    in T^0 and alpha through the hand-written swept adjoint (swept_adjoint).

    apply(T0, alpha, n_steps, dt, length=1.0, tile=0, boundary=BC_PERIODIC, boundary_value=0.0):
    T0 an (N, N) GPU tensor, alpha a 0-d tensor (or float), boundary/boundary_value the
    walls (swept.h).  The forward records a checkpoint per swept cycle; backward runs the
    reverse sweep and returns (dJ/dT0, dJ/dalpha)."""

    @staticmethod
    def forward(ctx, T0, alpha, n_steps, dt, length=1.0, tile=0, boundary=BC_PERIODIC, boundary_value=0.0):
        state = T0.detach().clone().contiguous()
        a = float(alpha)
        solver = SweptSolver(HEAT, state, dt=dt, length=length, alpha=a, tile=tile, boundary=boundary,
                             boundary_value=boundary_value)
        tape = solver.new_tape(n_steps)
        solver.swept_advance_checkpointed(n_steps, tape)
        ctx.solver, ctx.tape, ctx.n = solver, tape, int(n_steps)
        ctx.alpha_is_tensor = torch.is_tensor(alpha)
        if ctx.alpha_is_tensor:
            ctx.alpha_meta = (alpha.shape, alpha.dtype, alpha.device)
        return state.clone()

    @staticmethod
    def backward(ctx, gTM):
        gTM = gTM.contiguous()
        gT0 = torch.empty_like(gTM)
        dalpha = ctx.solver.swept_adjoint(ctx.n, ctx.tape, gTM, gT0)
        ga = None
        if ctx.alpha_is_tensor:
            shape, dtype, device = ctx.alpha_meta
            ga = torch.full(shape, dalpha, dtype=dtype, device=device)
        return gT0, ga, None, None, None, None, None, None


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


def swept_cfl_dt_noalloc(state: torch.Tensor, length: float, cfl: float, gamma: float = 1.4) -> float:
    """swept_cfl_dt with the library's static device scratch: no workspace, no allocation."""
    n = state.shape[-1]
    prob = make_problem(EULER, n, state.dtype, 1.0, length, gamma=gamma)
    out = ctypes.c_double(0.0)
    check(lib().swept_cfl_dt_noalloc(ctypes.byref(prob), _dev_ptr(state), float(cfl), _stream_ptr(),
                                     ctypes.byref(out)))
    return out.value


__all__ = ["SweptSolver", "SweptHetero", "SweptBatch", "SweptHeatAdvance", "swept_cfl_dt", "swept_cfl_dt_noalloc", "swept_workspace_bytes", "make_problem", "HEAT",
           "EULER", "LIMITER_LITERAL", "SPEED_ROE", "BC_PERIODIC", "BC_DIRICHLET", "BC_NEUMANN",
           "BC_REFLECT", "BATCH_COOPERATIVE", "BATCH_PER_PHASE", "_lib"]
