"""ctypes binding of libswept.so (argument marshalling only).

Every call goes straight to the C ABI declared in include/swept.h; no step
of the solver runs in Python.  If the library is missing the import of the
binding fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswept.so")

SWEPT_OK = 0
ERRORS = {
    -1: "SWEPT_EINVAL", -2: "SWEPT_ESHAPE", -3: "SWEPT_EUNSTABLE", -4: "SWEPT_ENOTSUP",
    -5: "SWEPT_EWORKSPACE", -6: "SWEPT_EHIP", -7: "SWEPT_ENONFINITE",
}
CODES = {v: k for k, v in ERRORS.items()}
HEAT, EULER = 0, 1
F64, F32 = 0, 1
LIMITER_LITERAL, SPEED_ROE = 1, 2  # Euler scheme variant bits (swept.h)
BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN, BC_REFLECT = 0, 1, 2, 3  # boundaries (swept.h)
BATCH_COOPERATIVE, BATCH_PER_PHASE = 0, 1  # batch launch modes (swept.h)


class SweptError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
                ("scheme", ctypes.c_int32), ("boundary", ctypes.c_int32), ("boundary_value", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("wg", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("nvar", ctypes.c_int32), ("n", ctypes.c_int32), ("levels_per_step", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("h", ctypes.c_int32), ("wg", ctypes.c_int32),
                ("r", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("state_bytes", ctypes.c_size_t), ("lds_bytes", ctypes.c_size_t)]


_P = ctypes.c_void_p
_SIGS = {
    "swept_workspace_bytes": [ctypes.POINTER(Problem), ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_size_t)],
    "swept_init": [ctypes.POINTER(_P), ctypes.POINTER(Problem), ctypes.POINTER(Tuning), _P, _P, ctypes.c_size_t, _P],
    "swept_query": [_P, ctypes.POINTER(Info)],
    "swept_set_stream": [_P, _P],
    "swept_advance": [_P, ctypes.c_int64],
    "standard_advance": [_P, ctypes.c_int64],
    "swept_conserved": [_P, ctypes.POINTER(ctypes.c_double)],
    "swept_cfl_dt": [ctypes.POINTER(Problem), _P, ctypes.c_double, _P, ctypes.c_size_t, _P,
                     ctypes.POINTER(ctypes.c_double)],
    "swept_cfl_dt_noalloc": [ctypes.POINTER(Problem), _P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double)],
    "swept_destroy": [_P],
    "swept_tape_bytes": [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
    "swept_advance_checkpointed": [_P, ctypes.c_int64, _P, ctypes.c_size_t],
    "swept_adjoint": [_P, ctypes.c_int64, _P, ctypes.c_size_t, _P, _P, ctypes.POINTER(ctypes.c_double)],
    "swept_batch_workspace_bytes": [ctypes.POINTER(Problem), ctypes.POINTER(Tuning), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_size_t)],
    "swept_batch_init": [ctypes.POINTER(_P), ctypes.POINTER(Problem), ctypes.POINTER(Tuning), ctypes.POINTER(_P),
                         ctypes.c_int32, _P, ctypes.c_size_t, _P],
    "swept_batch_advance": [_P, ctypes.c_int64],
    "swept_batch_query": [_P, ctypes.c_int32, ctypes.POINTER(Info)],
    "swept_batch_grid": [_P, ctypes.POINTER(ctypes.c_int32)],
    "swept_batch_set_mode": [_P, ctypes.c_int32],
    "swept_batch_set_stream": [_P, _P],
    "swept_batch_destroy": [_P],
    "swept_hetero_init": [ctypes.POINTER(_P), _P, ctypes.c_double, ctypes.c_int32],
    "swept_hetero_advance": [_P, ctypes.c_int64],
    "swept_hetero_query": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)],
    "swept_hetero_destroy": [_P],
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        # PyTorch ships its own HIP runtime library; importing it first makes libswept bind to that
        # same runtime, so the device pointers and streams torch hands over are valid here.  Loaded
        # the other way round, the process holds two HIP runtimes and libswept's sees no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.swept_last_error.argtypes = []
        L.swept_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(rc: int):
    if rc != SWEPT_OK:
        raise SweptError(rc, lib().swept_last_error().decode())
    return rc


def last_error() -> str:
    return lib().swept_last_error().decode()
