"""CPU oracle for the two-dimensional swept rule (arXiv:2105.10332).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.

Two independent CPU implementations of the same plain definitions live here:

* ``oracle.c`` (compiled to ``liboracle.so`` by :func:`build`) -- double
  loops, OpenMP over rows, FP64 and FP32 instantiations; the reference that
  GPU results are compared with and the timed CPU baseline;
* ``numpy_ref.py`` -- the same equations written with ``np.roll`` on whole
  fields, used to cross-check the C code on small grids.

Both follow the Standard solver of Sec. 3.1 (one step at a time), since the
swept rule reaches exactly that result (Sec. 3.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
_SRC = os.path.join(HERE, "oracle.c")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile oracle.c twice (FP64, FP32) with gcc into liboracle.so."""
    objs = []
    for real, sfx in (("double", "_f64"), ("float", "_f32")):
        obj = os.path.join(HERE, f"oracle{sfx}.o")
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-std=c11",
               f"-DREAL={real}", f"-DSFX={sfx}", "-c", _SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", tmp] + objs + ["-lm"])
    os.replace(tmp, LIB_PATH)
    for o in objs:
        os.remove(o)
    return LIB_PATH


def lib():
    """Load liboracle.so (building it first if it is absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I = ctypes.c_int64
_D = ctypes.c_double


def _declare(L):
    for s in ("_f64", "_f32"):
        getattr(L, "oracle_heat_step" + s).argtypes = [_P, _P, _I, _D]
        getattr(L, "oracle_heat_run" + s).argtypes = [_P, _P, _I, _D, _I]
        getattr(L, "oracle_heat_step_bc" + s).argtypes = [_P, _P, _I, _D, _I, _D]
        getattr(L, "oracle_heat_run_bc" + s).argtypes = [_P, _P, _I, _D, _I, _I, _D]
        getattr(L, "oracle_heat_adjoint_bc" + s).argtypes = [_P, _P, _P, ctypes.POINTER(_D), _I, _D, _I, _P, _P,
                                                             _I, _D]
        getattr(L, "oracle_heat_adjoint" + s).argtypes = [_P, _P, _P, ctypes.POINTER(_D), _I, _D, _I, _P, _P]
        getattr(L, "oracle_l2_mismatch" + s).argtypes = [_P, _P, _I]
        getattr(L, "oracle_l2_mismatch" + s).restype = _D
        getattr(L, "oracle_euler_run" + s).argtypes = [_P, _P, _I, _D, _D, _D, _D, _I, _I]
        getattr(L, "oracle_euler_run_bc" + s).argtypes = [_P, _P, _I, _D, _D, _D, _D, _I, _I, _I]
        getattr(L, "oracle_euler_work_values" + s).argtypes = [_I]
        getattr(L, "oracle_euler_work_values" + s).restype = _I
        getattr(L, "oracle_cfl_dt" + s).argtypes = [_P, _I, _D, _D, _D, _D]
        getattr(L, "oracle_cfl_dt" + s).restype = _D
        getattr(L, "oracle_plane_sums" + s).argtypes = [_P, _I, _I, _P]
        getattr(L, "oracle_face" + s).argtypes = [_P, _P, _P, _P, _I, _D, _I, _P, _P, _P]
        getattr(L, "oracle_roe_average" + s).argtypes = [_P, _P, _I, _D, _P]


def _sfx(a: np.ndarray) -> str:
    if a.dtype == np.float64:
        return "_f64"
    if a.dtype == np.float32:
        return "_f32"
    raise TypeError(f"oracle supports float64/float32, got {a.dtype}")


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN, BC_REFLECT = 0, 1, 2, 3  # boundaries (see oracle.c)


def heat_step(T: np.ndarray, r: float, bc: int = BC_PERIODIC, bcv: float = 0.0) -> np.ndarray:
    """One heat step (App. A update) of an N x N field; bc = boundary, bcv = Dirichlet ghost value."""
    T = np.ascontiguousarray(T)
    out = np.empty_like(T)
    if bc == BC_PERIODIC:
        getattr(lib(), "oracle_heat_step" + _sfx(T))(_ptr(T), _ptr(out), T.shape[0], float(r))
    else:
        getattr(lib(), "oracle_heat_step_bc" + _sfx(T))(_ptr(T), _ptr(out), T.shape[0], float(r), int(bc),
                                                        float(bcv))
    return out


def heat_run(T0: np.ndarray, r: float, steps: int, bc: int = BC_PERIODIC, bcv: float = 0.0) -> np.ndarray:
    """``steps`` forward-Euler heat steps; returns T^M (T0 is not modified)."""
    T = np.array(T0, copy=True, order="C")
    work = np.empty_like(T)
    if bc == BC_PERIODIC:
        getattr(lib(), "oracle_heat_run" + _sfx(T))(_ptr(T), _ptr(work), T.shape[0], float(r), int(steps))
    else:
        getattr(lib(), "oracle_heat_run_bc" + _sfx(T))(_ptr(T), _ptr(work), T.shape[0], float(r), int(steps),
                                                       int(bc), float(bcv))
    return T


def heat_adjoint(T0: np.ndarray, g: np.ndarray, r: float, steps: int, bc: int = 0, bcv: float = 0.0):
    """Discrete adjoint of ``heat_run``: returns (dJ/dT0, dJ/dr) for dJ/dT^M = g (bc, bcv: the walls)."""
    T0 = np.ascontiguousarray(T0)
    g = np.ascontiguousarray(g, dtype=T0.dtype)
    N = T0.shape[0]
    out = np.empty_like(T0)
    levels = np.empty((steps + 1, N, N), dtype=T0.dtype)
    work = np.empty_like(T0)
    dJdr = ctypes.c_double(0.0)
    if bc == BC_PERIODIC:
        getattr(lib(), "oracle_heat_adjoint" + _sfx(T0))(_ptr(T0), _ptr(g), _ptr(out), ctypes.byref(dJdr), N,
                                                         float(r), int(steps), _ptr(levels), _ptr(work))
    else:
        getattr(lib(), "oracle_heat_adjoint_bc" + _sfx(T0))(_ptr(T0), _ptr(g), _ptr(out), ctypes.byref(dJdr), N,
                                                            float(r), int(steps), _ptr(levels), _ptr(work), int(bc),
                                                            float(bcv))
    return out, dJdr.value


def l2_mismatch(T: np.ndarray, Tstar: np.ndarray) -> float:
    """J = 1/2 sum (T - T*)^2 accumulated in double."""
    T = np.ascontiguousarray(T)
    Tstar = np.ascontiguousarray(Tstar, dtype=T.dtype)
    return getattr(lib(), "oracle_l2_mismatch" + _sfx(T))(_ptr(T), _ptr(Tstar), T.size)


LIMITER_LITERAL, SPEED_ROE = 1, 2  # scheme variant bits (see oracle.c)


def euler_run(Q0: np.ndarray, dt: float, dx: float, dy: float, gamma: float, steps: int,
              scheme: int = 0, bc: int = 0) -> np.ndarray:
    """``steps`` RK2 steps of the 2D Euler equations; Q0 is (4, N, N); scheme = variant bits;
    bc = BC_PERIODIC, BC_NEUMANN (zero gradient) or BC_REFLECT (slip walls)."""
    Q = np.array(Q0, copy=True, order="C")
    N = Q.shape[1]
    s = _sfx(Q)
    nwork = getattr(lib(), "oracle_euler_work_values" + s)(N)
    work = np.empty(nwork, dtype=Q.dtype)
    getattr(lib(), "oracle_euler_run_bc" + s)(_ptr(Q), _ptr(work), N, float(dt), float(dx), float(dy),
                                              float(gamma), int(steps), int(scheme), int(bc))
    return Q


def cfl_dt(Q: np.ndarray, dx: float, dy: float, gamma: float, cfl: float) -> float:
    """dt = cfl / max((|u|+c)/dx + (|v|+c)/dy) over cells, in double."""
    Q = np.ascontiguousarray(Q)
    return getattr(lib(), "oracle_cfl_dt" + _sfx(Q))(_ptr(Q), Q.shape[1], float(dx), float(dy), float(gamma),
                                                    float(cfl))


def plane_sums(Q: np.ndarray) -> np.ndarray:
    """Sequential double sums of each plane of a (nvar, N, N) or (N, N) field."""
    Q = np.ascontiguousarray(Q)
    nvar = 1 if Q.ndim == 2 else Q.shape[0]
    NN = Q.shape[-1] * Q.shape[-2]
    out = np.zeros(nvar, dtype=np.float64)
    getattr(lib(), "oracle_plane_sums" + _sfx(Q))(_ptr(Q), nvar, NN, _ptr(out))
    return out


def face(A, B, C, D, axis: int, gamma: float, dtype=np.float64, scheme: int = 0):
    """Reconstructed left/right states and numerical flux at the face between B and C.

    A..D are conserved 4-vectors of consecutive cells along the face normal;
    axis 1 = x face (F), 2 = y face (G); scheme = variant bits.  Returns (Q_L, Q_R, flux).
    """
    arrs = [np.ascontiguousarray(v, dtype=dtype) for v in (A, B, C, D)]
    L = np.empty(4, dtype=dtype)
    R = np.empty(4, dtype=dtype)
    F = np.empty(4, dtype=dtype)
    getattr(lib(), "oracle_face" + _sfx(arrs[0]))(*[_ptr(a) for a in arrs], int(axis), float(gamma), int(scheme),
                                                 _ptr(L), _ptr(R), _ptr(F))
    return L, R, F


def roe_average(L, R, axis: int, gamma: float, dtype=np.float64):
    """(u~_a, u~_b, H~, |u~_a| + c~) of the Roe average of two conserved 4-vectors along axis a."""
    l = np.ascontiguousarray(L, dtype=dtype)
    r = np.ascontiguousarray(R, dtype=dtype)
    out = np.empty(4, dtype=dtype)
    getattr(lib(), "oracle_roe_average" + _sfx(l))(_ptr(l), _ptr(r), int(axis), float(gamma), _ptr(out))
    return out
