"""Shared helpers of the GPU tests: run the HIP library through its binding."""
from __future__ import annotations

import numpy as np
import torch

from paper_2105_10332_amd.solver import EULER, HEAT, SweptSolver

DEV = torch.device("cuda", 0)
TDT = {np.float64: torch.float64, np.float32: torch.float32}


def heat_gpu(T0: np.ndarray, r: float, steps: int, tile: int, method: str = "swept", wg: int = 0, poison=False,
             bc: int = 0, bcv: float = 0.0):
    """Run heat on the GPU; returns (result, r as the kernels used it)."""
    n = T0.shape[0]
    T = torch.tensor(T0, device=DEV)
    dx = 1.0 / n
    s = SweptSolver(HEAT, T, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile, wg=wg, boundary=bc,
                    boundary_value=bcv)
    if poison:  # all-ones bytes = NaN in every lane of the second level-parity buffer
        s.work[: s.info.state_bytes].fill_(255)
    getattr(s, method + "_advance")(steps)
    torch.cuda.synchronize()
    r_used = s.info.r
    s.close()
    return T.cpu().numpy(), r_used


def euler_gpu(Q0: np.ndarray, dt: float, steps: int, tile: int, method: str = "swept", length: float = 10.0,
              poison=False, scheme=0, bc=0, wg=0):
    Q = torch.tensor(Q0, device=DEV)
    s = SweptSolver(EULER, Q, dt=dt, length=length, gamma=1.4, tile=tile, scheme=scheme, boundary=bc, wg=wg)
    if poison:
        s.work[: s.info.state_bytes].fill_(255)
    getattr(s, method + "_advance")(steps)
    torch.cuda.synchronize()
    s.close()
    return Q.cpu().numpy()


def rel_err(a, b):
    """Normwise error per field: max|a - b| / max|b| (b the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 3:
        return max(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max() for k in range(a.shape[0]))
    return np.abs(a - b).max() / np.abs(b).max()
