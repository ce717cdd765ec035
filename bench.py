"""Benchmark: swept-rule heat diffusion on one MI355X.

Workload (one "step" of this benchmark = one whole swept advance):
heat equation on the periodic unit square, 4096 x 4096 cells, forward-Euler
5-point stencil, r = alpha dt / dx^2 = 0.2, 1000 time steps per advance,
initial state = 16 seeded random Fourier modes (wavenumbers 1-32, amplitudes
N(0,1)/k).  The state is resident in HBM before timing starts; each timed
step advances it 1000 more time steps in place.

Reported: cell-updates/s of the swept solver (value), the Standard solver's
rate on the same input and its speedup S = R_standard / R_swept (Eq. 3), the
effective bandwidth (bytes the Standard solver moves per step / time), the
roofline of the dominant kernel (the swept phase kernel) and the CPU oracle
timed on a bounded sample of the same workload.

Usage: python bench.py [--steps K] [--warmup W] [--dtype f64|f32] [--tile B]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 4096
STEPS_PER_ADVANCE = 1000
R = 0.2
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--tile", type=int, default=0, help="0: tuned or default tile")
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--advance-steps", type=int, default=STEPS_PER_ADVANCE)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-standard", action="store_true")
    return ap.parse_args()


def time_events(fn, k, stream):
    import torch

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(k):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / 1e3, wall


def cpu_baseline(dtype_np, n, budget_s=12.0):
    """The oracle, as it is, on the host cores: one step to size the sample, then a
    bounded number of steps of the same 4096^2 workload."""
    import numpy as np

    import oracle
    from paper_2105_10332_amd import problems

    T0 = problems.heat_fourier_modes(n).astype(dtype_np)
    t = time.perf_counter()
    T1 = oracle.heat_run(T0, R, 1)
    one = time.perf_counter() - t
    k = max(1, min(1000, int(budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.heat_run(T1, R, k)
    el = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": n * n * k / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"heat {n}x{n} {np.dtype(dtype_np).name}, {k} Standard steps of the C oracle "
                      f"(OpenMP over rows), {el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the swept path here is single-device); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2105_10332_amd import geometry, problems, tune
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    dev = torch.device("cuda", 0)
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    S = 8 if args.dtype == "f64" else 4
    n, M = args.n, args.advance_steps
    tile = args.tile or tune.best_tile("heat", args.dtype, n)
    T0 = problems.heat_fourier_modes(n)
    dx = 1.0 / n
    state = torch.tensor(T0, dtype=tdt, device=dev)
    solver = SweptSolver(HEAT, state, dt=R * dx * dx, length=1.0, alpha=1.0, tile=tile)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        solver.swept_advance(M)
    sec, wall = time_events(lambda: solver.swept_advance(M), args.steps, stream)
    updates = n * n * M * args.steps
    rate = updates / sec

    plan = geometry.totals(n, tile, 1, M)
    launches = plan["launches"] * args.steps
    avg_launch_s = sec / launches
    alg_bytes_per_launch = (plan["loads"] + plan["stores"]) * S / plan["launches"]
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9

    std = None
    if not args.no_standard:
        st_state = torch.tensor(T0, dtype=tdt, device=dev)
        st_solver = SweptSolver(HEAT, st_state, dt=R * dx * dx, length=1.0, alpha=1.0, tile=tile)
        st_solver.standard_advance(M)
        k_std = max(1, min(args.steps, 3))
        ssec, _ = time_events(lambda: st_solver.standard_advance(M), k_std, stream)
        srate = n * n * M * k_std / ssec
        std = {"value": srate, "unit": "cell-updates/s", "ms_per_advance": ssec / k_std * 1e3,
               "achieved_GBps": 2 * S * n * n * M * k_std / ssec / 1e9}

    out = {
        "metric": "cell-updates/s Swept vs Standard on 1 MI355X at equal accuracy; HBM GB/s",
        "value": rate,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"heat {n}x{n} periodic, 5-point forward Euler, r=0.2, {M} time steps per "
                               f"bench step, 16 seeded Fourier modes; swept tile {tile}",
                   "tile": tile, "time_steps_per_step": M, "launches_per_step": plan["launches"]},
        "effective_GBps": 2 * S * updates / sec / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "swept_phase_kernel<HeatS>",
                     "alg_bytes_per_launch": alg_bytes_per_launch, "avg_launch_us": avg_launch_s * 1e6},
        "standard": std,
        "speedup_vs_standard": (rate / std["value"]) if std else None,
        "wall_s": wall,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(np.float64 if args.dtype == "f64" else np.float32, n)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
