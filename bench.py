"""Benchmark of the swept-rule solver on one MI355X.

Default workload (one bench "step" = one whole swept advance): heat
diffusion on the periodic unit square, 4096 x 4096 cells, forward-Euler
5-point stencil, r = alpha dt / dx^2 = 0.2, 1000 time steps per advance,
initial state = 16 seeded random Fourier modes.  The state is resident in
HBM before timing starts; each timed step advances it 1000 more time steps
in place.

Reported: cell-updates/s of the swept solver (value), the Standard
solver's rate on the same input and the paper's speedup S = R_standard /
R_swept (Eq. 3), the effective bandwidth (bytes the Standard solver would
move / time), the roofline of the dominant kernel (the swept phase kernel),
its three per-update bounds (HBM bytes, vector-ALU flops, LDS bytes; heat only),
the HBM traffic the counters measured for these kernel sources (else null) and the CPU
oracle timed on a bounded sample of the same workload.

Other workloads (--workload): euler (2048^2 vortex, 500 RK2 steps per
step), adjoint (1024^2 FP32 heat, 2000 steps: forward with checkpoints +
reverse sweep per step), batch (48 heat + 16 Euler problems, FP32, 200 steps,
one persistent launch per step), study (the paper's parameter study at a
GPU share of 100%: speedup over array sizes 320-1120 and block sizes 8-32), graphs
(eager launches against replayed HIP graphs at 320^2 and 1024^2), hetero (the advance split
between the GPU and the host cores at GPU shares 0-100%, Eq. 2).

Usage: python bench.py [--steps K] [--warmup W] [--dtype f64|f32] [--tile B] [--workload W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s Swept vs Standard on 1 MI355X at equal accuracy; HBM GB/s"

# HBM bytes per launch of the swept phase kernel from two rocprofv3 --pmc passes (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0: the factors a plain copy of known size reads), keyed by workload and launch
# shape, valid only for the kernel sources whose hash is recorded with it (null otherwise).
MEASURED_TRAFFIC = {
    ("heat", "f64", 4096, 64, 512, 1000): (632.4e6, "d2f8f8f34ab44653"),
    ("heat", "f32", 4096, 64, 256, 1000): (371.0e6, "d2f8f8f34ab44653"),
    ("euler", "f64", 2048, 32, 1024, 500): (694.5e6, "d2f8f8f34ab44653"),
    ("euler", "f32", 2048, 32, 512, 500): (478.5e6, "d2f8f8f34ab44653"),
}
# The same two passes over the Standard kernels: HBM bytes per launch (one time step).
MEASURED_STANDARD_TRAFFIC = {
    ("heat", "f64", 4096): (293.7e6, "d2f8f8f34ab44653"),
    ("heat", "f32", 4096): (151.0e6, "d2f8f8f34ab44653"),
    ("euler", "f64", 2048): (538.6e6, "d2f8f8f34ab44653"),
    ("euler", "f32", 2048): (336.8e6, "d2f8f8f34ab44653"),
}
KERNEL_SOURCES = ("scheme.h", "device_common.h", "kernels.hip", "launch.h")


def code_text(src: str) -> str:
    """Source text without comments and whitespace runs: what the compiler sees."""
    import re

    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_hash():
    """Hash of the heat kernel's sources (comments ignored): a measured traffic figure is
    reported only while the code it was measured on is unchanged."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2105_10332_amd", "csrc", f)) as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(key, table=MEASURED_TRAFFIC):
    rec = table.get(key)
    return rec[0] if rec and rec[1] == kernel_hash() else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["heat", "euler", "adjoint", "batch", "study", "graphs", "hetero"],
                    default="heat")
    ap.add_argument("--threads", type=int, default=0, help="hetero workload: host worker threads (0: default)")
    ap.add_argument("--dtype", choices=["f64", "f32"], default=None)
    ap.add_argument("--tile", type=int, default=0, help="0: tuned or default tile")
    ap.add_argument("--wg", type=int, default=0, help="0: tuned or library default")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--boundary", type=int, default=0,
                    help="0 periodic; heat 1 Dirichlet (ghost value --boundary-value), 2 zero flux; "
                         "Euler 2 zero gradient, 3 slip walls")
    ap.add_argument("--boundary-value", type=float, default=0.0)
    ap.add_argument("--scheme", type=int, default=0,
                    help="Euler scheme variant bits: 1 limiter factors as printed, 2 Roe-averaged speed")
    ap.add_argument("--advance-steps", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-standard", action="store_true")
    ap.add_argument("--batch-per-phase", action="store_true",
                    help="batch workload: one ordinary launch per global phase instead of one cooperative launch")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only run a plain device copy of the C2 state size (calibrates rocprofv3 FETCH/WRITE_SIZE)")
    return ap.parse_args()


def timed(fn, k):
    """Run fn k times between two events on the current stream; (seconds, wall seconds)."""
    import torch

    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(k):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3, time.perf_counter() - t0


def cores():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()


def cpu_heat(dtype_np, n, r, budget_s=25.0, bc=0, bcv=0.0):
    """The oracle as it is on the host cores: a warm step, a few steps to size the sample,
    then a bounded number of Standard steps of the same grid (about budget_s seconds)."""
    import numpy as np

    import oracle
    from paper_2105_10332_amd import problems

    T0 = problems.heat_fourier_modes(n).astype(dtype_np)
    T1 = oracle.heat_run(T0, r, 2, bc, bcv)
    t = time.perf_counter()
    T1 = oracle.heat_run(T1, r, 16, bc, bcv)
    one = (time.perf_counter() - t) / 16
    k = max(1, min(20000, int(budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.heat_run(T1, r, k, bc, bcv)
    el = time.perf_counter() - t
    return {"value": n * n * k / el, "unit": "cell-updates/s", "cores": cores(), "kind": "oracle",
            "sample": f"heat {n}x{n} {np.dtype(dtype_np).name}, {k} Standard steps of the C oracle "
                      f"(OpenMP over rows), {el:.1f} s"}


def cpu_euler(dtype_np, n, dt, budget_s=15.0, scheme=0, bc=0):
    import numpy as np

    import oracle
    from paper_2105_10332_amd import problems

    Q0 = problems.shu_vortex(n).astype(dtype_np)
    Q1 = oracle.euler_run(Q0, dt, 10 / n, 10 / n, 1.4, 1, scheme, bc)
    t = time.perf_counter()
    Q1 = oracle.euler_run(Q1, dt, 10 / n, 10 / n, 1.4, 2, scheme, bc)
    one = (time.perf_counter() - t) / 2
    k = max(1, min(1000, int(budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.euler_run(Q1, dt, 10 / n, 10 / n, 1.4, k, scheme, bc)
    el = time.perf_counter() - t
    return {"value": n * n * k / el, "unit": "cell-steps/s", "cores": cores(), "kind": "oracle",
            "sample": f"Euler vortex {n}x{n} {np.dtype(dtype_np).name}, {k} RK2 steps of the C oracle, {el:.1f} s"}


def base_record(args, value, unit, sec, dtype, config):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": sec / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def roofline(plan, S, nvar, launches, sec, kernel):
    """Algorithmic HBM bytes of the swept phase kernel per launch / its average launch time."""
    alg = (plan["loads"] + plan["stores"]) * S * nvar / plan["launches"]
    avg = sec / launches
    ach = alg / avg / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": kernel, "alg_bytes_per_launch": alg, "avg_launch_us": avg * 1e6,
            "clock": "HIP events recorded on the launch stream around the timed advances, divided by the "
                     "phase launches they hold (the rocprofv3 kernel-trace average of the same command is "
                     "in profiles/)"}


# Per-update costs of the swept heat kernel beside its HBM bytes, for the bound
# t_min = max(HBM bytes / HBM peak, flops / vector peak, LDS bytes / LDS peak): the 9 flops of
# the 5-point update, and the LDS values of the pair-strip walk (per pair of cells the next row
# of both columns and the outer left and right neighbours are read and both results written:
# 3 values per update).  LDS peak: 128 B per clock per CU x 256 CUs x 2.4 GHz.
LDS_PEAK_GBS = 128 * 256 * 2.4
VECTOR_PEAK_TFLOPS = {8: 78.6, 4: 157.3}
HEAT_FLOPS, HEAT_LDS_VALUES = 9, 3


def heat_bounds(plan, S, updates_per_advance, rate):
    t = {"hbm": (plan["loads"] + plan["stores"]) * S / updates_per_advance / (HBM_PEAK_GBS * 1e9),
         "lds": HEAT_LDS_VALUES * S / (LDS_PEAK_GBS * 1e9),
         "valu": HEAT_FLOPS / (VECTOR_PEAK_TFLOPS[S] * 1e12)}
    return {"model": "t_min = max(HBM bytes/HBM peak, flops/vector peak, LDS bytes/LDS peak) per cell-update",
            "ps_per_update": {k: v * 1e12 for k, v in t.items()},
            "frac": {k: v * rate for k, v in t.items()}, "binding": max(t, key=t.get)}


def run_heat(args):
    import numpy as np
    import torch

    from paper_2105_10332_amd import geometry, problems, tune
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    dt_name = args.dtype or "f64"
    tdt = torch.float64 if dt_name == "f64" else torch.float32
    S = 8 if dt_name == "f64" else 4
    n, M, r = args.n or 4096, args.advance_steps or 1000, 0.2
    tile, wg = tune.best("heat", dt_name, n)
    tile, wg = args.tile or tile, args.wg or wg
    T0 = problems.heat_fourier_modes(n)
    dx = 1.0 / n
    state = torch.tensor(T0, dtype=tdt, device="cuda")
    bc = dict(boundary=args.boundary, boundary_value=args.boundary_value)
    solver = SweptSolver(HEAT, state, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile, wg=wg, **bc)
    for _ in range(args.warmup):
        solver.swept_advance(M)
    sec, wall = timed(lambda: solver.swept_advance(M), args.steps)
    updates = n * n * M * args.steps
    rate = updates / sec
    plan = geometry.totals(n, tile, 1, M)
    walls = {0: "periodic", 1: f"Dirichlet walls (ghost value {args.boundary_value})", 2: "zero-flux walls"}
    cfg = {"workload": f"heat {n}x{n} {walls[args.boundary]}, 5-point forward Euler, r=0.2, {M} time steps per "
                       f"bench step, 16 seeded Fourier modes; swept tile {tile}",
           "tile": tile, "wg": solver.info.wg, "time_steps_per_step": M, "launches_per_step": plan["launches"]}
    out = base_record(args, rate, "cell-updates/s", sec, dt_name, cfg)
    out["effective_GBps"] = 2 * S * updates / sec / 1e9
    out["roofline"] = roofline(plan, S, 1, plan["launches"] * args.steps, sec, "swept_phase_kernel<HeatS>")
    out["bounds"] = heat_bounds(plan, S, n * n * M, rate)
    if args.boundary == 0:
        out["roofline"]["traffic"] = measured_traffic(("heat", dt_name, n, tile, solver.info.wg, M))
    if not args.no_standard:
        st = torch.tensor(T0, dtype=tdt, device="cuda")
        ss = SweptSolver(HEAT, st, dt=r * dx * dx, length=1.0, alpha=1.0, tile=tile, **bc)
        ss.standard_advance(M)
        k = max(1, min(args.steps, 3))
        ssec, _ = timed(lambda: ss.standard_advance(M), k)
        out["standard"] = {"value": n * n * M * k / ssec, "unit": "cell-updates/s", "ms_per_advance": ssec / k * 1e3,
                           "achieved_GBps": 2 * S * n * n * M * k / ssec / 1e9}
        if args.boundary == 0:
            out["standard"]["traffic_per_launch"] = measured_traffic(("heat", dt_name, n), MEASURED_STANDARD_TRAFFIC)
        out["speedup_vs_standard"] = rate / out["standard"]["value"]
    out["wall_s"] = wall
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_heat(np.float64 if dt_name == "f64" else np.float32, n, r, bc=args.boundary,
                                        bcv=args.boundary_value)
    return out


def reductions(solver, q, S, n, calls=50):
    """The two whole-state reductions on the Euler state: the CFL time step (max over cells)
    and the FP64 conservation sums.  Both return host scalars, so each call synchronises;
    the figure is the mean latency per call over back-to-back calls, and the rate counts the
    one read of the 4 planes each makes."""
    import ctypes

    import torch

    from paper_2105_10332_amd.solver import EULER, _dev_ptr, _stream_ptr, make_problem, swept_workspace_bytes
    from paper_2105_10332_amd._lib import check, lib

    prob = make_problem(EULER, n, q.dtype, 1.0, 10.0, gamma=1.4)
    nbytes = swept_workspace_bytes(prob)
    work = torch.empty(nbytes, dtype=torch.uint8, device=q.device)
    out = ctypes.c_double(0.0)

    def cfl():
        check(lib().swept_cfl_dt(ctypes.byref(prob), _dev_ptr(q), 0.4, _dev_ptr(work), nbytes, _stream_ptr(),
                                 ctypes.byref(out)))

    res = {}
    for name, fn in (("cfl_dt", cfl), ("conserved", solver.swept_conserved)):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(calls):
            fn()
        el = (time.perf_counter() - t) / calls
        b = 4 * S * n * n
        res[name] = {"us_per_call": el * 1e6, "bytes_read": b, "GBps": b / el / 1e9, "frac": b / el / 1e9 / HBM_PEAK_GBS,
                     "note": "synchronous call: kernels + result copy + host wait"}
    return res


def run_euler(args):
    import numpy as np
    import torch

    from paper_2105_10332_amd import geometry, problems, tune
    from paper_2105_10332_amd.solver import EULER, SweptSolver, swept_cfl_dt

    dt_name = args.dtype or "f64"
    tdt = torch.float64 if dt_name == "f64" else torch.float32
    S = 8 if dt_name == "f64" else 4
    n, M = args.n or 2048, args.advance_steps or 500
    tile, wg = tune.best("euler", dt_name, n)
    tile, wg = args.tile or tile, args.wg or wg
    Q0 = problems.shu_vortex(n)
    q = torch.tensor(Q0, dtype=tdt, device="cuda")
    dt = swept_cfl_dt(torch.tensor(Q0, device="cuda"), 10.0, 0.4)
    solver = SweptSolver(EULER, q, dt=dt, length=10.0, gamma=1.4, tile=tile, wg=wg, scheme=args.scheme,
                         boundary=args.boundary)
    for _ in range(args.warmup):
        solver.swept_advance(M)
    sec, wall = timed(lambda: solver.swept_advance(M), args.steps)
    cells = n * n * M * args.steps
    rate = cells / sec
    plan = geometry.totals(n, tile, 2, 2 * M, True)
    scheme = {0: "minmod + Rusanov", 1: "limiter factors as printed + Rusanov", 2: "minmod + Roe-averaged speed",
              3: "limiter factors as printed + Roe-averaged speed"}[args.scheme]
    walls = {0: "periodic", 2: "zero-gradient walls", 3: "slip walls"}[args.boundary]
    cfg = {"workload": f"Euler {n}x{n} {walls} [0,10]^2, gamma 1.4, vortex eps 5 on (1,1), {scheme}, "
                       f"RK2, CFL 0.4 (dt {dt:.6e}), {M} steps per bench step; swept tile {tile}",
           "tile": tile, "scheme": args.scheme, "time_steps_per_step": M, "launches_per_step": plan["launches"]}
    out = base_record(args, rate, "cell-steps/s", sec, dt_name, cfg)
    out["effective_GBps"] = 8 * S * cells / sec / 1e9
    out["roofline"] = roofline(plan, S, 4, plan["launches"] * args.steps, sec, "swept_phase_kernel<EulerS>")
    if args.boundary == 0 and args.scheme == 0:
        out["roofline"]["traffic"] = measured_traffic(("euler", dt_name, n, tile, solver.info.wg, M))
    if not args.no_standard:
        st = torch.tensor(Q0, dtype=tdt, device="cuda")
        ss = SweptSolver(EULER, st, dt=dt, length=10.0, gamma=1.4, tile=tile, scheme=args.scheme,
                         boundary=args.boundary)
        ss.standard_advance(M)
        ssec, _ = timed(lambda: ss.standard_advance(M), 1)
        out["standard"] = {"value": n * n * M / ssec, "unit": "cell-steps/s", "ms_per_advance": ssec * 1e3}
        if args.boundary == 0 and args.scheme == 0:
            out["standard"]["traffic_per_launch"] = measured_traffic(("euler", dt_name, n), MEASURED_STANDARD_TRAFFIC)
        out["speedup_vs_standard"] = rate / out["standard"]["value"]
    out["reductions"] = reductions(solver, q, S, n)
    out["wall_s"] = wall
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_euler(np.float64 if dt_name == "f64" else np.float32, n, dt, scheme=args.scheme,
                                        bc=args.boundary)
    return out


def run_adjoint(args):
    import numpy as np
    import torch

    from paper_2105_10332_amd import problems
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    dt_name = args.dtype or "f32"
    tdt = torch.float64 if dt_name == "f64" else torch.float32
    n, M = args.n or 1024, args.advance_steps or 2000
    tile = args.tile or 32
    dx = 1.0 / n
    T0 = torch.tensor(problems.heat_fourier_modes(n, seed=problems.SEED_ADJ_T0), dtype=tdt, device="cuda")
    Ts = torch.tensor(problems.heat_fourier_modes(n, seed=problems.SEED_ADJ_TARGET), dtype=tdt, device="cuda")
    x = T0.clone()
    s = SweptSolver(HEAT, x, dt=0.2 * dx * dx, length=1.0, alpha=1.0, tile=tile, wg=args.wg)
    tape = s.new_tape(M)
    gT0 = torch.empty_like(x)

    def one():
        x.copy_(T0)
        s.swept_advance_checkpointed(M, tape)
        s.swept_adjoint(M, tape, x - Ts, gT0)

    for _ in range(args.warmup):
        one()
    sec, wall = timed(one, args.steps)
    fsec, _ = timed(lambda: s.swept_advance(M), 1)
    csec, _ = timed(lambda: s.swept_advance_checkpointed(M, tape), 1)
    gTM = x - Ts
    asec, _ = timed(lambda: s.swept_adjoint(M, tape, gTM, gT0), 1)
    cfg = {"workload": f"adjoint of heat {n}x{n} periodic, r=0.2, {M} steps, loss 1/2 sum (T^M - T*)^2, "
                       f"gradients wrt T0 and alpha, checkpoint per swept cycle of {tile // 2} steps; tile {tile}",
           "tile": tile}
    out = base_record(args, n * n * M * args.steps / sec, "cell-updates/s (forward+adjoint)", sec, dt_name, cfg)
    out["forward_ms"] = fsec * 1e3
    out["forward_checkpointed_ms"] = csec * 1e3
    out["adjoint_ms"] = asec * 1e3
    out["adjoint_over_forward"] = asec / fsec
    out["wall_s"] = wall
    return out


def run_batch(args):
    import torch

    from paper_2105_10332_amd import problems, tune
    from paper_2105_10332_amd.solver import BATCH_PER_PHASE, EULER, HEAT, SweptBatch, SweptSolver, swept_cfl_dt

    dt_name = args.dtype or "f32"
    tdt = torch.float64 if dt_name == "f64" else torch.float32
    M = args.advance_steps or 200
    items, cells = [], 0
    ens = problems.batch_ensemble()
    tiles = tune.batch_tiles([(it.kind, it.n) for it in ens], dt_name)
    for it, tile in zip(ens, tiles):
        n = it.n
        if it.kind == "heat":
            x = torch.tensor(problems.heat_fourier_modes(n, seed=it.seed), dtype=tdt, device="cuda")
            items.append((HEAT, x, it.r / n / n, 1.0, 1.0, 1.4, tile))
        else:
            q0 = torch.tensor(problems.shu_vortex(n, eps=it.eps), device="cuda")
            dt = swept_cfl_dt(q0, 10.0, 0.4)
            items.append((EULER, q0.to(tdt), dt, 10.0, 1.0, 1.4, tile))
        cells += n * n * M
    init = [it[1].clone() for it in items]
    b = SweptBatch(items)
    if args.batch_per_phase:
        b.swept_batch_set_mode(BATCH_PER_PHASE)

    def one():
        for it, x0 in zip(items, init):
            it[1].copy_(x0)
        b.swept_batch_advance(M)

    for _ in range(args.warmup):
        one()
    sec, wall = timed(one, args.steps)
    # the same problems (same tiles) one after another, each with its own swept advance (reference rate)
    solvers = [SweptSolver(k, x, dt=dt, length=L, alpha=a, gamma=g, tile=t) for (k, x, dt, L, a, g, t) in items]

    def seq():
        for sv, x0 in zip(solvers, init):
            sv.state.copy_(x0)
            sv.swept_advance(M)

    ssec, _ = timed(seq, 1)
    # explicit teardown: finish the stream and release the batch, the solvers and their device
    # memory before the process exits
    torch.cuda.synchronize()
    grid = b.grid
    b.close()
    for sv in solvers:
        sv.close()
    del solvers, b, items, init
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    cfg = {"workload": f"batch of 48 heat (edges 128-1024, r 0.05-0.24) + 16 Euler vortex (edges 256-1024, "
                       f"eps 1-5) problems, {M} steps each, "
                       f"{'one launch per global phase' if args.batch_per_phase else 'one persistent launch'}; "
                       f"grid {grid} workgroups",
           "problems": len(ens), "grid": grid,
           "tiles": {"heat": sorted(set(t for it, t in zip(ens, tiles) if it.kind == "heat")),
                     "euler": sorted(set(t for it, t in zip(ens, tiles) if it.kind == "euler"))}}
    out = base_record(args, cells * args.steps / sec, "cell-updates/s", sec, dt_name, cfg)
    out["sequential_swept"] = {"value": cells / ssec, "unit": "cell-updates/s", "ms": ssec * 1e3}
    out["wall_s"] = wall
    return out


HETERO_SHARES = tuple(k / 10 for k in range(11))  # GPU shares 0 %, 10 %, ..., 100 % (Sec. 4)


def run_hetero(args):
    """The paper's GPU share (Eq. 2, Sec. 4): the swept advance split between the GPU (tile rows
    below the share) and the host cores, shares 0 ... 100 % in 10 % steps.  Heat FP64 (r = 0.2,
    16 Fourier modes) on the paper's array sizes (500 steps, tile 32) and on the 4096^2 grid of the
    default workload (tile 64, --advance-steps steps, default 100); Euler FP64 (vortex, CFL 0.4,
    tile 16, 500 steps) on the two smallest sizes.  Each (grid, share) is timed over one advance
    after a warm advance; every result is checked bit for bit against the all-GPU advance."""
    import numpy as np
    import torch

    from paper_2105_10332_amd import problems
    from paper_2105_10332_amd.solver import EULER, HEAT, SweptHetero, SweptSolver, swept_cfl_dt

    cases = [("heat", n, 32, 500) for n in STUDY_SIZES] + [("heat", 4096, 64, args.advance_steps or 100)]
    cases += [("euler", n, 16, 500) for n in STUDY_SIZES[:2]]
    table, t_all, threads = {}, time.perf_counter(), None
    for kind, n, tile, M in cases:
        if kind == "heat":
            x0 = torch.tensor(problems.heat_fourier_modes(n), device="cuda")
            code, dt, L = HEAT, 0.2 / n / n, 1.0
        else:
            x0 = torch.tensor(problems.shu_vortex(n), device="cuda")
            code, dt, L = EULER, swept_cfl_dt(x0, 10.0, 0.4), 10.0
        x = x0.clone()
        sv = SweptSolver(code, x, dt=dt, length=L, alpha=1.0, gamma=1.4, tile=tile)
        sv.swept_advance(M)
        x.copy_(x0)
        ref_sec, _ = timed(lambda: sv.swept_advance(M), 1)
        ref = x.clone()
        row = {}
        for share in HETERO_SHARES:
            h = SweptHetero(sv, share, args.threads)
            threads = h.query()[2]
            x.copy_(x0)
            h.swept_hetero_advance(min(M, 2 * tile))  # warm: pinned buffers and worker threads
            x.copy_(x0)
            torch.cuda.synchronize()
            t = time.perf_counter()
            h.swept_hetero_advance(M)
            el = time.perf_counter() - t
            g, c, _ = h.query()
            h.close()
            if not torch.equal(x, ref):
                raise RuntimeError(f"{kind} {n} share {share}: result differs from the all-GPU advance")
            row[f"{share:.1f}"] = {"ms": el * 1e3, "gpu_rows": g, "cpu_rows": c}
        sv.close()
        best = min(row, key=lambda k: row[k]["ms"])
        table[f"{kind} {n}"] = {"tile": tile, "steps": M, "all_gpu_swept_ms": ref_sec * 1e3, "by_share": row,
                                "fastest_share": best}
        print(f"hetero {kind} {n}: " + ", ".join(f"{k}:{v['ms']:.1f}" for k, v in row.items()), file=sys.stderr,
              flush=True)
    cfg = {"workload": "GPU share of the swept advance (Eq. 2), 0-100% in 10% steps: heat FP64 r=0.2 on "
                       f"{list(STUDY_SIZES)} (500 steps, tile 32) and 4096^2 (tile 64), Euler FP64 vortex on "
                       f"{list(STUDY_SIZES[:2])} (500 steps, tile 16); host worker threads {threads}",
           "shares": list(HETERO_SHARES)}
    c2 = table["heat 4096"]
    out = base_record(args, c2["all_gpu_swept_ms"] / c2["by_share"]["0.9"]["ms"],
                      "x (all-GPU swept time / time at a GPU share of 90%, heat 4096^2)",
                      time.perf_counter() - t_all, "f64", cfg)
    out["ms_per_step"] = None
    out["table"] = table
    out["host_threads"] = threads
    return out


STUDY_SIZES = (320, 480, 640, 800, 960, 1120)  # array edges of the paper's parameter study (Sec. 4)
STUDY_TILES = (8, 12, 16, 24, 32)                # its block sizes


def run_study(args):
    """The paper's one-node parameter study at a GPU share of 100%: speedup S = R_standard /
    R_swept (Sec. 4) over its array sizes and block sizes, heat and Euler, 500 time steps.
    Pairs the library rejects (N % b != 0, LDS) are left out.  For each (kind, N, b) the
    workgroup size is the fastest of 64 ... 1024 (heat) or 64 ... 256 (Euler) on one advance;
    then swept and Standard are each timed over args.steps advances."""
    import math

    import torch

    from paper_2105_10332_amd import _lib, problems
    from paper_2105_10332_amd.solver import EULER, HEAT, SweptSolver, swept_cfl_dt, swept_workspace_bytes, make_problem

    dt_name = args.dtype or "f64"
    tdt = torch.float64 if dt_name == "f64" else torch.float32
    M = args.advance_steps or 500
    k = max(1, args.steps)
    table, logs = {"heat": {}, "euler": {}}, []
    t_all = time.perf_counter()
    for kind in ("heat", "euler"):
        for n in STUDY_SIZES:
            if kind == "heat":
                x0 = torch.tensor(problems.heat_fourier_modes(n), dtype=tdt, device="cuda")
                dt, L, code = 0.2 / n / n, 1.0, HEAT
            else:
                q64 = torch.tensor(problems.shu_vortex(n), device="cuda")
                dt, L, code = swept_cfl_dt(q64, 10.0, 0.4), 10.0, EULER
                x0 = q64.to(tdt)
            row = {}
            std = None
            for b in STUDY_TILES:
                try:
                    swept_workspace_bytes(make_problem(code, n, tdt, dt, L, 1.0, 1.4), b, 0)
                except _lib.SweptError:
                    continue
                best = None
                for wg in (64, 128, 256, 512, 1024):
                    st = x0.clone()
                    sv = SweptSolver(code, st, dt=dt, length=L, alpha=1.0, gamma=1.4, tile=b, wg=wg)
                    sv.swept_advance(M)
                    sec, _ = timed(lambda: sv.swept_advance(M), 1)
                    if best is None or sec < best[0]:
                        best = (sec, wg)
                    sv.close()
                st = x0.clone()
                sv = SweptSolver(code, st, dt=dt, length=L, alpha=1.0, gamma=1.4, tile=b, wg=best[1])
                sv.swept_advance(M)
                sw, _ = timed(lambda: sv.swept_advance(M), k)
                if std is None:
                    sv.standard_advance(M)
                    std, _ = timed(lambda: sv.standard_advance(M), k)
                sv.close()
                row[b] = {"S": std / sw, "swept_ms": sw / k * 1e3, "wg": best[1]}
            for b in row:
                row[b]["standard_ms"] = std / k * 1e3
            table[kind][n] = row
            logs.append(f"{kind} {n}: " + ", ".join(f"b{b} S={v['S']:.2f}" for b, v in row.items()))
            print(logs[-1], file=sys.stderr, flush=True)
    heat_s = [v["S"] for row in table["heat"].values() for v in row.values()]
    euler_s = [v["S"] for row in table["euler"].values() for v in row.values()]
    gmean = math.exp(sum(math.log(v) for v in heat_s) / len(heat_s))

    def best_of(kind):
        return {n: max(row.items(), key=lambda kv: kv[1]["S"])[0] for n, row in table[kind].items()}

    cfg = {"workload": f"parameter study: heat (r=0.2, 16 Fourier modes) and Euler (vortex eps 5, CFL 0.4) on "
                       f"N x N, N in {list(STUDY_SIZES)}, block sizes {list(STUDY_TILES)} where valid, {M} steps, "
                       f"GPU share 100%", "sizes": list(STUDY_SIZES), "tiles": list(STUDY_TILES)}
    out = base_record(args, gmean, "x (Standard time / Swept time, geometric mean over heat cases)",
                      time.perf_counter() - t_all, dt_name, cfg)
    out["ms_per_step"] = None
    out["table"] = table
    out["range"] = {"heat": [min(heat_s), max(heat_s)], "euler": [min(euler_s), max(euler_s)]}
    out["best_tile"] = {"heat": best_of("heat"), "euler": best_of("euler")}
    return out


def run_graphs(args):
    """Launch overhead at the paper's small array sizes: heat FP64, 500 steps, b = 32, each
    advance issued eagerly (one call per launch) and replayed from a captured HIP graph,
    for the swept and the Standard solver."""
    import torch

    from paper_2105_10332_amd import problems
    from paper_2105_10332_amd.solver import HEAT, SweptSolver

    M = args.advance_steps or 500
    k = max(1, args.steps)
    rows = {}
    t_all = time.perf_counter()
    for n in (320, 1024):
        x = torch.tensor(problems.heat_fourier_modes(n), device="cuda")
        s = SweptSolver(HEAT, x, dt=0.2 / n / n, length=1.0, alpha=1.0, tile=32, wg=512)
        row = {}
        for method in ("swept", "standard"):
            fn = getattr(s, method + "_advance")
            fn(M)
            eager, _ = timed(lambda: fn(M), k)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                fn(1)
            torch.cuda.current_stream().wait_stream(side)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn(M)
            g.replay()
            graph, _ = timed(g.replay, k)
            row[method] = {"eager_ms": eager / k * 1e3, "graph_ms": graph / k * 1e3}
        row["S_eager"] = row["standard"]["eager_ms"] / row["swept"]["eager_ms"]
        row["S_graph"] = row["standard"]["graph_ms"] / row["swept"]["graph_ms"]
        s.close()
        rows[n] = row
        print(f"graphs {n}: {row}", file=sys.stderr, flush=True)
    cfg = {"workload": f"heat N x N FP64, N in (320, 1024), r=0.2, {M} steps, b=32 wg 512: each advance eager "
                       f"and as a replayed HIP graph", "sizes": [320, 1024]}
    out = base_record(args, rows[320]["S_graph"], "x (Standard / Swept time, both replayed from graphs, N=320)",
                      time.perf_counter() - t_all, "f64", cfg)
    out["ms_per_step"] = None
    out["table"] = rows
    return out


def copy_reference(n: int = 4096, reps: int = 3):
    """A plain device-to-device copy of one n x n FP64 state, reps times: the known-size
    traffic that scales the HBM counters of the profiles."""
    import torch

    x = torch.ones(n * n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_bytes_each_way": x.numel() * 8, "copies": reps}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (the swept path here is single-device); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_reference:
        copy_reference()
        return
    fn = {"heat": run_heat, "euler": run_euler, "adjoint": run_adjoint, "batch": run_batch,
          "study": run_study, "graphs": run_graphs, "hetero": run_hetero}[args.workload]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
