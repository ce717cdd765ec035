"""Autotuner for the swept solver: picks the tile edge b (which fixes the swept
depth k = b/(2n) - 1 levels per window, Eq. 1) and the workgroup size by
timing candidates on the GPU, and caches the winner as JSON.

The paper finds the best block size hardware- and problem-dependent and
recommends tuning (Sec. 5-6); this automates that per (problem kind,
precision, grid edge, GPU architecture).  Cache location: $SWEPT_TUNE_CACHE
or tune_cache.json next to this file.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path() -> str:
    return os.environ.get("SWEPT_TUNE_CACHE", os.path.join(HERE, "tune_cache.json"))


def _arch() -> str:
    try:
        import torch

        if torch.cuda.is_available():
            return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        pass
    return "gfx950"


def _key(kind: str, dtype: str, n: int, arch: str | None = None) -> str:
    return f"{kind}/{dtype}/{n}/{arch or _arch()}"


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict):
    p = cache_path()
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def candidates(kind: str, dtype: str, n: int):
    """Tiles the library accepts for this grid (b > 2n, b % 2n == 0, n_grid % b == 0,
    n_grid >= 2b, LDS fits; checked by swept_workspace_bytes on the host) x workgroup sizes."""
    from . import _lib
    from .solver import EULER, HEAT, make_problem, swept_workspace_bytes

    import torch

    k = HEAT if kind == "heat" else EULER
    tdt = torch.float64 if dtype == "f64" else torch.float32
    dt = 0.2 / (n * n) if kind == "heat" else 1e-4  # any valid time step: only the geometry matters here
    prob = make_problem(k, n, tdt, dt, 1.0 if kind == "heat" else 10.0, 1.0)
    tiles = []
    for b in (8, 12, 16, 24, 32, 48, 64):
        try:
            swept_workspace_bytes(prob, b, 0)
        except _lib.SweptError:
            continue
        tiles.append(b)
    wgs = (64, 128, 256, 512, 1024) if kind == "heat" else (128, 256, 512, 1024)
    return [(b, wg) for b in tiles for wg in wgs]


def default_tile(kind: str, dtype: str, n: int) -> int:
    order = {"heat": (64, 32, 16, 8), "euler": (16, 32, 8)}[kind]
    valid = {b for b, _ in candidates(kind, dtype, n)}
    for b in order:
        if b in valid:
            return b
    return min(valid) if valid else 0


def best(kind: str, dtype: str, n: int):
    """(tile, wg) from the cache, else the heuristic default (wg 0 = library default)."""
    e = load_cache().get(_key(kind, dtype, n))
    if e:
        return int(e["tile"]), int(e["wg"])
    return default_tile(kind, dtype, n), 0


def best_tile(kind: str, dtype: str, n: int) -> int:
    return best(kind, dtype, n)[0]


def tune(kind: str, dtype: str, n: int, steps: int = 0, reps: int = 3, save: bool = True, verbose: bool = False):
    """Time every candidate on the GPU (swept advance of `steps` steps, default a few
    windows of the deepest tile) and cache the fastest."""
    import torch

    from . import problems
    from .solver import EULER, HEAT, SweptSolver

    dev = torch.device("cuda", 0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if kind == "heat":
        x0 = torch.tensor(problems.heat_fourier_modes(n), dtype=tdt, device=dev)
        mk = lambda b, wg, x: SweptSolver(HEAT, x, dt=0.2 / n / n, length=1.0, alpha=1.0, tile=b, wg=wg)
        steps = steps or 512
    else:
        x0 = torch.tensor(problems.shu_vortex(n), dtype=tdt, device=dev)
        mk = lambda b, wg, x: SweptSolver(EULER, x, dt=0.4 * (10.0 / n) / 6.0, length=10.0, tile=b, wg=wg)
        steps = steps or 64
    results = []
    for b, wg in candidates(kind, dtype, n):
        x = x0.clone()
        s = mk(b, wg, x)
        s.swept_advance(steps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            s.swept_advance(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        results.append((ms, b, wg))
        if verbose:
            print(f"tune {kind} {dtype} n={n}: tile {b} wg {wg}: {ms:.3f} ms", flush=True)
        s.close()
    results.sort()
    ms, b, wg = results[0]
    if save:
        c = load_cache()
        c[_key(kind, dtype, n)] = {"tile": b, "wg": wg, "ms": ms, "steps": steps,
                                   "all": [[r[1], r[2], round(r[0], 4)] for r in results]}
        save_cache(c)
    return b, wg, results


# ---------------------------------------------------------------- batches
# One persistent launch runs every problem's phases in lockstep global
# phases, so a batch has its own best tiles: the deepest tile that fits a
# problem cuts its phase count, while the largest LDS window sets how many
# workgroups share a compute unit.  The batch tuner times a preferred tile
# per problem kind (each problem takes the largest valid tile not above it).

BATCH_PREFS = {"heat": (64, 32, 16), "euler": (32, 16)}
BATCH_DEFAULT = {"heat": 64, "euler": 32}


def _batch_key(specs, dtype: str, arch: str | None = None) -> str:
    import hashlib

    sig = hashlib.sha256(repr(sorted((k, int(n)) for k, n in specs)).encode()).hexdigest()[:12]
    return f"batch/{dtype}/{len(specs)}x{sig}/{arch or _arch()}"


def tile_at_most(kind: str, dtype: str, n: int, pref: int) -> int:
    valid = sorted({b for b, _ in candidates(kind, dtype, n)})
    below = [b for b in valid if b <= pref]
    return below[-1] if below else (valid[0] if valid else 0)


def batch_tiles(specs, dtype: str, prefs: dict | None = None):
    """Tile per problem of a batch given as [(kind, n), ...]: from the batch cache entry
    for this ensemble if there is one, else the batch defaults."""
    if prefs is None:
        e = load_cache().get(_batch_key(specs, dtype))
        prefs = {"heat": int(e["heat"]), "euler": int(e["euler"])} if e else BATCH_DEFAULT
    return [tile_at_most(k, dtype, n, prefs[k]) for k, n in specs]


def tune_batch(specs, dtype: str, steps: int = 64, reps: int = 2, save: bool = True, verbose: bool = False):
    """Time the batch for every pair of preferred tiles and cache the fastest."""
    import itertools

    import torch

    from . import problems
    from .solver import EULER, HEAT, SweptBatch

    dev = torch.device("cuda", 0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    states = []
    for k, n in specs:
        if k == "heat":
            states.append(torch.tensor(problems.heat_fourier_modes(n), dtype=tdt, device=dev))
        else:
            states.append(torch.tensor(problems.shu_vortex(n), dtype=tdt, device=dev))
    results = []
    for hp, ep in itertools.product(BATCH_PREFS["heat"], BATCH_PREFS["euler"]):
        tiles = batch_tiles(specs, dtype, {"heat": hp, "euler": ep})
        items = []
        for (k, n), x, b in zip(specs, states, tiles):
            if k == "heat":
                items.append((HEAT, x.clone(), 0.2 / n / n, 1.0, 1.0, 1.4, b))
            else:
                items.append((EULER, x.clone(), 0.4 * (10.0 / n) / 6.0, 10.0, 1.0, 1.4, b))
        try:
            bt = SweptBatch(items)
        except Exception:  # e.g. the largest window does not fit: not a candidate
            continue
        bt.swept_batch_advance(steps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            bt.swept_batch_advance(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        results.append((ms, hp, ep))
        if verbose:
            print(f"tune batch {dtype}: heat <= {hp}, euler <= {ep}: {ms:.3f} ms", flush=True)
        bt.close()
    results.sort()
    ms, hp, ep = results[0]
    if save:
        c = load_cache()
        c[_batch_key(specs, dtype)] = {"heat": hp, "euler": ep, "ms": ms, "steps": steps,
                                       "all": [[r[1], r[2], round(r[0], 4)] for r in results]}
        save_cache(c)
    return {"heat": hp, "euler": ep}, results
