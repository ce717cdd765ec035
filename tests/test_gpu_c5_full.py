"""The batched ensemble at its full size and length, built as the benchmark builds it
(48 heat problems with edges 128-1024 and r in [0.05, 0.24], 16 Euler vortices with edges
256-1024 and strength 1-5, FP32, 200 steps, the tuned batch tiles): one batched advance
equals each problem's own swept advance bit for bit and the FP32 oracle of each problem
(0 measured for all 64)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2105_10332_amd import problems, tune
from paper_2105_10332_amd.solver import EULER, HEAT, SweptBatch, SweptSolver, swept_cfl_dt

from gpu_helpers import DEV, rel_err

pytestmark = pytest.mark.gpu
STEPS = 200


def test_c5_full_ensemble():
    ens = problems.batch_ensemble()
    tiles = tune.batch_tiles([(it.kind, it.n) for it in ens], "f32")
    items = []
    for it, tile in zip(ens, tiles):
        n = it.n
        if it.kind == "heat":
            x = torch.tensor(problems.heat_fourier_modes(n, seed=it.seed), dtype=torch.float32, device=DEV)
            items.append((HEAT, x, it.r / n / n, 1.0, 1.0, 1.4, tile))
        else:
            q0 = torch.tensor(problems.shu_vortex(n, eps=it.eps), device=DEV)
            dt = swept_cfl_dt(q0, 10.0, 0.4)
            items.append((EULER, q0.to(torch.float32), dt, 10.0, 1.0, 1.4, tile))
    init = [it[1].cpu().numpy().copy() for it in items]
    own = []
    for kind, x, dt, length, alpha, gamma, tile in items:
        y = x.clone()
        s = SweptSolver(kind, y, dt=dt, length=length, alpha=alpha, gamma=gamma, tile=tile)
        s.swept_advance(STEPS)
        own.append((y, s.info.r))
        s.close()
    print(f"C5: {len(items)} problems, FP32, {STEPS} steps", flush=True)
    b = SweptBatch(items)
    b.swept_batch_advance(STEPS)
    torch.cuda.synchronize()
    worst = 0.0
    for q, ((kind, x, dt, *_), (y, r)) in enumerate(zip(items, own)):
        assert torch.equal(x, y), (q, ens[q])
        got = x.cpu().numpy()
        n = got.shape[-1]
        if kind == HEAT:
            ref = oracle.heat_run(init[q], r, STEPS)
        else:
            ref = oracle.euler_run(init[q], dt, 10 / n, 10 / n, 1.4, STEPS)
        worst = max(worst, rel_err(got, ref))
    print(f"C5 batch vs FP32 oracle, worst problem: {worst:.3e}")
    assert worst <= 1e-6
