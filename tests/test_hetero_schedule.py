"""CPU proof of the heterogeneous split's exchange rule (Sec. 3.2, Eq. 2).

The GPU runs the shape instances of tile rows jy < G, the host cores the
others, each on its own copy of the two level-parity buffers.  After every
phase the two copies are merged on the band rows (rows within b of the row
boundaries 0 and G*b): cells the host wrote in the phase take the host's
value on both sides, all other band cells the GPU's value.  At the end the
host's rows [G*b, N) of the final level go to the GPU.

This test runs that protocol on level tags only (which level each buffer
cell holds on each side) for every instance's reads and writes, as the
memory protocol defines them (tests/swept_sim.py): an instance of level l
reads Box(F(l), n) minus F(l-1) at level l-1 (and, two-stage with even
first level, F(l) at level l-2) and writes F(l) minus F(l+2) at level l.
Every read must find the right level in its side's copy, and the GPU's copy
must hold level L everywhere at the end -- for every split G, so the result
equals the all-GPU advance bit for bit.  A band narrower than the reach of
a window must fail (negative control).
"""
from __future__ import annotations

import numpy as np
import pytest

from swept_sim import Geom


def _instances(g: Geom, phase: int):
    for (wx, wy) in g.shapes(phase):
        for jy in range(g.tiles):
            for jx in range(g.tiles):
                yield wx, wy, jx, jy


def _rect(g: Geom, f, grow=0):
    if f is None:
        return set()
    xs = range(f[0] - grow, f[1] + grow)
    ys = range(f[2] - grow, f[3] + grow)
    return {(y % g.N, x % g.N) for y in ys for x in xs}


def _reads_writes(g: Geom, two_stage: bool, wx, wy, jx, jy):
    lo, hi = g.levels(wx, wy)
    reads, writes = [], []
    for lvl in range(lo, hi + 1):
        F = g.footprint(wx, wy, jx, jy, lvl)
        if F is None:
            continue
        prev = _rect(g, g.footprint(wx, wy, jx, jy, lvl - 1)) if lvl > lo else set()
        reads += [((lvl - 1) % 2, c, lvl - 1) for c in _rect(g, F, g.n) - prev]
        if two_stage and lvl % 2 == 0 and lvl == lo:
            reads += [(lvl % 2, c, lvl - 2) for c in _rect(g, F)]
        f2 = g.footprint(wx, wy, jx, jy, lvl + 2) if lvl + 2 <= hi else None
        writes += [(lvl % 2, c, lvl) for c in _rect(g, F) - _rect(g, f2)]
    return reads, writes


def run_split(g: Geom, G: int, two_stage: bool, band_halfwidth: int | None = None):
    """Level-tag run of the split; raises AssertionError on a stale read."""
    N, b = g.N, g.b
    B = b if band_halfwidth is None else band_halfwidth
    dev = [np.full((N, N), -1), np.full((N, N), -1)]
    dev[0][:] = 0
    host = [dev[0].copy(), np.full((N, N), -9)]  # buffer 1 on the host starts unrelated
    band = set()
    if 0 < G < g.tiles:
        for Y in (0, G * b):
            band |= {(Y + d) % N for d in range(-B, B)}
    band = sorted(band)
    for phase in range(g.n_phases()):
        marks = [np.zeros((N, N), bool), np.zeros((N, N), bool)]
        dev_writes, host_writes = [], []
        for (wx, wy, jx, jy) in _instances(g, phase):
            on_gpu = jy < G
            side = dev if on_gpu else host
            reads, writes = _reads_writes(g, two_stage, wx, wy, jx, jy)
            for (buf, (y, x), lvl) in reads:
                assert side[buf][y, x] == lvl, (
                    f"{'gpu' if on_gpu else 'host'} instance {(wx, wy, jx, jy)} phase {phase} reads "
                    f"buffer {buf} cell {(y, x)}: level {side[buf][y, x]} instead of {lvl}")
            (dev_writes if on_gpu else host_writes).extend(writes)
        for (buf, (y, x), lvl) in dev_writes:  # instances of a phase read nothing their phase writes
            dev[buf][y, x] = lvl
        for (buf, (y, x), lvl) in host_writes:
            host[buf][y, x] = lvl
            marks[buf][y, x] = True
        for buf in range(2):
            for y in band:
                m = marks[buf][y]
                host[buf][y, ~m] = dev[buf][y, ~m]
                dev[buf][y, m] = host[buf][y, m]
    fb = g.L % 2
    if G < g.tiles:
        dev[fb][G * b:] = host[fb][G * b:]
    assert np.all(dev[fb] == g.L), "the GPU's copy does not hold the final level everywhere"


CASES = [
    (32, 8, 1, 11), (48, 8, 1, 9), (64, 16, 1, 21), (32, 8, 2, 14), (48, 8, 2, 10), (64, 16, 2, 18),
]


@pytest.mark.parametrize("N,b,n,L", CASES)
def test_every_split_reads_current_values(N, b, n, L):
    g = Geom(N, b, n, L)
    for G in range(0, g.tiles + 1):
        run_split(g, G, two_stage=(n == 2))


def test_narrow_band_is_detected():
    """Negative control: a band that stops short of a window's reach gives a stale read."""
    g = Geom(64, 16, 1, 21)
    with pytest.raises(AssertionError):
        run_split(g, 2, two_stage=False, band_halfwidth=4)
