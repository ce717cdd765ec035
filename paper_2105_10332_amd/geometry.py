"""Host-side accounting of the swept plan: phases, launches, cell-levels and the
algorithmic HBM traffic of the phase kernels (values loaded and stored).

This mirrors the loop bounds of the phase kernel in csrc/kernels.hip (one
workgroup per shape instance; per level l it loads Box(F(l), n) minus F(l-1)
and stores F(l) minus F(l+2)); every instance of a phase has the same shape,
so per-phase totals are one instance's sums times the instance count.  Used
for reporting (roofline, effective bandwidth), not by the solver.
"""
from __future__ import annotations

from dataclasses import dataclass


def half_width(w: int, lvl: int, h: int, n: int) -> int:
    t = lvl - (w - 1) * h
    if lvl < 1 or t < 1 or t > 2 * h - 1:
        return 0
    return n * min(t, 2 * h - t)


@dataclass
class PhaseStats:
    phase: int
    instances: int
    cell_levels: int
    loads: int    # cell values read from HBM (per variable)
    stores: int   # cell values written to HBM (per variable)


def plan(N: int, b: int, n: int, L: int, two_stage: bool = False):
    """Per-phase statistics of one swept advance of L levels."""
    h = b // (2 * n)
    tiles = N // b
    W = -(-L // h) if L > 0 else 0
    out = []
    for p in range(2 * W + 1 if L > 0 else 0):
        shapes = [(p // 2, p // 2)] if p % 2 == 0 else [((p + 1) // 2, (p - 1) // 2), ((p - 1) // 2, (p + 1) // 2)]
        cl = ld = st = 0
        for wx, wy in shapes:
            lo = max(1, (max(wx, wy) - 1) * h + 1)
            hi = min(L, (min(wx, wy) + 1) * h - 1)
            c1 = l1 = s1 = 0
            for lvl in range(lo, hi + 1):
                hx, hy = half_width(wx, lvl, h, n), half_width(wy, lvl, h, n)
                area = 4 * hx * hy
                c1 += area
                box = (2 * hx + 2 * n) * (2 * hy + 2 * n)
                prev = 4 * half_width(wx, lvl - 1, h, n) * half_width(wy, lvl - 1, h, n) if lvl > lo else 0
                l1 += box - prev
                if two_stage and lvl == lo and lvl % 2 == 0:
                    l1 += area
                if lvl + 2 <= hi:  # |F(l) & F(l+2)|: bridges grow on one axis, so intersect per axis
                    keep = 4 * min(hx, half_width(wx, lvl + 2, h, n)) * min(hy, half_width(wy, lvl + 2, h, n))
                else:
                    keep = 0
                s1 += area - keep
            cl += c1 * tiles * tiles
            ld += l1 * tiles * tiles
            st += s1 * tiles * tiles
        out.append(PhaseStats(p, len(shapes) * tiles * tiles, cl, ld, st))
    return out


def totals(N: int, b: int, n: int, L: int, two_stage: bool = False):
    ps = plan(N, b, n, L, two_stage)
    return {
        "launches": len(ps),
        "cell_levels": sum(p.cell_levels for p in ps),
        "loads": sum(p.loads for p in ps),
        "stores": sum(p.stores for p in ps),
    }


def ring_load_parities(wx: int, wy: int, lo: int, hi: int, h: int, n: int, b: int, lx: int, ly: int,
                       two_stage: bool = False):
    """Which level-parity buffers the phase kernel's up-front load fills at local cell
    (lx, ly) of the (b+2n)^2 window of shape (wx, wy) cut to levels [lo, hi]; returns a
    dict parity -> level of the value loaded.  Mirrors the kernel's closed form.

    A cell belongs to ring(l) = Box(F(l), n) minus F(l-1) (F(lo-1) empty) and is then
    loaded at level l-1 into buffer (l-1) % 2; rings of one parity never overlap.  With
    t = l - (w-1)h the level within the window and a the cell's distance index from the
    centre along a growing axis (a < hw <=> inside), ring(t) holds the cells with
    (t-1)n <= a < (t+1)n, so the two candidate levels t = floor(a/n), floor(a/n)+1
    have opposite parities and each parity has at most one:
      * Octahedron w >= 1 (both axes grow for t <= h): a = max(ax, ay), t <= min(h, tmax);
      * Bridge (w, w-1): a = ax (grows), and the shrinking axis needs ay < (h-t+1)n;
        the Y-Bridge swaps the axes; t <= min(h-1, tmax);
      * Up-Pyramid (w = 0): only the first level, the tile itself (max(ax, ay) < b/2) at
        level 0;
    tmax = hi - (w-1)h.  A two-stage scheme whose first level lo is even also needs F(lo)
    at level lo-2 (buffer lo % 2)."""
    C = b // 2 + n
    ax = lx - C if lx >= C else C - 1 - lx
    ay = ly - C if ly >= C else C - 1 - ly
    out = {}
    wmax = max(wx, wy)
    if wmax == 0:
        if max(ax, ay) < b // 2:
            out[0] = 0
        return out
    base = (wmax - 1) * h  # level = base + t
    tmax = hi - base
    if wx == wy:
        a, other_ok = max(ax, ay), (lambda t: True)
        tcap = min(h, tmax)
    else:
        a, s = (ax, ay) if wx > wy else (ay, ax)
        other_ok = (lambda t, s=s: s < (h - t + 1) * n)
        tcap = min(h - 1, tmax)
    t1 = a // n
    for t in (t1, t1 + 1):
        if 1 <= t <= tcap and other_ok(t):
            out[(base + t - 1) % 2] = base + t - 1
    if two_stage and lo % 2 == 0:
        hx = half_width(wx, lo, h, n)
        hy = half_width(wy, lo, h, n)
        if ax < hx and ay < hy:
            assert lo % 2 not in out
            out[lo % 2] = lo - 2
    return out
