"""FP32 heat windows inside the domain write their outputs once, after the
shape's last level, instead of level by level (device_common.h,
heat_store_inner).  This checks on the CPU, for every shape type, tile and cut
at the final level, that the closed forms the kernel uses for the cells
written from each level-parity buffer equal the per-level store rule of the
memory protocol: the union over the shape's levels l of F(l) minus F(l+2),
with F(l+2) empty past the shape's last level (Sec. 3.3 shapes; n = 1).  It
also checks that a cell's write under the per-level rule comes from its last
computed level of that parity, which is the value its LDS slot holds at the
end, and that a plausible slip in the Bridge parity is caught."""
import pytest

from paper_2105_10332_amd.geometry import half_width
from swept_sim import Geom


def footprint(g, wx, wy, lvl):
    """Cells (ax, ay), by distance index from the window centre, of the footprint of level lvl."""
    hx, hy = half_width(wx, lvl, g.h, 1), half_width(wy, lvl, g.h, 1)
    return {(ax, ay) for ax in range(hx) for ay in range(hy)}


def per_level_rule(g, wx, wy):
    lo, hi = g.levels(wx, wy)
    sets = {0: {}, 1: {}}
    for lvl in range(lo, hi + 1):
        nxt = footprint(g, wx, wy, lvl + 2) if lvl + 2 <= hi else set()
        for c in footprint(g, wx, wy, lvl) - nxt:
            assert c not in sets[lvl & 1], "a cell is stored twice at one parity"
            sets[lvl & 1][c] = lvl
    return sets


def closed_form(g, wx, wy, lo, hi, ax, ay, parity_slip=False):
    """Membership of the two parities as heat_store_inner evaluates it."""
    h = g.h
    wsh = (max(wx, wy) - 1) * h
    t0, t1 = lo - wsh, hi - wsh
    if wx == wy:
        M = [0, 0]
        for t in range(t0, t1 + 1):
            M[(t + wsh) & 1] = max(M[(t + wsh) & 1], min(t, 2 * h - t))
        a = max(ax, ay)
        return a < M[0], a < M[1]
    a, s = (ax, ay) if wx > wy else (ay, ax)
    tlo, thi = max(a + 1, t0), min(h - s - 1, t1)
    anyt, two = tlo <= thi, tlo < thi
    plo = ((wsh + parity_slip) & 1) ^ (tlo & 1)
    return anyt and (two or plo == 0), anyt and (two or plo == 1)


def shapes_of(g, L):
    for phase in range(1, 2 * (L // g.h) + 6):
        for wx, wy in g.shapes(phase):
            lo, hi = g.levels(wx, wy)
            if max(wx, wy) >= 1 and lo <= hi:
                yield wx, wy, lo, hi


@pytest.mark.parametrize("b", [4, 6, 8, 16, 32, 64])
def test_end_of_shape_store_sets_equal_per_level_rule(b):
    h = b // 2
    checked = 0
    for L in (3 * h + 1, 5 * h, 7 * h - 1, 9 * h + 2):
        g = Geom(4 * b, b, 1, L)
        for wx, wy, lo, hi in shapes_of(g, L):
            sets = per_level_rule(g, wx, wy)
            for ax in range(h + 1):  # the kernel visits distance indices 0..h-1 of each half
                for ay in range(h + 1):
                    got = closed_form(g, wx, wy, lo, hi, ax, ay)
                    assert got == ((ax, ay) in sets[0], (ax, ay) in sets[1]), (b, L, wx, wy, ax, ay)
            for p in (0, 1):  # the stored value is the cell's last computed level of that parity
                for c, lvl in sets[p].items():
                    assert not [m for m in range(lvl + 2, hi + 1, 2) if c in footprint(g, wx, wy, m)]
            checked += 1
    assert checked > 0


def test_parity_slip_is_detected():
    g = Geom(64, 16, 1, 41)
    bad = 0
    for wx, wy, lo, hi in shapes_of(g, 41):
        if wx == wy:
            continue
        sets = per_level_rule(g, wx, wy)
        for ax in range(g.h):
            for ay in range(g.h):
                got = closed_form(g, wx, wy, lo, hi, ax, ay, parity_slip=True)
                bad += got != ((ax, ay) in sets[0], (ax, ay) in sets[1])
    assert bad > 0
