"""Host check of the Euler walls' index arithmetic (CPU only).

A face whose four-cell run reaches across the domain edge reads, instead of
the wrapped cells, ghost cells from its own side: the edge cell (zero
gradient) or the mirrored cell (slip wall), and the first cell past the edge
recomputes its own wall face.  This restates the window-local index rules of
the kernels and checks, for every swept shape, level and Standard tile of a
range of grids, that every index read lies inside the face run's own range,
the pressure pass's range and the window, and that a window meets the edge at
most once."""
import itertools

import pytest

from swept_sim import Geom


def wall_cell(m, E, left, bc):
    if (m < E) if left else (m >= E):
        return m
    if bc == 3:
        return 2 * E - 1 - m
    return E - 1 if left else E


def window_edge(o, W, N):
    return -o if o < 0 else (N - o if o + W > N else -(1 << 20))


def _check_level(x0, fw, E, W, bc):
    lo, hi = x0 - 2, x0 + fw + 2  # cells the pressure pass covers
    assert 0 <= lo and hi <= W
    for k in range(fw + 1):  # faces after local cells a = x0 - 1 .. x0 + fw - 1
        a = x0 - 1 + k
        if a - 1 < E <= a + 2:
            for o in range(4):
                m = wall_cell(a - 1 + o, E, a < E, bc)
                assert a - 1 <= m <= a + 2 and lo <= m < hi
    if x0 <= E < x0 + fw:  # the first cell past the edge recomputes its wall face
        for o in range(4):
            m = wall_cell(E - 2 + o, E, False, bc)
            assert E - 2 <= m <= E + 1 and lo <= m < hi


def _std_tile(N):
    return 16 if (N % 16 == 0 and N >= 24) else (8 if (N % 8 == 0 and N >= 16) else 4)


@pytest.mark.parametrize("N,b", [(16, 8), (24, 8), (32, 16), (48, 16), (64, 32), (36, 12), (96, 32)])
def test_wall_reads_stay_inside_the_run(N, b):
    g = Geom(N, b, 2, 40)
    W, C = b + 4, b // 2 + 2
    for phase in range(g.n_phases()):
        for (wx, wy) in g.shapes(phase):
            lo, hi = g.levels(wx, wy)
            for jx, jy in itertools.product(range(g.tiles), repeat=2):
                ox, oy = g.centre(wx, jx) - C, g.centre(wy, jy) - C
                assert W <= N  # one edge per window and axis
                ex, ey = window_edge(ox, W, N), window_edge(oy, W, N)
                for lvl in range(lo, hi + 1):
                    F = g.footprint(wx, wy, jx, jy, lvl)
                    if F is None:
                        continue
                    for bc in (2, 3):
                        _check_level(F[0] - ox, F[1] - F[0], ex, W, bc)
                        _check_level(F[2] - oy, F[3] - F[2], ey, W, bc)
    TS = _std_tile(N)
    Ws = TS + 8
    assert Ws <= N  # the Standard window meets the edge at most once
    for t in range(N // TS):
        E = window_edge(t * TS - 4, Ws, N)
        for bc in (2, 3):
            _check_level(2, TS + 4, E, Ws, bc)
            _check_level(4, TS, E, Ws, bc)
