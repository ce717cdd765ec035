"""CPU simulator of the swept schedule and of the GPU memory protocol.

Test infrastructure: an independent Python statement of the swept
decomposition (Sec. 3.3, Figs. 1-2) and of the exact load/compute/store
protocol the HIP phase kernels follow, executed on small grids with the
oracle's numpy stencil.  It proves, with no GPU:

* the shapes partition space-time exactly (every (cell, level) once);
* every value a shape reads is present, at the right level, in the buffer
  it reads (level-tag check), so the swept result equals Standard bit for
  bit (compared with the oracle);
* no two instances of one phase write the same buffer cell, and no instance
  reads a buffer cell another instance of its phase writes (the instances
  of a phase run concurrently);
* the HBM traffic of the protocol (values loaded and stored per phase).

Geometry (1D, applied per axis).  Radius n per level, tile b, window
h = b/(2n) levels.  Diamond w >= 0 is centred at tile centres j*b + b/2 when
w is even and at tile edges j*b when w is odd; it lives on levels
(w-1)h+1 .. (w+1)h-1 (levels >= 1) and at level l covers [c-hw, c+hw) with
hw = n*min(t, 2h-t), t = l-(w-1)h.  A 2D shape is a pair (wx, wy) with
|wx-wy| <= 1: (w, w) is Octahedron w (w = 0 is the Up-Pyramid, an
Octahedron cut at the final level is the Down-Pyramid) and runs in phase 2w;
(w, w-1) and (w-1, w) are the X- and Y-Bridges of window w and share phase
2w-1.  Every shape is cut at the final level L.

Memory protocol.  Two full-size buffers; level l of a cell lives in buffer
l mod 2.  For each level l of its shape an instance
  1. loads Box(F(l), n) minus F(l-1) at level l-1 from buffer (l-1) mod 2
     (F = footprint rectangle; Box = the rectangle grown by n on each side);
     for a two-stage scheme whose first level is even it also loads F(l) at
     level l-2 from buffer l mod 2;
  2. computes F(l) in its local window (two level-parity local buffers);
  3. stores the cells of F(l) that are not in F(l+2) to buffer l mod 2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from oracle import numpy_ref


# ------------------------------------------------------------------ geometry


@dataclass(frozen=True)
class Geom:
    N: int      # cells per side
    b: int      # tile edge
    n: int      # stencil radius per level
    L: int      # final level
    shift: int = 0  # 1: even diamonds centred at tile edges, odd ones at tile centres (the other tiling)

    @property
    def h(self) -> int:
        return self.b // (2 * self.n)

    @property
    def tiles(self) -> int:
        return self.N // self.b

    def n_phases(self) -> int:
        return 2 * math.ceil(self.L / self.h) + 1 if self.L > 0 else 0

    def centre(self, w: int, j: int) -> int:
        return j * self.b + (self.b // 2 if (w + self.shift) % 2 == 0 else 0)

    def half_width(self, w: int, lvl: int) -> int:
        t = lvl - (w - 1) * self.h
        if lvl < 1 or t < 1 or t > 2 * self.h - 1:
            return 0
        return self.n * min(t, 2 * self.h - t)

    def levels(self, wx: int, wy: int):
        lo = max(1, (max(wx, wy) - 1) * self.h + 1)
        hi = min(self.L, (min(wx, wy) + 1) * self.h - 1)
        return lo, hi

    def shapes(self, phase: int):
        if phase % 2 == 0:
            w = phase // 2
            return [(w, w)]
        w = (phase + 1) // 2
        return [(w, w - 1), (w - 1, w)]

    def footprint(self, wx, wy, jx, jy, lvl):
        """(x0, x1, y0, y1) in unwrapped global coordinates, or None if empty."""
        lo, hi = self.levels(wx, wy)
        if lvl < lo or lvl > hi:
            return None
        hx = self.half_width(wx, lvl)
        hy = self.half_width(wy, lvl)
        if hx == 0 or hy == 0:
            return None
        cx, cy = self.centre(wx, jx), self.centre(wy, jy)
        return (cx - hx, cx + hx, cy - hy, cy + hy)


def check_partition(g: Geom):
    """Every (cell, level) for levels 1..L is owned by exactly one shape instance, and the
    owner's phase is not later than that of anything reading it (dependencies go backwards)."""
    own = np.full((g.L + 1, g.N, g.N), -1, dtype=np.int64)
    for p in range(g.n_phases()):
        for (wx, wy) in g.shapes(p):
            for jx in range(g.tiles):
                for jy in range(g.tiles):
                    lo, hi = g.levels(wx, wy)
                    for lvl in range(lo, hi + 1):
                        f = g.footprint(wx, wy, jx, jy, lvl)
                        if f is None:
                            continue
                        xs = np.arange(f[0], f[1]) % g.N
                        ys = np.arange(f[2], f[3]) % g.N
                        sub = own[lvl][np.ix_(ys, xs)]
                        assert np.all(sub == -1), f"overlap at level {lvl}, phase {p}, shape {(wx, wy)}"
                        own[lvl][np.ix_(ys, xs)] = p
    assert np.all(own[1:] >= 0), "uncovered (cell, level)"
    return own


# ------------------------------------------------------------------ executor


@dataclass
class Traffic:
    loads: int = 0
    stores: int = 0
    per_phase: list = field(default_factory=list)


class ProtocolError(AssertionError):
    pass


class SweptSim:
    """Executes the swept schedule with the GPU memory protocol on the CPU."""

    def __init__(self, g: Geom, kind: str, params: dict, dtype=np.float64, store_lag: int = 2,
                 preload: bool = False):
        self.store_lag = store_lag  # stores F(l) minus F(l+store_lag); 2 is the protocol
        self.preload = preload      # issue every level's loads before the first compute
        self.g = g
        self.kind = kind
        self.p = params
        self.dtype = dtype
        self.nvar = 1 if kind == "heat" else 4
        self.W = g.b + 2 * g.n
        assert g.N % g.b == 0 and g.b % (2 * g.n) == 0 and g.N >= 2 * g.b

    # one level of the scheme on a local window; values outside the window garbage.
    # gx, gy: global column / row of each window cell (walls need them)
    def _compute(self, prev, prev2, lvl, gx=None, gy=None):
        if self.kind == "heat":
            bc = self.p.get("bc", 0)
            if bc == 0:
                return numpy_ref.heat_step(prev[0], self.p["r"])[None]
            T = prev[0]
            t = self.dtype
            N = self.g.N
            g = np.full_like(T, t(self.p.get("bcv", 0.0))) if bc == 1 else T
            xp = np.where(gx[None, :] == N - 1, g, np.roll(T, -1, axis=1))
            xm = np.where(gx[None, :] == 0, g, np.roll(T, 1, axis=1))
            yp = np.where(gy[:, None] == N - 1, g, np.roll(T, -1, axis=0))
            ym = np.where(gy[:, None] == 0, g, np.roll(T, 1, axis=0))
            r = t(self.p["r"])
            two = T + T
            return ((T + r * ((xp - two) + xm)) + r * ((yp - two) + ym))[None]
        t = self.dtype
        gam = t(self.p["gamma"])
        dt, dx = self.p["dt"], self.p["dx"]
        if lvl % 2 == 1:
            return numpy_ref.euler_stage(prev, prev, t(0.5 * dt / dx), t(0.5 * dt / dx), gam)
        return numpy_ref.euler_stage(prev2, prev, t(dt / dx), t(dt / dx), gam)

    def run(self, state0: np.ndarray) -> tuple[np.ndarray, Traffic]:
        g, W, N = self.g, self.W, self.g.N
        S = state0.reshape(self.nvar, N, N).astype(self.dtype)
        B = [S.copy(), np.full_like(S, np.nan)]
        tags = [np.zeros((N, N), dtype=np.int64), np.full((N, N), -1, dtype=np.int64)]
        traffic = Traffic()
        two_stage = self.kind == "euler"
        for phase in range(g.n_phases()):
            reads = {}   # (buf, y, x) -> instance id
            writes = {}
            pending = []
            nload = nstore = 0
            for (wx, wy) in g.shapes(phase):
                lo, hi = g.levels(wx, wy)
                if lo > hi:
                    continue
                for jx in range(g.tiles):
                    for jy in range(g.tiles):
                        inst = (wx, wy, jx, jy)
                        ox = g.centre(wx, jx) - g.b // 2 - g.n
                        oy = g.centre(wy, jy) - g.b // 2 - g.n
                        gx = (ox + np.arange(W)) % N
                        gy = (oy + np.arange(W)) % N
                        lds = [np.full((self.nvar, W, W), np.nan, dtype=self.dtype) for _ in range(2)]
                        ltag = [np.full((W, W), -1, dtype=np.int64) for _ in range(2)]
                        my_writes = {}

                        def rect_mask(f, grow=0):
                            m = np.zeros((W, W), dtype=bool)
                            if f is None:
                                return m
                            x0, x1 = f[0] - ox - grow, f[1] - ox + grow
                            y0, y1 = f[2] - oy - grow, f[3] - oy + grow
                            assert 0 <= x0 and x1 <= W and 0 <= y0 and y1 <= W, "window overflow"
                            m[y0:y1, x0:x1] = True
                            return m

                        def load(mask, lvl, dst):
                            nonlocal nload
                            buf = lvl % 2
                            ys, xs = np.nonzero(mask)
                            for y, x in zip(ys, xs):
                                key = (buf, int(gy[y]), int(gx[x]))
                                if key in my_writes and my_writes[key] != lvl:
                                    raise ProtocolError(f"{inst} reads back its own write {key}")
                                reads.setdefault(key, set()).add(inst)
                                ok = tags[buf][gy[y], gx[x]] == lvl
                                lds[dst][:, y, x] = B[buf][:, gy[y], gx[x]] if ok else np.nan
                                ltag[dst][y, x] = lvl if ok else -2
                            nload += len(ys)

                        def level_loads(lvl):
                            F = g.footprint(wx, wy, jx, jy, lvl)
                            prevmask = rect_mask(g.footprint(wx, wy, jx, jy, lvl - 1)) if lvl > lo else \
                                np.zeros((W, W), bool)
                            out = [(rect_mask(F, g.n) & ~prevmask, lvl - 1)]
                            if two_stage and lvl % 2 == 0 and lvl == lo:
                                out.append((rect_mask(F), lvl - 2))
                            return out

                        if self.preload:
                            # every level's loads first; within one LDS parity buffer they must not overlap
                            placed = [np.zeros((W, W), bool), np.zeros((W, W), bool)]
                            for lvl in range(lo, hi + 1):
                                for mask, src in level_loads(lvl):
                                    if np.any(placed[src % 2] & mask):
                                        raise ProtocolError(f"{inst}: preloaded rings overlap in LDS buffer {src % 2}")
                                    placed[src % 2] |= mask
                                    load(mask, src, src % 2)
                            self.preloaded = placed
                        for lvl in range(lo, hi + 1):
                            F = g.footprint(wx, wy, jx, jy, lvl)
                            if F is None:
                                continue
                            fmask = rect_mask(F)
                            if not self.preload:
                                for mask, src in level_loads(lvl):
                                    load(mask, src, src % 2)
                            # dependency check: the cross stencil at lvl-1 and (two-stage, even) own cell at lvl-2
                            ys, xs = np.nonzero(fmask)
                            cur = ltag[(lvl - 1) % 2]
                            for d in range(1, g.n + 1):
                                for (dy, dx) in ((0, d), (0, -d), (d, 0), (-d, 0)):
                                    if np.any(cur[ys + dy, xs + dx] != lvl - 1):
                                        raise ProtocolError(f"{inst} level {lvl}: neighbour not at level {lvl-1}")
                            if np.any(cur[ys, xs] != lvl - 1):
                                raise ProtocolError(f"{inst} level {lvl}: centre not at level {lvl-1}")
                            if two_stage and lvl % 2 == 0 and np.any(ltag[lvl % 2][ys, xs] != lvl - 2):
                                raise ProtocolError(f"{inst} level {lvl}: own cell not at level {lvl-2}")
                            new = self._compute(lds[(lvl - 1) % 2], lds[lvl % 2], lvl, gx, gy)
                            dst = lds[lvl % 2]
                            dst[:, fmask] = new[:, fmask]
                            ltag[lvl % 2][fmask] = lvl
                            lag = self.store_lag
                            f2 = g.footprint(wx, wy, jx, jy, lvl + lag) if lvl + lag <= hi else None
                            smask = fmask & ~rect_mask(f2)
                            ys, xs = np.nonzero(smask)
                            for y, x in zip(ys, xs):
                                key = (lvl % 2, int(gy[y]), int(gx[x]))
                                if key in my_writes:
                                    raise ProtocolError(f"{inst} writes {key} twice")
                                my_writes[key] = lvl
                                pending.append((key, dst[:, y, x].copy(), lvl))
                            nstore += len(ys)
                        for key in my_writes:
                            if key in writes:
                                raise ProtocolError(f"phase {phase}: {inst} and {writes[key]} both write {key}")
                            writes[key] = inst
            for key, insts in reads.items():
                if key in writes and (len(insts) > 1 or writes[key] not in insts):
                    raise ProtocolError(f"phase {phase}: {key} read by {insts} while written by {writes[key]}")
            for (buf, y, x), val, lvl in pending:
                B[buf][:, y, x] = val
                tags[buf][y, x] = lvl
            traffic.loads += nload
            traffic.stores += nstore
            traffic.per_phase.append((nload, nstore))
        fb = g.L % 2
        if not np.all(tags[fb] == g.L):
            raise ProtocolError("final level not complete")
        out = B[fb]
        return (out[0] if self.nvar == 1 else out), traffic
