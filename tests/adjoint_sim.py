"""CPU simulation of the swept heat adjoint (test infrastructure).

Forward: the run is cut into cycles of h steps (h = b/(2n)); the flat state
at each cycle start is a checkpoint.  Backward, per cycle, from the last:

  F0  forward Up-Pyramid of the cycle from the checkpoint, strips -> buffers P;
  F1  forward Bridges, reading P and the checkpoint, strips -> buffers Q;
  R0, R1, R2  the adjoint lambda^j = A^T lambda^{j+1} = A lambda^{j+1} (A is
      symmetric) is itself a swept advance of h levels in reversed time
      k = h - j, from the flat lambda^{(c+1)h}, on the other tiling (shift 1).
      Its k-time Up-Pyramid, Bridges and Down-Pyramid cover exactly the
      footprints of the forward Octahedron 1 (cut at h), Bridges (X <-> Y) and
      Up-Pyramid plus level 0, so each reverse instance recomputes the forward
      T of its own footprint in local memory -- R0 from P, Q and the
      checkpoint (source chosen by the owner of each input cell), R1 from P and
      the checkpoint, R2 from the checkpoint -- and pairs every computed
      lambda^j(x) with T^j(x):  dJ/dr = sum_j <L lambda^{j+1}, T^j>.

Every buffer access is level-tagged and checked, like swept_sim.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import numpy_ref
from swept_sim import Geom, ProtocolError


def _mask(W, ox, oy, f, grow=0):
    m = np.zeros((W, W), bool)
    if f is None:
        return m
    m[f[2] - oy - grow:f[3] - oy + grow, f[0] - ox - grow:f[1] - ox + grow] = True
    return m


class Buffers:
    """Named level-parity buffer pairs with level tags."""

    def __init__(self, N):
        self.N = N
        self.v = {}
        self.t = {}

    def pair(self, name, init=None, lvl=-1):
        for p in (0, 1):
            self.v[(name, p)] = np.full((self.N, self.N), np.nan)
            self.t[(name, p)] = np.full((self.N, self.N), -1, dtype=np.int64)
        if init is not None:
            self.v[(name, lvl % 2)][:] = init
            self.t[(name, lvl % 2)][:] = lvl

    def read(self, name, lvl, ys, xs):
        key = (name, lvl % 2)
        ok = self.t[key][ys, xs] == lvl
        return np.where(ok, self.v[key][ys, xs], np.nan), ok

    def write(self, name, lvl, ys, xs, vals):
        key = (name, lvl % 2)
        self.v[key][ys, xs] = vals
        self.t[key][ys, xs] = lvl


def forward_phase(g: Geom, phase, r, bufs: Buffers, src_of, dst, level0):
    """One forward phase of a flat-to-flat cycle (levels 1..g.L).  src_of(lvl, inst, ax, ay, owner_axes) names
    the buffer a ring value comes from; level 0 comes from the array level0; stores go to pair dst."""
    W = g.b + 2 * g.n
    pending = []
    for (wx, wy) in g.shapes(phase):
        lo, hi = g.levels(wx, wy)
        for jx in range(g.tiles):
            for jy in range(g.tiles):
                T, _ = local_forward(g, (wx, wy, jx, jy), r, bufs, src_of, level0)
                ox = g.centre(wx, jx) - g.b // 2 - g.n
                oy = g.centre(wy, jy) - g.b // 2 - g.n
                for lvl in range(lo, hi + 1):
                    f = g.footprint(wx, wy, jx, jy, lvl)
                    f2 = g.footprint(wx, wy, jx, jy, lvl + 2) if lvl + 2 <= hi else None
                    sm = _mask(W, ox, oy, f) & ~_mask(W, ox, oy, f2)
                    ys, xs = np.nonzero(sm)
                    pending.append((dst, lvl, (oy + ys) % g.N, (ox + xs) % g.N, T[lvl][ys, xs]))
    for name, lvl, gy, gx, vals in pending:
        bufs.write(name, lvl, gy, gx, vals)


def local_forward(g: Geom, inst, r, bufs: Buffers, src_of, level0):
    """Recompute the forward T levels of one instance in a local window; returns {lvl: window array}."""
    wx, wy, jx, jy = inst
    W = g.b + 2 * g.n
    N = g.N
    lo, hi = g.levels(wx, wy)
    ox = g.centre(wx, jx) - g.b // 2 - g.n
    oy = g.centre(wy, jy) - g.b // 2 - g.n
    gxs = (ox + np.arange(W)) % N
    gys = (oy + np.arange(W)) % N
    C = g.b // 2 + g.n
    cur = {}
    T = {}
    for lvl in range(lo, hi + 1):
        f = g.footprint(wx, wy, jx, jy, lvl)
        prevf = g.footprint(wx, wy, jx, jy, lvl - 1) if lvl > lo else None
        ring = _mask(W, ox, oy, f, g.n) & ~_mask(W, ox, oy, prevf)
        prev = np.full((W, W), np.nan) if lvl == lo else T[lvl - 1].copy()
        ys, xs = np.nonzero(ring)
        if lvl - 1 == 0:
            prev[ys, xs] = level0[gys[ys], gxs[xs]]
        else:
            ax = np.where(xs >= C, xs - C, C - 1 - xs)
            ay = np.where(ys >= C, ys - C, C - 1 - ys)
            names = src_of(lvl - 1, inst, ax, ay)
            for name in set(names):
                sel = names == name
                v, ok = bufs.read(name, lvl - 1, gys[ys[sel]], gxs[xs[sel]])
                prev[ys[sel], xs[sel]] = v
        fm = _mask(W, ox, oy, f)
        step = numpy_ref.heat_step(prev, r)
        T[lvl] = np.where(fm, step, np.nan)  # only F(lvl) holds level lvl; the next ring comes from buffers
        cur[lvl] = fm
    return T, cur


class AdjointSim:
    def __init__(self, N, b, r):
        self.N, self.b, self.r = N, b, r
        self.h = b // 2

    def run(self, T0, g_final, M):
        N, b, r, h = self.N, self.b, self.r, self.h
        assert M % h == 0
        C = M // h
        ckpt = [np.array(T0, dtype=np.float64)]
        for c in range(C):
            ckpt.append(numpy_ref.heat_run(ckpt[-1], r, h))
        lam = np.array(g_final, dtype=np.float64)
        dJdr = 0.0
        gf = Geom(N, b, 1, h)          # forward cycle geometry
        gk = Geom(N, b, 1, h, shift=1)  # reverse (k-time) geometry on the other tiling
        W = b + 2
        Cc = b // 2 + 1
        for c in range(C - 1, -1, -1):
            T0c = ckpt[c]
            bufs = Buffers(N)
            bufs.pair("P")
            bufs.pair("Q")
            forward_phase(gf, 0, r, bufs, lambda lvl, inst, ax, ay: np.array(["P"] * len(ax)), "P", T0c)
            forward_phase(gf, 1, r, bufs, lambda lvl, inst, ax, ay: np.array(["P"] * len(ax)), "Q", T0c)

            def src_oct1(lvl, inst, ax, ay):
                hw = gf.half_width(1, lvl)  # diamond 1 of the cycle at that level, centred on this instance
                own = (ax < hw).astype(int) + (ay < hw).astype(int)
                if np.any(own == 2):
                    raise ProtocolError("ring cell inside the Octahedron's own footprint")
                return np.where(own == 0, "P", "Q")

            src = {0: src_oct1, 1: lambda lvl, inst, ax, ay: np.array(["P"] * len(ax)),
                   2: lambda lvl, inst, ax, ay: np.array(["P"] * len(ax))}
            # lambda sweep in k-time: buffers L, level-tagged by k
            bufs.pair("L", init=lam, lvl=0)
            pending_all = []
            for kphase in range(3):
                pending = []
                for (kx, ky) in gk.shapes(kphase):
                    klo, khi = gk.levels(kx, ky)
                    fwd = (1 - kx, 1 - ky)  # forward shape with the same footprints
                    for jx in range(gk.tiles):
                        for jy in range(gk.tiles):
                            Tloc, fms = local_forward(gf, (fwd[0], fwd[1], jx, jy), r, bufs, src[kphase], T0c)
                            ox = gk.centre(kx, jx) - b // 2 - 1
                            oy = gk.centre(ky, jy) - b // 2 - 1
                            assert ox == gf.centre(fwd[0], jx) - b // 2 - 1 and oy == gf.centre(fwd[1], jy) - b // 2 - 1
                            gxs = (ox + np.arange(W)) % N
                            gys = (oy + np.arange(W)) % N
                            L = {}
                            for k in range(klo, khi + 1):
                                f = gk.footprint(kx, ky, jx, jy, k)
                                prevf = gk.footprint(kx, ky, jx, jy, k - 1) if k > klo else None
                                ring = _mask(W, ox, oy, f, 1) & ~_mask(W, ox, oy, prevf)
                                prev = np.full((W, W), np.nan) if k == klo else L[k - 1].copy()
                                ys, xs = np.nonzero(ring)
                                v, ok = bufs.read("L", k - 1, gys[ys], gxs[xs])
                                prev[ys, xs] = v
                                fm = _mask(W, ox, oy, f)
                                lap = numpy_ref.laplacian(prev)
                                new = numpy_ref.heat_step(prev, r)
                                j = h - k
                                if j == 0:
                                    Tj = T0c[np.ix_(gys, gxs)]
                                else:
                                    if not np.array_equal(fms[j], fm):
                                        raise ProtocolError("reverse footprint != forward footprint")
                                    Tj = Tloc[j]
                                if np.any(np.isnan(Tj[fm])) or np.any(np.isnan(new[fm])):
                                    raise ProtocolError(f"missing value at k={k} shape {(kx, ky)}")
                                dJdr_part = float(np.sum(lap[fm] * Tj[fm]))
                                pending.append(("acc", dJdr_part))
                                L[k] = np.where(fm, new, np.nan)
                                f2 = gk.footprint(kx, ky, jx, jy, k + 2) if k + 2 <= khi else None
                                sm = fm & ~_mask(W, ox, oy, f2)
                                sy, sx = np.nonzero(sm)
                                pending.append(("L", k, gys[sy], gxs[sx], L[k][sy, sx]))
                for item in pending:
                    if item[0] == "acc":
                        dJdr += item[1]
                    else:
                        bufs.write(item[0], item[1], item[2], item[3], item[4])
            key = ("L", h % 2)
            if not np.all(bufs.t[key] == h):
                raise ProtocolError("lambda^0 of the cycle incomplete")
            lam = bufs.v[key].copy()
        return lam, dJdr
