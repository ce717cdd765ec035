// host_swept.h -- one swept shape instance on a host core: the CPU's share of
// a heterogeneous advance (Sec. 3.2, Eq. 2).  It follows the GPU phase
// kernel (device_common.h, phase_instance) step for step -- the same rings
// loaded up front from the level-parity buffers, the same footprints from
// the level table, the same per-cell arithmetic (scheme.h) in the same order,
// the same store rule (each cell's top two levels) -- on a window held in a
// per-thread host array, so that a cell computed here is bit-identical to the
// one the GPU computes.  Periodic problems only.
#pragma once

#include <stdint.h>

#include <vector>

#include "device_common.h"

namespace swept {

// What every host instance of one advance shares.
struct HostPlan {
    int N, b, h, L, tiles;
    const LevelEntry* tab;  // host copy of the level table
    double p[5];            // scheme constants, as in PhaseArgs
};

// Records which cells of the exchange band a host instance wrote in this
// phase: mark[parity][band row][x] is set for every store into a row whose
// band index (row_band[y]) is non-negative.
struct WriteLog {
    uint8_t* mark;         // 2 x band_rows x N bytes
    const int* row_band;   // N entries: band index of a global row, or -1
    int N;
    size_t plane;          // band_rows * N
    inline void note(int parity, int gy, int gx) const
    {
        const int r = row_band[gy];
        if (r >= 0) mark[parity * plane + (size_t)r * N + gx] = 1;
    }
};

// Shape instance (wx, wy) at tile (jx, jy) on the host level-parity buffers
// H[0], H[1] (nvar planes of N*N each).  win is the thread's window scratch.
template <typename T>
void host_heat_instance(const HostPlan& P, int wx, int wy, int jx, int jy, T* const H[2], std::vector<T>& win,
                        const WriteLog& log)
{
    const int b = P.b, h = P.h, N = P.N;
    const int wmax = wx > wy ? wx : wy, wmin = wx < wy ? wx : wy;
    const int lo = (wmax - 1) * h + 1 > 1 ? (wmax - 1) * h + 1 : 1;
    const int hi = P.L < (wmin + 1) * h - 1 ? P.L : (wmin + 1) * h - 1;
    if (lo > hi) return;
    const int W = b + 2, C = b / 2 + 1;
    const int ox = jx * b + ((wx & 1) ? 0 : b / 2) - C, oy = jy * b + ((wy & 1) ? 0 : b / 2) - C;
    win.resize((size_t)2 * W * W);
    T* buf[2] = {win.data(), win.data() + (size_t)W * W};
    for (int ly = 0; ly < W; ++ly)
        for (int lx = 0; lx < W; ++lx) {
            const int pm = ring_parities<1, 0>(wx, wy, lo, hi, h, b, C, lx, ly);
            const size_t gi = (size_t)wrapi(oy + ly, N) * N + wrapi(ox + lx, N);
            if (pm & 1) buf[0][ly * W + lx] = H[0][gi];
            if (pm & 2) buf[1][ly * W + lx] = H[1][gi];
        }
    const LevelEntry* tab = wx == wy ? P.tab : P.tab + (wx > wy ? 2 * h : 3 * h);
    const int kbase = wx == wy ? (wx == 0 ? -h : (wx - 1) * h) : (wmax - 1) * h;
    const T r = (T)P.p[0];
    for (int lvl = lo; lvl <= hi; ++lvl) {
        const LevelEntry& e = tab[lvl - kbase];
        const bool has2 = lvl + 2 <= hi;
        const int hx2 = has2 ? e.hx2 : 0, hy2 = has2 ? e.hy2 : 0;
        const T* prev = buf[(lvl - 1) & 1];
        T* cur = buf[lvl & 1];
        T* out = H[lvl & 1];
        for (int y = e.y0; y < e.y0 + e.fh; ++y) {
            const int gy = wrapi(oy + y, N);
            const bool yk = (y - C >= -hy2) && (y - C < hy2);
            for (int x = e.x0; x < e.x0 + e.fw; ++x) {
                const int li = y * W + x;
                const T v = heat_update<T>(prev[li], prev[li + 1], prev[li - 1], prev[li + W], prev[li - W], r);
                cur[li] = v;
                if (!(yk && (x - C >= -hx2) && (x - C < hx2))) {
                    const int gx = wrapi(ox + x, N);
                    out[(size_t)gy * N + gx] = v;
                    log.note(lvl & 1, gy, gx);
                }
            }
        }
    }
}

// Euler instance (scheme bits V): state planes 4 x W x W per level parity and
// the pressure plane of each parity; level l = (base - cx dF) - cy dG with the
// faces of App. B, as in euler_level.
template <typename T, int V>
void host_euler_instance(const HostPlan& P, int wx, int wy, int jx, int jy, T* const H[2], std::vector<T>& win,
                         const WriteLog& log)
{
    const int b = P.b, h = P.h, N = P.N;
    const size_t NN = (size_t)N * N;
    const int wmax = wx > wy ? wx : wy, wmin = wx < wy ? wx : wy;
    const int lo = (wmax - 1) * h + 1 > 1 ? (wmax - 1) * h + 1 : 1;
    const int hi = P.L < (wmin + 1) * h - 1 ? P.L : (wmin + 1) * h - 1;
    if (lo > hi) return;
    const int W = b + 4, C = b / 2 + 2, WW = W * W;
    const int ox = jx * b + ((wx & 1) ? 0 : b / 2) - C, oy = jy * b + ((wy & 1) ? 0 : b / 2) - C;
    win.resize((size_t)10 * WW + 8 * (size_t)(b + 1));
    T* st[2] = {win.data(), win.data() + 4 * (size_t)WW};  // 4 planes each
    T* pr[2] = {win.data() + 8 * (size_t)WW, win.data() + 9 * (size_t)WW};
    T* faces = win.data() + 10 * (size_t)WW;  // 4 x (b + 1) fluxes of one row or column
    const T gamma = (T)P.p[0], gm1 = gamma - T(1);
    for (int ly = 0; ly < W; ++ly)
        for (int lx = 0; lx < W; ++lx) {
            const int pm = ring_parities<2, 1>(wx, wy, lo, hi, h, b, C, lx, ly);
            const size_t gi = (size_t)wrapi(oy + ly, N) * N + wrapi(ox + lx, N);
            for (int p = 0; p < 2; ++p)
                if (pm & (1 << p)) {
                    T q[4];
                    for (int c = 0; c < 4; ++c) q[c] = st[p][c * WW + ly * W + lx] = H[p][c * NN + gi];
                    pr[p][ly * W + lx] = pressure(q, gm1);
                }
        }
    const LevelEntry* tab = wx == wy ? P.tab : P.tab + (wx > wy ? 2 * h : 3 * h);
    const int kbase = wx == wy ? (wx == 0 ? -h : (wx - 1) * h) : (wmax - 1) * h;
    for (int lvl = lo; lvl <= hi; ++lvl) {
        const LevelEntry& e = tab[lvl - kbase];
        const bool has2 = lvl + 2 <= hi;
        const int hx2 = has2 ? e.hx2 : 0, hy2 = has2 ? e.hy2 : 0;
        const T* prev = st[(lvl - 1) & 1];
        T* cur = st[lvl & 1];
        const T* pp = pr[(lvl - 1) & 1];
        T* pc = pr[lvl & 1];
        T* out = H[lvl & 1];
        const bool second = (lvl & 1) == 0;
        const T cx = (T)(second ? P.p[3] : P.p[1]), cy = (T)(second ? P.p[4] : P.p[2]);
        const int x0 = e.x0, y0 = e.y0, fw = e.fw, fh = e.fh;
        for (int y = y0; y < y0 + fh; ++y) {  // x faces and the x update, row by row
            for (int k = 0; k <= fw; ++k) {
                const int a = y * W + x0 - 1 + k;  // face between cells a and a+1
                T qa[4], qb[4], qc[4], qd[4], f[4];
                for (int c = 0; c < 4; ++c) {
                    qa[c] = prev[c * WW + a - 1];
                    qb[c] = prev[c * WW + a];
                    qc[c] = prev[c * WW + a + 1];
                    qd[c] = prev[c * WW + a + 2];
                }
                face_flux<T, 1, V>(qa, qb, qc, qd, pp[a - 1], pp[a], pp[a + 1], pp[a + 2], gamma, f);
                for (int c = 0; c < 4; ++c) faces[c * (b + 1) + k] = f[c];
            }
            for (int k = 0; k < fw; ++k) {
                const int li = y * W + x0 + k;
                for (int c = 0; c < 4; ++c) {
                    const T base = second ? cur[c * WW + li] : prev[c * WW + li];
                    const T dF = faces[c * (b + 1) + k + 1] - faces[c * (b + 1) + k];
                    cur[c * WW + li] = base - cx * dF;
                }
            }
        }
        for (int x = x0; x < x0 + fw; ++x) {  // y faces, the y update and the store, column by column
            for (int k = 0; k <= fh; ++k) {
                const int a = (y0 - 1 + k) * W + x;  // face between cells a and a+W
                T qa[4], qb[4], qc[4], qd[4], g[4];
                for (int c = 0; c < 4; ++c) {
                    qa[c] = prev[c * WW + a - W];
                    qb[c] = prev[c * WW + a];
                    qc[c] = prev[c * WW + a + W];
                    qd[c] = prev[c * WW + a + 2 * W];
                }
                face_flux<T, 2, V>(qa, qb, qc, qd, pp[a - W], pp[a], pp[a + W], pp[a + 2 * W], gamma, g);
                for (int c = 0; c < 4; ++c) faces[c * (b + 1) + k] = g[c];
            }
            const bool xk = (x - C >= -hx2) && (x - C < hx2);
            const int gx = wrapi(ox + x, N);
            for (int k = 0; k < fh; ++k) {
                const int y = y0 + k, li = y * W + x;
                T q[4];
                for (int c = 0; c < 4; ++c) {
                    const T dG = faces[c * (b + 1) + k + 1] - faces[c * (b + 1) + k];
                    q[c] = cur[c * WW + li] - cy * dG;
                    cur[c * WW + li] = q[c];
                }
                pc[li] = pressure(q, gm1);
                if (!(xk && (y - C >= -hy2) && (y - C < hy2))) {
                    const int gy = wrapi(oy + y, N);
                    for (int c = 0; c < 4; ++c) out[c * NN + (size_t)gy * N + gx] = q[c];
                    log.note(lvl & 1, gy, gx);
                }
            }
        }
    }
}

}  // namespace swept
