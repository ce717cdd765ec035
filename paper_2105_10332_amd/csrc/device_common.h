// device_common.h -- device helpers shared by the swept phase kernels and
// the adjoint kernels: exact small quotients, periodic wrap, the 1D diamond
// geometry, the up-front ring load, and the per-level heat and Euler updates
// of a window in LDS.  Memory protocol: see kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"
#include "scheme.h"

namespace swept {

// Exact quotient i / d from a float reciprocal inv = 1.0f/d: the rounding
// error of (i + 0.5) * inv stays below the 0.5/d distance of (i + 0.5)/d to
// an integer.  Checked exhaustively for 0 <= i < 2^21, 1 <= d <= 160 (the
// kernels use i < 2^15 and d < 150: window cells, thread indices, widths).
__device__ __forceinline__ int qdiv(int i, float inv) { return (int)(((float)i + 0.5f) * inv); }

__host__ __device__ __forceinline__ int wrapi(int g, int N)
{
    g += (g < 0) ? N : 0;
    g -= (g >= N) ? N : 0;
    return g;
}

// Heat with boundary BC (0 periodic, 1 Dirichlet ghost value, 2 zero flux)
template <int BC>
struct HeatSV {
    static constexpr int NVAR = 1, R = 1, TWO_STAGE = 0, MAXWG = 1024, SCHEME = 0, BOUNDARY = BC;
};
using HeatS = HeatSV<0>;
// Euler with scheme variant V (limiter and spectral-radius bits, scheme.h);
// up to 1024 threads (the per-cell update fits in 64 VGPRs in either precision)
template <int V, int BC = 0>
struct EulerSV {
    static constexpr int NVAR = 4, R = 2, TWO_STAGE = 1, MAXWG = 1024, SCHEME = V, BOUNDARY = BC;
};
using EulerS = EulerSV<0>;

// Euler walls.  A face's run of four cells that reaches across the domain
// edge reads ghost cells from its own side of the edge instead of the
// wrapped cells: BC 2 (zero gradient) the edge cell, BC 3 (slip wall) the
// cell mirrored across the edge with its normal momentum negated.  E is the
// window-local index of the first cell past the edge (global index 0) along
// the face normal; `left` says the face belongs to the cells below E.
// Returns the window-local index to read for run cell m; flip = negate the
// normal momentum.  The returned index lies inside the run's own range.
template <int BC>
__device__ __forceinline__ int wall_cell(int m, int E, bool left, bool& flip)
{
    flip = false;
    if (left ? m < E : m >= E) return m;
    if constexpr (BC == 3) {
        flip = true;
        return 2 * E - 1 - m;
    }
    return left ? E - 1 : E;
}

// Window-local index of the domain's first column (row) in a window whose
// cell 0 is at global o and which holds W cells, or a sentinel far below 0
// when the window does not reach the edge.
__device__ __forceinline__ int window_edge(int o, int W, int N)
{
    return o < 0 ? -o : (o + W > N ? N - o : -(1 << 20));
}

// Numerical flux through the face after window-local cell a (A = 1: x, the
// run a-1 .. a+2 along a row starting at row offset `base`; A = 2: y, the run
// along a column, `base` the column) with the walls' ghost cells.
template <typename T, int A, int V, int BC>
__device__ __forceinline__ void wall_face(const T* __restrict__ prev, const T* __restrict__ pbuf, int W, int P,
                                          int base, int a, int E, bool left, T gamma, T out[4])
{
    T q[4][4], p[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        bool flip;
        const int m = wall_cell<BC>(a - 1 + o, E, left, flip);
        const int li = A == 1 ? base + m : m * W + base;
#pragma unroll
        for (int c = 0; c < 4; ++c) q[o][c] = prev[c * P + li];
        if (flip) q[o][A] = -q[o][A];
        p[o] = pbuf[li];
    }
    face_flux<T, A, V>(q[0], q[1], q[2], q[3], p[0], p[1], p[2], p[3], gamma, out);
}

__host__ __device__ __forceinline__ int half_width(int w, int lvl, int h, int n)
{
    const int t = lvl - (w - 1) * h;
    if (lvl < 1 || t < 1 || t > 2 * h - 1) return 0;
    return n * (t < 2 * h - t ? t : 2 * h - t);
}

// Which level-parity buffers the up-front load fills at local cell (lx, ly):
// bit p set <=> the cell lies in a ring(l) = Box(F(l), n) minus F(l-1) with
// (l-1)%2 == p.  With t = l - (w-1)h and a the cell's distance index from
// the centre along a growing axis (inside <=> a < hw), ring(t) holds
// (t-1)n <= a < (t+1)n, so the candidates t = a/n and a/n + 1 have opposite
// parities:
//   Octahedron w >= 1: a = max(ax, ay), t <= min(h, tmax);
//   Bridge: a along the growing axis, t <= min(h-1, tmax), and the shrinking
//     axis must satisfy s < (h-t+1)n;
//   Up-Pyramid (w = 0): only its first level, the tile at level 0;
// tmax = hi - (w-1)h (the cut at the final level).  A two-stage scheme whose
// first level is even also needs F(lo) at level lo-2 (buffer lo%2).
// Extra bits: RING_LEVEL0 -- the parity-0 value is level 0 (the initial
// state, which may live in its own buffer); RING_Q0/RING_Q1 (only when
// owner_q is set, for Octahedron 1 of a flat-to-flat cycle) -- the value
// was produced by a Bridge rather than the Up-Pyramid (the adjoint keeps
// the two in separate buffers): at level l-1 >= 1 a ring cell belongs to
// the Up-Pyramid iff it is outside diamond 1 on both axes.
constexpr int RING_LEVEL0 = 4, RING_Q0 = 8, RING_Q1 = 16;

template <int R, int TWO_STAGE>
__host__ __device__ __forceinline__ int ring_parities(int wx, int wy, int lo, int hi, int h, int b, int C, int lx, int ly,
                                             bool owner_q = false)
{
    const int ax = lx >= C ? lx - C : C - 1 - lx;
    const int ay = ly >= C ? ly - C : C - 1 - ly;
    const int wmax = wx > wy ? wx : wy;
    if (wmax == 0) return (ax < b / 2 && ay < b / 2) ? (1 | RING_LEVEL0) : 0;
    const int base = (wmax - 1) * h;
    const int tmax = hi - base;
    int a, s, tcap;
    if (wx == wy) {
        a = ax > ay ? ax : ay;
        s = -1;  // no shrinking axis
        tcap = h < tmax ? h : tmax;
    } else {
        a = wx > wy ? ax : ay;
        s = wx > wy ? ay : ax;
        tcap = (h - 1) < tmax ? (h - 1) : tmax;
    }
    const int t1 = a / R;
    int m = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int t = t1 + k;
        if (t >= 1 && t <= tcap && s < (h - t + 1) * R) {
            const int lev = base + t - 1;
            const int p = lev & 1;
            m |= 1 << p;
            if (lev == 0) m |= RING_LEVEL0;
            if (owner_q && lev > 0) {
                const int hw = half_width(wx, lev, h, R);
                if ((ax < hw) || (ay < hw)) m |= p ? RING_Q1 : RING_Q0;
            }
        }
    }
    if (TWO_STAGE && (lo & 1) == 0 && ax < half_width(wx, lo, h, R) && ay < half_width(wy, lo, h, R))
        m |= 1 << (lo & 1);
    return m;
}

// Sources of the up-front load: level-parity buffers g0/g1, the level-0
// state (normally g0 itself) and, for the adjoint, the Bridges' buffers.
// Kept as plain pointers (a struct of them ends up indexed in scratch).
template <typename T>
struct RingSrc {
    const T* g0;
    const T* g1;
    const T* lvl0;
    const T* q0;
    const T* q1;
    bool owner_q;
};

// Up-front load of every ring of the shape: a strided pass over the W x W
// window (LDS row pitch PITCH), KB cells per thread per batch with all their
// loads issued before any LDS write, so the batch costs one memory latency
// (two cells per batch for the FP64 Euler state, whose 2 x 4 values per cell
// would otherwise hold 64 registers).  WRAP = false when the window stays
// inside the domain (no periodic wrap of the global index).
//
// Euler (NVAR = 4) also writes the pressure of every loaded value into the
// pressure plane of its level parity (LDS after the two state buffers), so
// that no level recomputes the pressures of its ring.
template <class S, typename T, bool WRAP = true, int B = 0>
__device__ __forceinline__ void preload_rings(T* lds, int BUF, const RingSrc<T>& src, int W, int P, int PITCH, int N,
                                              size_t NN,
                                              int ox, int oy, int wx, int wy, int lo, int hi, int h, int C,
                                              int nthr, T gm1 = T(0))
{
    // heat with a compile-time tile B: enough cells per thread that a 512-thread workgroup loads
    // its whole window in one batch (measured: 2% faster in FP32 than four cells per thread, the
    // same in FP64)
    constexpr int NVAR = S::NVAR;
    constexpr int KB = NVAR == 4 ? ((NVAR * sizeof(T) >= 32) ? 2 : 4) : (B > 0 ? ((B + 2) * (B + 2) + 511) / 512 : 4);
    const T* __restrict__ g0 = src.g0;
    const T* __restrict__ g1 = src.g1;
    const T* __restrict__ z0 = src.lvl0;
    const T* __restrict__ q0 = src.q0;
    const T* __restrict__ q1 = src.q1;
    const bool owner_q = src.owner_q;
    const int cnt = W * W;
    const float invW = 1.0f / (float)W;
    for (int base = 0; base < cnt; base += KB * nthr) {
        T v[KB][2][NVAR];
        int li[KB], pm[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int i = base + k * nthr + (int)threadIdx.x;
            pm[k] = 0;
            li[k] = i;
            if (i < cnt) {
                const int ly = qdiv(i, invW), lx = i - ly * W;
                li[k] = ly * PITCH + lx;
                pm[k] = ring_parities<S::R, S::TWO_STAGE>(wx, wy, lo, hi, h, W - 2 * S::R, C, lx, ly, owner_q);
                if (pm[k] & 3) {
                    const size_t gi = WRAP ? (size_t)wrapi(oy + ly, N) * N + wrapi(ox + lx, N)
                                           : (size_t)(oy + ly) * N + (ox + lx);
                    if (pm[k] & 1) {
                        if (pm[k] & RING_LEVEL0) {
#pragma unroll
                            for (int c = 0; c < NVAR; ++c) v[k][0][c] = z0[c * NN + gi];
                        } else if (pm[k] & RING_Q0) {
#pragma unroll
                            for (int c = 0; c < NVAR; ++c) v[k][0][c] = q0[c * NN + gi];
                        } else {
#pragma unroll
                            for (int c = 0; c < NVAR; ++c) v[k][0][c] = g0[c * NN + gi];
                        }
                    }
                    if (pm[k] & 2) {
                        if (pm[k] & RING_Q1) {
#pragma unroll
                            for (int c = 0; c < NVAR; ++c) v[k][1][c] = q1[c * NN + gi];
                        } else {
#pragma unroll
                            for (int c = 0; c < NVAR; ++c) v[k][1][c] = g1[c * NN + gi];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                if (pm[k] & (1 << p)) {
#pragma unroll
                    for (int c = 0; c < NVAR; ++c) lds[p * BUF + c * P + li[k]] = v[k][p][c];
                    if constexpr (NVAR == 4) lds[2 * BUF + p * P + li[k]] = pressure(v[k][p], gm1);
                }
    }
}

// Value of the next lane (lane + 1) of the wavefront: a DPP wavefront shift
// (wave_shl:1, lane i reads lane i+1), one VALU move per 32 bits.  Lane 63
// gets 0; the face passes never use that lane's result.
__device__ __forceinline__ int next_lane_b32(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float next_lane(float v) { return __int_as_float(next_lane_b32(__float_as_int(v))); }
__device__ __forceinline__ double next_lane(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)next_lane_b32((int)(unsigned)b);
    const unsigned hi = (unsigned)next_lane_b32((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One Euler stage-level on the footprint [x0, x0+fw) x [y0, y0+fh) of the
// window (LDS row pitch PW, plane stride P): Q^l = base - cx dF - cy dG with
// base = Q^{l-1} (first RK stage) or Q^{l-2} held in cur (second stage),
// evaluated as (base - cx (F+ - F-)) - cy (G+ - G-) -- the oracle's order.
// pprev holds the pressures of the Q^{l-1} values in prev (every cell of the
// footprint grown by 2, the four-cell runs); PNEXT: pcur receives the
// pressure of each finished cell, for the next level.
//   X: face fluxes and the x update, row by row.  A row of fw cells has fw+1
//      faces; the items (row, face) are numbered row by row and each
//      wavefront takes 64 consecutive items starting 63 after the previous
//      one, so the face right of every updated cell is the next lane's face
//      (one shuffle per value) and the wave's last lane only computes the
//      face the lane before it needs.  No face buffer, no barrier between the
//      fluxes and the update.
//   Y: the same column by column, then the finished cell goes to cur (and its
//      pressure to pcur) and to the store policy.
// Lanes past the last item compute a copy of the last item's face so that
// every lane takes part in the shuffle; their results are dropped.
// BC != 0: walls (see wall_cell); ex, ey are the window-local indices of the
// domain's first column and row (window_edge).  A face at the edge itself
// exists once per side: the pass computes the lower side's flux, and the
// first cell past the edge recomputes its own.
template <typename T, int V, class Store, int BC = 0, bool PNEXT = true>
__device__ __forceinline__ void euler_level(const T* __restrict__ prev, T* cur, const T* __restrict__ pbuf,
                                            T* __restrict__ pcur, int PW, int P, int x0, int y0, int fw, int fh,
                                            bool second_stage, T gamma, T cx, T cy, const Store& store, int nthr,
                                            int ex = 0, int ey = 0)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, slots = nthr >> 6;
    const T gm1 = gamma - T(1);
    {  // X: faces between cells x0-1+k and x0+k of row y0+q (k = 0..fw), then the x update of cell x0+k
        const int nf = fw + 1, cnt = nf * fh;
        const float inv = 1.0f / (float)nf;
        for (int s = tid >> 6; 63 * s <= cnt - 2; s += slots) {
            const int i = 63 * s + lane;
            const int ic = i < cnt ? i : cnt - 1;
            const int q = qdiv(ic, inv);
            const int k = ic - q * nf;
            const int a = x0 - 1 + k;
            const int lb = (y0 + q) * PW + a;
            T f[4];
            if (BC != 0 && a - 1 < ex && a + 2 >= ex) {
                wall_face<T, 1, V, BC>(prev, pbuf, PW, P, (y0 + q) * PW, a, ex, a < ex, gamma, f);
            } else {
                T qa[4], qb[4], qc[4], qd[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    qa[c] = prev[c * P + lb - 1];
                    qb[c] = prev[c * P + lb];
                    qc[c] = prev[c * P + lb + 1];
                    qd[c] = prev[c * P + lb + 2];
                }
                face_flux<T, 1, V>(qa, qb, qc, qd, pbuf[lb - 1], pbuf[lb], pbuf[lb + 1], pbuf[lb + 2], gamma, f);
            }
            T fr[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) fr[c] = next_lane(f[c]);
            if (i < cnt && lane < 63 && k < fw) {
                const int li = lb + 1;  // cell x0+k: face f on its left, fr on its right
                if (BC != 0 && x0 + k == ex)  // the wall face as seen from this side
                    wall_face<T, 1, V, BC>(prev, pbuf, PW, P, (y0 + q) * PW, ex - 1, ex, false, gamma, f);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const T base = second_stage ? cur[c * P + li] : prev[c * P + li];
                    const T dF = fr[c] - f[c];
                    cur[c * P + li] = base - cx * dF;
                }
            }
        }
    }
    __syncthreads();
    {  // Y: faces between rows y0-1+k and y0+k of column x0+c (k = 0..fh), the y update of cell (x0+c, y0+k), the store
        const int nf = fh + 1, cnt = nf * fw;
        const float inv = 1.0f / (float)nf;
        for (int s = tid >> 6; 63 * s <= cnt - 2; s += slots) {
            const int i = 63 * s + lane;
            const int ic = i < cnt ? i : cnt - 1;
            const int col = qdiv(ic, inv);
            const int k = ic - col * nf;
            const int a = y0 - 1 + k;
            const int lx = x0 + col;
            const int lb = a * PW + lx;
            T g[4];
            if (BC != 0 && a - 1 < ey && a + 2 >= ey) {
                wall_face<T, 2, V, BC>(prev, pbuf, PW, P, lx, a, ey, a < ey, gamma, g);
            } else {
                T qa[4], qb[4], qc[4], qd[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    qa[c] = prev[c * P + lb - PW];
                    qb[c] = prev[c * P + lb];
                    qc[c] = prev[c * P + lb + PW];
                    qd[c] = prev[c * P + lb + 2 * PW];
                }
                face_flux<T, 2, V>(qa, qb, qc, qd, pbuf[lb - PW], pbuf[lb], pbuf[lb + PW], pbuf[lb + 2 * PW], gamma,
                                   g);
            }
            T gr[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) gr[c] = next_lane(g[c]);
            if (i < cnt && lane < 63 && k < fh) {
                const int ly = a + 1;
                const int li = lb + PW;
                if (BC != 0 && ly == ey)  // the wall face as seen from this side
                    wall_face<T, 2, V, BC>(prev, pbuf, PW, P, lx, ey - 1, ey, false, gamma, g);
                T out[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const T dG = gr[c] - g[c];
                    out[c] = cur[c * P + li] - cy * dG;
                    cur[c * P + li] = out[c];
                }
                if constexpr (PNEXT) pcur[li] = pressure(out, gm1);
                store(lx, ly, out);
            }
        }
    }
}

// Swept store policy: cells outside F(l+2) go to the level's global buffer.
// WRAP = false when the window stays inside the domain (no periodic wrap).
template <typename T, int NVAR, bool WRAP = true>
struct SweptStore {
    T* g;
    size_t NN;
    int N, ox, oy, C, hx2, hy2;
    __device__ __forceinline__ void operator()(int lx, int ly, const T* v) const
    {
        const int dx = lx - C, dy = ly - C;  // in F(l+2) <=> -hw2 <= d < hw2
        if ((dx >= -hx2) && (dx < hx2) && (dy >= -hy2) && (dy < hy2)) return;
        const size_t gi = WRAP ? (size_t)wrapi(oy + ly, N) * N + wrapi(ox + lx, N) : (size_t)(oy + ly) * N + (ox + lx);
#pragma unroll
        for (int c = 0; c < NVAR; ++c) g[c * NN + gi] = v[c];
    }
};

struct NoStore {
    template <typename V>
    __device__ __forceinline__ void operator()(int, int, const V*) const {}
};

// LDS layout of an Euler window of W x W cells with row pitch W + kEulerPad
// (the pad staggers the banks of the column-wise face pass): two
// level-parity state buffers of 4 planes, then the pressure planes of the two
// level parities.
constexpr int kEulerPad = 1;
__host__ __device__ inline size_t euler_lds_values(int W) { return (size_t)10 * W * (W + kEulerPad); }

// One heat level on the footprint [x0, x0+fw) x [y0, y0+fh) of the window.
// Each thread takes two adjacent columns and walks a vertical strip of R
// rows of them (R from the level table, so the footprint spreads over the
// whole workgroup), keeping the vertical neighbours in registers: per row
// two paired LDS reads (the next row of both columns; the outer left/right
// neighbours) and one paired LDS write for two cell-updates (W here is the
// LDS row pitch).  Cells outside F(l+2) (half-widths hx2, hy2) also go to
// the level's global buffer.  WRAP = false when the window does not cross
// the periodic boundary, so global indices need no wrap.
//
// BC != 0 (only with WRAP: a window that stays inside the square never
// reaches its edge) replaces every neighbour outside the square by a ghost
// value: the constant bcv (Dirichlet, BC = 1) or the edge cell itself (zero
// flux, BC = 2).  The window's wrapped copy of the far side is then unused.
template <typename T, bool WRAP, int BC = 0>
__device__ __forceinline__ void heat_level(const T* __restrict__ prev, T* __restrict__ cur, T* __restrict__ gout,
                                           int W, int C, const LevelEntry& e, int hx2, int hy2, int ox, int oy,
                                           int N, T r, int nthr, T bcv = T(0))
{
    static_assert(BC == 0 || WRAP, "boundaries are met only by windows that cross the edge");
    const int pw = e.pw;
    const int NN = N * N;
    const int ylo2 = C - hy2, yhi2 = C + hy2;  // rows inside F(l+2)
    for (int t = threadIdx.x; t < pw * e.spc; t += nthr) {
        const int sidx = qdiv(t, e.inv_pw);
        const int x = e.x0 + 2 * (t - sidx * pw);
        const int ys = e.y0 + sidx * e.R;
        const int ye = min(ys + e.R, e.y0 + e.fh);
        // the pair lies inside F(l+2) along x: both columns alike, since F(l+2) and the footprint
        // have half-widths of equal parity (they differ by 0 or 2n = 2), so pairs never straddle it
        const bool xk = (x - C >= -hx2) && (x - C < hx2);
        const int gx0 = WRAP ? wrapi(ox + x, N) : ox + x, gx1 = WRAP ? wrapi(ox + x + 1, N) : ox + x + 1;
        int gy = WRAP ? wrapi(oy + ys, N) : oy + ys;
        int grow = gy * N;
        int li = ys * W + x;
        T up0 = prev[li - W], up1 = prev[li - W + 1];
        T c0 = prev[li], c1 = prev[li + 1];
        for (int y = ys; y < ye; ++y) {
            const T dn0 = prev[li + W], dn1 = prev[li + W + 1];
            const T lft = prev[li - 1], rgt = prev[li + 2];
            T v0, v1;
            if constexpr (BC != 0) {
                // the pair straddles the x edge iff gx0 == N-1 (then gx1 == 0)
                const bool xl = gx0 == 0, xm = gx0 == N - 1, xr = gx1 == N - 1;
                const bool yt = gy == 0, yb = gy == N - 1;
                const T g0 = BC == 1 ? bcv : c0, g1 = BC == 1 ? bcv : c1;
                v0 = heat_update<T>(c0, xm ? g0 : c1, xl ? g0 : lft, yb ? g0 : dn0, yt ? g0 : up0, r);
                v1 = heat_update<T>(c1, xr ? g1 : rgt, xm ? g1 : c0, yb ? g1 : dn1, yt ? g1 : up1, r);
                gy = gy + 1 == N ? 0 : gy + 1;
            } else {
                v0 = heat_update<T>(c0, c1, lft, dn0, up0, r);
                v1 = heat_update<T>(c1, rgt, c0, dn1, up1, r);
            }
            cur[li] = v0;
            cur[li + 1] = v1;
            const bool yk = (y >= ylo2) && (y < yhi2);
            if (!(yk && xk)) {
                gout[grow + gx0] = v0;
                gout[grow + gx1] = v1;
            }
            up0 = c0;
            up1 = c1;
            c0 = dn0;
            c1 = dn1;
            li += W;
            grow += N;
            if (WRAP) grow = grow >= NN ? grow - NN : grow;
        }
    }
}

// heat_level for a window inside the domain, with cheaper strip set-up: the
// strip's position from 24-bit multiplies (full-rate; every operand is below
// 2^23), and its global stores addressed by 32-bit byte offsets from gw, the
// level buffer at the window's origin cell (ox, oy).  A window spans fewer than
// 256 rows of at most 2^16 cells, so every offset fits in 32 bits.  The test
// "inside F(l+2)" becomes one unsigned comparison per row.  STORE = false
// leaves the stores to heat_store_inner after the shape's last level.
template <typename T, bool STORE>
__device__ __forceinline__ void heat_level_inner(const T* __restrict__ prev, T* __restrict__ cur,
                                                 char* __restrict__ gw, int W, int C, const LevelEntry& e, int hx2,
                                                 int hy2, int N, T r, int nthr)
{
    const int pw = e.pw, R = e.R, items = pw * e.spc;
    const unsigned rowb = (unsigned)N * (unsigned)sizeof(T);
    const int yend = e.y0 + e.fh, ylo2 = C - hy2;
    const unsigned span2 = (unsigned)(2 * hy2);
    for (int t = threadIdx.x; t < items; t += nthr) {
        const int sidx = qdiv(t, e.inv_pw);
        const int x = e.x0 + 2 * (t - (int)__umul24(sidx, pw));
        const int ys = e.y0 + (int)__umul24(sidx, R);
        const int nr = min(R, yend - ys);  // at least 1: sidx < spc = ceil(fh / R)
        __builtin_assume(nr >= 1);
        // rows y with (y - (C - hy2)) < span (unsigned) lie inside F(l+2) and are not stored;
        // span = 0 when the pair is outside F(l+2) along x (see heat_level)
        const unsigned span = (unsigned)(x - C + hx2) < (unsigned)(2 * hx2) ? span2 : 0u;
        unsigned yrel = (unsigned)(ys - ylo2);
        int li = (int)__umul24(ys, W) + x;
        unsigned boff = ((unsigned)__umul24(ys, N) + (unsigned)x) * (unsigned)sizeof(T);
        T up0 = prev[li - W], up1 = prev[li - W + 1];
        T c0 = prev[li], c1 = prev[li + 1];
        int k = 0;
#pragma unroll 2
        do {
            const T dn0 = prev[li + W], dn1 = prev[li + W + 1];
            const T lft = prev[li - 1], rgt = prev[li + 2];
            const T v0 = heat_update<T>(c0, c1, lft, dn0, up0, r);
            const T v1 = heat_update<T>(c1, rgt, c0, dn1, up1, r);
            cur[li] = v0;
            cur[li + 1] = v1;
            if (STORE && yrel >= span) {
                T* gp = reinterpret_cast<T*>(gw + boff);
                gp[0] = v0;
                gp[1] = v1;
            }
            up0 = c0;
            up1 = c1;
            c0 = dn0;
            c1 = dn1;
            li += W;
            boff += rowb;
            ++yrel;
        } while (++k < nr);
    }
}

// The outputs of a heat shape inside the domain, written after its last
// level (FP32; see phase_instance).  The store rule keeps, for each level
// parity p, every cell of the union U_p of the footprints of the shape's
// levels of parity p, at the last such level that computed it: F(l) minus
// F(l+2) at each level l is exactly where a cell of U_p computes its last
// parity-p value, since a cell enters and leaves a shape's footprints once.
// That value is what LDS buffer p holds when the shape ends: later levels of
// parity p do not reach the cell, and the ring load came before every level.
// So the window's outputs go out in one pass over the footprints' bounding
// square [C-h, C+h)^2, row by row, each wavefront writing consecutive cells
// (a per-level store of an FP32 column pair writes 8 bytes of a row, and the
// memory system moves whole lines).  Membership of U_p (n = 1; t = l -
// (w-1)h the level within the shape, [t0, t1] the shape's range, q0 the
// level parity of t = 0):
//   Octahedron: max(ax, ay) < M_p, the largest half-width min(t, 2h - t) at
//     the levels of parity p;
//   Bridge (distance a along the growing axis, s along the shrinking one):
//     the footprint at t is a < t, s < h - t, so some t of parity p lies in
//     [max(a + 1, t0), min(h - s - 1, t1)].
template <typename T, int B, bool OCT>
__device__ __forceinline__ void heat_store_inner(const T* __restrict__ lds, int BUF, int PITCH, T* __restrict__ g0w,
                                                 T* __restrict__ g1w, int N, int C, int h, bool xgrows, int t0, int t1,
                                                 int q0, int M0, int M1, int nthr)
{
    const int b = B > 0 ? B : 2 * h;
    for (int i = threadIdx.x; i < b * b; i += nthr) {
        const int ry = i / b, rx = i - ry * b;  // B > 0: shifts
        const int lx = C - h + rx, ly = C - h + ry;
        const int ax = lx >= C ? lx - C : C - 1 - lx;
        const int ay = ly >= C ? ly - C : C - 1 - ly;
        bool m0, m1;
        if constexpr (OCT) {
            const int a = max(ax, ay);
            m0 = a < M0;
            m1 = a < M1;
        } else {
            const int a = xgrows ? ax : ay, s = xgrows ? ay : ax;
            const int lo = max(a + 1, t0), hi = min(h - s - 1, t1);
            // the level at t = lo has parity q0 ^ (lo & 1); two or more levels hold both parities
            const bool any = lo <= hi, two = lo < hi;
            const int plo = q0 ^ (lo & 1);
            m0 = any && (two || plo == 0);
            m1 = any && (two || plo == 1);
        }
        const int li = (int)__umul24(ly, PITCH) + lx;
        const unsigned gi = (unsigned)__umul24(ly, N) + (unsigned)lx;
        if (m0) g0w[gi] = lds[li];
        if (m1) g1w[gi] = lds[BUF + li];
    }
}

// Up-front ring load of a heat window inside the domain (n = 1; not the
// Up-Pyramid, and level 0 in buffer 0 when the window reaches it): the cells
// and parities of ring_parities, in the same strided order as preload_rings,
// with the strided cell index stepped in row/column form instead of divided
// and the global reads addressed by 32-bit byte offsets from the window
// origin in g0 and g1.  A cell at distance index a from the centre along the
// growing axis (the larger of the two in an Octahedron, OCT) holds the
// candidates t = a and t = a + 1, which lie at opposite level parities: the
// one at parity p is t_p = a + ((base + a + 1 + p) % 2), loaded when
// 1 <= t_p <= cap, cap = tcap (Octahedron) or min(tcap, h - s) (Bridge, s
// the distance index along the shrinking axis, and at least 0).  Cells past the
// window's last row have a >= h + 1 > cap (Octahedron, Y-Bridge) or cap = 0
// (X-Bridge), so they need no separate test.
template <typename T, int B, bool OCT>
__device__ __forceinline__ void preload_heat_inner(T* lds, int BUF, const T* g0, const T* g1, int W, int PITCH,
                                                   int N, int ox, int oy, bool xgrows, int base, int tcap, int h,
                                                   int C, int nthr)
{
    constexpr int KB = B > 0 ? ((B + 2) * (B + 2) + 511) / 512 : 4;
    const int tid = threadIdx.x;
    const char* s0 = reinterpret_cast<const char*>(g0 + ((size_t)oy * N + ox));
    const char* s1 = reinterpret_cast<const char*>(g1 + ((size_t)oy * N + ox));
    const int sdy = nthr / W, sdx = nthr - sdy * W;  // the stride nthr in rows and columns
    const int pb = (base + 1) & 1;
    int ly = qdiv(tid, 1.0f / (float)W);
    int lx = tid - ly * W;
    for (int i0 = 0; i0 < W * W; i0 += KB * nthr) {
        T v0[KB], v1[KB];
        int li[KB];
        bool n0[KB], n1[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int ax = lx >= C ? lx - C : C - 1 - lx;
            const int ay = ly >= C ? ly - C : C - 1 - ly;
            int a, cap;
            if constexpr (OCT) {
                a = max(ax, ay);
                cap = tcap;
            } else {
                a = xgrows ? ax : ay;
                cap = max(0, min(tcap, h - (xgrows ? ay : ax)));
            }
            const int pa = (a + pb) & 1;  // parity of t = a's level
            n0[k] = (unsigned)(a + pa - 1) < (unsigned)cap;
            n1[k] = (unsigned)(a - pa) < (unsigned)cap;
            li[k] = __mul24(ly, PITCH) + lx;
            const unsigned boff = (unsigned)(__mul24(ly, N) + lx) * (unsigned)sizeof(T);
            if (n0[k]) v0[k] = *reinterpret_cast<const T*>(s0 + boff);
            if (n1[k]) v1[k] = *reinterpret_cast<const T*>(s1 + boff);
            lx += sdx;
            ly += sdy;
            if (lx >= W) {
                lx -= W;
                ++ly;
            }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if (n0[k]) lds[li[k]] = v0[k];
            if (n1[k]) lds[BUF + li[k]] = v1[k];
        }
    }
}

// A level-table entry read through the constant address space (scalar loads),
// field by field.
typedef __attribute__((address_space(4))) LevelEntry ConstLevelEntry;
__device__ __forceinline__ LevelEntry load_entry(const ConstLevelEntry* p)
{
    LevelEntry e;
    e.x0 = p->x0;
    e.y0 = p->y0;
    e.fw = p->fw;
    e.fh = p->fh;
    e.hx2 = p->hx2;
    e.hy2 = p->hy2;
    e.pw = p->pw;
    e.R = p->R;
    e.spc = p->spc;
    e.inv_fw = p->inv_fw;
    e.inv_pw = p->inv_pw;
    return e;
}

// Largest workgroup of a phase kernel (its launch bound).
template <class S, typename T>
constexpr int max_wg()
{
    return S::MAXWG;
}

// One shape instance (workgroup index blk) of phase a.phase; the body of the
// phase kernel, also run by the batched persistent kernel.  B > 0 fixes the
// tile edge at compile time (a.tile must equal it), which turns the window
// pitch into an immediate in every LDS address; B = 0 takes a.tile.
template <class S, typename T, int B = 0, bool TAPED = false>
__device__ __forceinline__ void phase_instance(const PhaseArgs& a, int blk, unsigned char* smem_raw)
{
    // heat, and Euler with walls: windows that cross the domain edge first (heat -2.7% FP64,
    // -3.6% FP32 on the 4096^2 advance; walled Euler windows at the edge recompute a wall
    // face per row); periodic Euler keeps the row-major order (edge-first measured +1%)
    constexpr bool ORDER_EDGE_FIRST = S::NVAR == 1 || S::BOUNDARY != 0;
    T* lds = reinterpret_cast<T*>(smem_raw);
    constexpr int NVAR = S::NVAR, R = S::R;
    const int b = B > 0 ? B : a.tile, h = B > 0 ? B / (2 * R) : a.h, N = a.N, L = a.L;
    // heat pads its LDS rows by one value (fewer bank conflicts between the
    // rows a wave touches at once); Euler keeps the pitch W
    const int W = b + 2 * R, PITCH = W + (NVAR == 1 ? kHeatPad : kEulerPad), P = PITCH * W;
    const size_t NN = (size_t)N * N;
    const int tiles = a.tiles, t2 = tiles * tiles;

    // instance decode: phase 2w -> Octahedron (w, w); phase 2w-1 -> Bridges (w, w-1) then (w-1, w);
    // a heterogeneous advance launches only the tile rows jy < jrows (row-major order)
    const int per = a.jrows > 0 ? tiles * a.jrows : t2;
    int wx, wy, inst = blk;
    if ((a.phase & 1) == 0) {
        wx = wy = a.phase >> 1;
    } else {
        const int w = (a.phase + 1) >> 1;
        const int k = inst >= per;
        inst -= k * per;
        wx = k ? w - 1 : w;
        wy = k ? w : w - 1;
    }
    int jx, jy;
    if (a.jrows > 0) {
        jx = inst % tiles;
        jy = inst / tiles;
    } else if constexpr (ORDER_EDGE_FIRST) {
        // windows that cross the domain edge take the slower path (periodic
        // wrap or ghost values): give them the lowest workgroup indices so
        // they start first.  The wrapping row and column are jy = ey and
        // jx = ex (centres at 0 for odd w, at N - b/2 for even w); then that
        // column without its corner; then the rest.
        const int ex = (wx & 1) ? 0 : tiles - 1, ey = (wy & 1) ? 0 : tiles - 1, m = tiles - 1;
        if (inst < tiles) {
            jx = inst;
            jy = ey;
        } else if (inst < 2 * tiles - 1) {
            const int k = inst - tiles;
            jx = ex;
            jy = k < ey ? k : k + 1;
        } else {
            const int k = inst - (2 * tiles - 1), ix = k % m, iy = k / m;
            jx = ix < ex ? ix : ix + 1;
            jy = iy < ey ? iy : iy + 1;
        }
    } else {
        jx = inst % tiles;
        jy = inst / tiles;
    }
    const int wmax = wx > wy ? wx : wy, wmin = wx < wy ? wx : wy;
    const int lo = max(1, (wmax - 1) * h + 1);
    const int hi = min(L, (wmin + 1) * h - 1);
    if (lo > hi) return;

    const int C = b / 2 + R;  // window centre (local): footprints are [C-hw, C+hw)
    const int cx = jx * b + ((wx & 1) ? 0 : b / 2);
    const int cy = jy * b + ((wy & 1) ? 0 : b / 2);
    const int ox = cx - C, oy = cy - C;
    T* g0 = reinterpret_cast<T*>(a.out0);
    T* g1 = reinterpret_cast<T*>(a.out1);
    const int BUF = NVAR * P;  // LDS values per level-parity buffer (address arithmetic keeps ds_* access)

    // TAPED (the adjoint's taped cycle, first Octahedron): the Up-Pyramid's strips are in
    // buf0/buf1 and the Bridges' in q0/q1, and each ring cell comes from its owner's buffers
    const RingSrc<T> src{reinterpret_cast<const T*>(a.buf0), reinterpret_cast<const T*>(a.buf1),
                         reinterpret_cast<const T*>(a.lvl0), TAPED ? reinterpret_cast<const T*>(a.q0) : nullptr,
                         TAPED ? reinterpret_cast<const T*>(a.q1) : nullptr, TAPED};
    // global indices need the periodic wrap only when the window crosses the boundary
    const bool wraps = ox < 0 || oy < 0 || ox + W > N || oy + W > N;
    const T gm1 = (T)a.p[0] - T(1);  // Euler: gamma - 1 for the ring pressures (heat: unused)
    // the workgroup size, read once: a read inside a level would be a vector load whose wait
    // also waits for the level's global stores
    const int nthr = blockDim.x;
    // heat windows inside the domain past the Up-Pyramid take the lean load (level 0 must then be
    // buffer 0 itself whenever the window reaches it)
    bool lean = false;
    if constexpr (NVAR == 1 && !TAPED) lean = !wraps && wmax >= 1 && (wmax >= 2 || src.lvl0 == src.g0);
    // FP32 lean windows write their outputs after the last level (heat_store_inner): the same time
    // as per-level stores, half the HBM writes (measured at 4096^2); FP64 ones store level by level,
    // which measured 5% faster
    constexpr bool DEFER = NVAR == 1 && !TAPED && sizeof(T) == 4;
    if (lean) {
        const int base = (wmax - 1) * h;
        if (wx == wy)
            preload_heat_inner<T, B, true>(lds, BUF, src.g0, src.g1, W, PITCH, N, ox, oy, false, base,
                                           min(h, hi - base), h, C, nthr);
        else
            preload_heat_inner<T, B, false>(lds, BUF, src.g0, src.g1, W, PITCH, N, ox, oy, wx > wy, base,
                                            min(h - 1, hi - base), h, C, nthr);
    } else if (wraps)
        preload_rings<S, T, true, B>(lds, BUF, src, W, P, PITCH, N, NN, ox, oy, wx, wy, lo, hi, h, C, nthr, gm1);
    else
        preload_rings<S, T, false, B>(lds, BUF, src, W, P, PITCH, N, NN, ox, oy, wx, wy, lo, hi, h, C, nthr, gm1);
    __syncthreads();

    // level table of this shape type, indexed by the level within its window
    const LevelEntry* tab;
    int kbase;
    if (wx == wy) {
        tab = a.tab;
        kbase = wx == 0 ? -h : (wx - 1) * h;  // the Up-Pyramid is the Octahedron's upper half
    } else {
        tab = a.tab + (wx > wy ? 2 * h : 3 * h);
        kbase = (wmax - 1) * h;
    }
    // the level table is read through the constant address space: nothing writes it during a
    // launch, so every entry comes in with scalar loads, which a wait for the level's global
    // stores never holds up (a vector load would share their counter)
    const ConstLevelEntry* ctab = (const ConstLevelEntry*)(tab - kbase);
    for (int lvl = lo; lvl <= hi; ++lvl) {
        const LevelEntry e = load_entry(ctab + lvl);
        const bool has2 = lvl + 2 <= hi;
        const int hx2 = has2 ? e.hx2 : 0, hy2 = has2 ? e.hy2 : 0;
        const T* prev = lds + ((lvl - 1) & 1) * BUF;
        T* cur = lds + (lvl & 1) * BUF;
        T* gout = (lvl & 1) ? g1 : g0;
        if constexpr (NVAR == 1) {
            if (wraps)
                heat_level<T, true, S::BOUNDARY>(prev, cur, gout, PITCH, C, e, hx2, hy2, ox, oy, N, (T)a.p[0],
                                                 nthr, (T)a.p[1]);
            else if (!DEFER || !lean)  // stores level by level (inside the domain but not lean: level 0 is
                                       // not buffer 0)
                heat_level_inner<T, true>(prev, cur, reinterpret_cast<char*>(gout + ((size_t)oy * N + ox)), PITCH,
                                          C, e, hx2, hy2, N, (T)a.p[0], nthr);
            else
                heat_level_inner<T, false>(prev, cur, nullptr, PITCH, C, e, hx2, hy2, N, (T)a.p[0], nthr);
        } else {
            const T* pprev = lds + 2 * BUF + ((lvl - 1) & 1) * P;
            T* pcur = lds + 2 * BUF + (lvl & 1) * P;
            const bool second = (lvl & 1) == 0;
            const T g = (T)a.p[0], cxl = (T)(second ? a.p[3] : a.p[1]), cyl = (T)(second ? a.p[4] : a.p[2]);
            if (wraps) {
                const SweptStore<T, NVAR, true> st{gout, NN, N, ox, oy, C, hx2, hy2};
                if (S::BOUNDARY != 0)
                    euler_level<T, S::SCHEME, SweptStore<T, NVAR, true>, S::BOUNDARY>(
                        prev, cur, pprev, pcur, PITCH, P, e.x0, e.y0, e.fw, e.fh, second, g, cxl, cyl, st, nthr,
                        window_edge(ox, W, N), window_edge(oy, W, N));
                else
                    euler_level<T, S::SCHEME>(prev, cur, pprev, pcur, PITCH, P, e.x0, e.y0, e.fw, e.fh, second, g,
                                              cxl, cyl, st, nthr);
            } else {
                const SweptStore<T, NVAR, false> st{gout, NN, N, ox, oy, C, hx2, hy2};
                euler_level<T, S::SCHEME>(prev, cur, pprev, pcur, PITCH, P, e.x0, e.y0, e.fw, e.fh, second, g, cxl,
                                          cyl, st, nthr);
            }
        }
        __syncthreads();
    }
    if constexpr (DEFER) {
        if (lean) {
            T* g0w = g0 + ((size_t)oy * N + ox);
            T* g1w = g1 + ((size_t)oy * N + ox);
            const int wsh = (wmax - 1) * h, t0 = lo - wsh, t1 = hi - wsh;
            if (wx == wy) {
                int M[2] = {0, 0};
                for (int t = t0; t <= t1; ++t) M[(t + wsh) & 1] = max(M[(t + wsh) & 1], min(t, 2 * h - t));
                heat_store_inner<T, B, true>(lds, BUF, PITCH, g0w, g1w, N, C, h, false, t0, t1, 0, M[0], M[1], nthr);
            } else {
                heat_store_inner<T, B, false>(lds, BUF, PITCH, g0w, g1w, N, C, h, wx > wy, t0, t1, wsh & 1, 0, 0,
                                              nthr);
            }
        }
    }
}

}  // namespace swept
