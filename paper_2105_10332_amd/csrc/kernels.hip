// kernels.hip -- gfx950 kernels of the swept-rule solver.
//
// Swept phase kernel: one workgroup per space-time shape instance (Sec. 3.3,
// Figs. 1-2).  Shapes are products of 1D "diamonds": diamond w is centred at
// tile centres (w even) or tile edges (w odd), lives on levels
// (w-1)h+1 .. (w+1)h-1 and at level l covers [c-hw, c+hw) with
// hw = n*min(t, 2h-t), t = l-(w-1)h, h = b/(2n) (Eq. 1 gives k = h-1 levels
// before an exchange).  Phase 2w runs Octahedron (w, w) -- the Up-Pyramid for
// w = 0 and, cut at the final level, the Down-Pyramid -- and phase 2w-1 runs
// the two Bridges (w, w-1), (w-1, w) of window w in the same launch.
//
// Memory protocol (level l of a cell lives in global buffer l mod 2).  Level l
// of a shape needs ring(l) = Box(F(l), n) minus F(l-1) at level l-1 from
// outside (F = footprint rectangle of the level, Box = grown by n); every
// ring was written by earlier phases, and the rings of one level parity are
// disjoint, so a workgroup
//   1. loads all its rings up front, ring(l) from buffer (l-1)%2 into LDS
//      buffer (l-1)%2, in one pass over its (b+2n)^2 window -- one memory
//      latency per shape instead of one per level;
//   2. computes each level l of F(l) into LDS buffer l%2 (Euler's second
//      stage also reads the cell's own level l-2 value there, in place), one
//      barrier per level;
//   3. stores the cells of F(l) that are not in F(l+2) to buffer l%2: each
//      cell's top two levels, exactly the values later shapes read.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "scheme.h"

namespace swept {

// Exact quotient i / d for 0 <= i < 2^13 and 1 <= d <= 160 from a float
// reciprocal: the rounding error of (i + 0.5) * inv stays far below the
// 0.5/d distance of (i + 0.5)/d to an integer.
__device__ __forceinline__ int qdiv(int i, float inv) { return (int)(((float)i + 0.5f) * inv); }

__device__ __forceinline__ int wrapi(int g, int N)
{
    g += (g < 0) ? N : 0;
    g -= (g >= N) ? N : 0;
    return g;
}

struct HeatS {
    static constexpr int NVAR = 1, R = 1, TWO_STAGE = 0, MAXWG = 1024;
};
struct EulerS {  // register-heavy per-cell update: at most 256 threads so nothing spills
    static constexpr int NVAR = 4, R = 2, TWO_STAGE = 1, MAXWG = 256;
};

__device__ __forceinline__ int half_width(int w, int lvl, int h, int n)
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
template <int R, int TWO_STAGE>
__device__ __forceinline__ int ring_parities(int wx, int wy, int lo, int hi, int h, int b, int C, int lx, int ly)
{
    const int ax = lx >= C ? lx - C : C - 1 - lx;
    const int ay = ly >= C ? ly - C : C - 1 - ly;
    const int wmax = wx > wy ? wx : wy;
    if (wmax == 0) return (ax < b / 2 && ay < b / 2) ? 1 : 0;
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
        if (t >= 1 && t <= tcap && s < (h - t + 1) * R) m |= 1 << ((base + t - 1) & 1);
    }
    if (TWO_STAGE && (lo & 1) == 0 && ax < half_width(wx, lo, h, R) && ay < half_width(wy, lo, h, R))
        m |= 1 << (lo & 1);
    return m;
}

// Up-front load of every ring of the shape: a strided pass over the window,
// KB cells per thread per batch with all their loads issued before any LDS
// write, so the batch costs one memory latency.
template <class S, typename T>
__device__ __forceinline__ void preload_rings(T* lds, int BUF, const T* g0, const T* g1, int W, int P, int N,
                                              size_t NN, int ox, int oy, int wx, int wy, int lo, int hi, int h, int C)
{
    constexpr int NVAR = S::NVAR, KB = 4;
    const int cnt = W * W;
    const float invW = 1.0f / (float)W;
    for (int base = 0; base < cnt; base += KB * (int)blockDim.x) {
        T v[KB][2][NVAR];
        int li[KB], pm[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int i = base + k * (int)blockDim.x + (int)threadIdx.x;
            pm[k] = 0;
            li[k] = i;
            if (i < cnt) {
                const int ly = qdiv(i, invW), lx = i - ly * W;
                pm[k] = ring_parities<S::R, S::TWO_STAGE>(wx, wy, lo, hi, h, W - 2 * S::R, C, lx, ly);
                if (pm[k]) {
                    const size_t gi = (size_t)wrapi(oy + ly, N) * N + wrapi(ox + lx, N);
                    if (pm[k] & 1)
#pragma unroll
                        for (int c = 0; c < NVAR; ++c) v[k][0][c] = g0[c * NN + gi];
                    if (pm[k] & 2)
#pragma unroll
                        for (int c = 0; c < NVAR; ++c) v[k][1][c] = g1[c * NN + gi];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                if (pm[k] & (1 << p))
#pragma unroll
                    for (int c = 0; c < NVAR; ++c) lds[p * BUF + c * P + li[k]] = v[k][p][c];
    }
}

template <class S, typename T>
__device__ __forceinline__ void cell_update(const T* prev, const T* cur, int li, int W, int P, int lvl,
                                            const PhaseArgs& a, T out[S::NVAR]);

template <>
__device__ __forceinline__ void cell_update<HeatS, double>(const double* prev, const double*, int li, int W, int,
                                                           int, const PhaseArgs& a, double out[1])
{
    out[0] = heat_update<double>(prev[li], prev[li + 1], prev[li - 1], prev[li + W], prev[li - W], a.p[0]);
}
template <>
__device__ __forceinline__ void cell_update<HeatS, float>(const float* prev, const float*, int li, int W, int, int,
                                                          const PhaseArgs& a, float out[1])
{
    out[0] = heat_update<float>(prev[li], prev[li + 1], prev[li - 1], prev[li + W], prev[li - W], (float)a.p[0]);
}
template <typename T>
__device__ __forceinline__ void euler_update(const T* prev, const T* cur, int li, int W, int P, int lvl,
                                             const PhaseArgs& a, T out[4])
{
    const T gamma = (T)a.p[0];
    if (lvl & 1)  // Q* = Q^m - dt/2 ...: base and fluxes from level l-1
        euler_cell<T>(prev, P, W, li, prev, P, li, gamma, (T)a.p[1], (T)a.p[2], out);
    else  // Q^{m+1} = Q^m - dt ...(Q*): base is the cell's own level l-2 value in `cur`
        euler_cell<T>(prev, P, W, li, cur, P, li, gamma, (T)a.p[3], (T)a.p[4], out);
}
template <>
__device__ __forceinline__ void cell_update<EulerS, double>(const double* prev, const double* cur, int li, int W,
                                                            int P, int lvl, const PhaseArgs& a, double out[4])
{
    euler_update<double>(prev, cur, li, W, P, lvl, a, out);
}
template <>
__device__ __forceinline__ void cell_update<EulerS, float>(const float* prev, const float* cur, int li, int W, int P,
                                                           int lvl, const PhaseArgs& a, float out[4])
{
    euler_update<float>(prev, cur, li, W, P, lvl, a, out);
}

// One heat level on the footprint [C-hx, C+hx) x [C-hy, C+hy) of the window:
// each thread takes a vertical strip of R cells of one column (R chosen so
// the footprint spreads over the whole workgroup) and walks it top to
// bottom, keeping the vertical neighbours in registers: about three LDS
// reads per cell-update.  Cells outside F(l+2) (half-widths hx2, hy2) are
// also written to the level's global buffer.
template <typename T>
__device__ __forceinline__ void heat_level(const T* __restrict__ prev, T* __restrict__ cur, T* __restrict__ gout,
                                           int W, int C, const LevelEntry& e, int hx2, int hy2, int ox, int oy,
                                           int N, T r)
{
    const int fw = e.fw, nthr = blockDim.x;
    for (int t = threadIdx.x; t < fw * e.spc; t += nthr) {
        const int sidx = qdiv(t, e.inv_fw);
        const int x = e.x0 + (t - sidx * fw);
        const int ys = e.y0 + sidx * e.R;
        const int ye = min(ys + e.R, e.y0 + e.fh);
        const bool xkeep = (x - C >= -hx2) && (x - C < hx2);
        const int gx = wrapi(ox + x, N);
        int gy = wrapi(oy + ys, N);
        int li = ys * W + x;
        T up = prev[li - W];
        T c = prev[li];
        for (int y = ys; y < ye; ++y) {
            const T dn = prev[li + W];
            const T v = heat_update<T>(c, prev[li + 1], prev[li - 1], dn, up, r);
            cur[li] = v;
            const bool keep = xkeep && (y - C >= -hy2) && (y - C < hy2);
            if (!keep) gout[(size_t)gy * N + gx] = v;
            up = c;
            c = dn;
            li += W;
            gy = (gy + 1 == N) ? 0 : gy + 1;
        }
    }
}

template <class S, typename T>
__global__ void __launch_bounds__(S::MAXWG) swept_phase_kernel(PhaseArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    constexpr int NVAR = S::NVAR, R = S::R;
    const int b = a.tile, h = a.h, N = a.N, L = a.L;
    const int W = b + 2 * R, P = W * W;
    const size_t NN = (size_t)N * N;
    const int tiles = a.tiles, t2 = tiles * tiles;

    // instance decode: phase 2w -> Octahedron (w, w); phase 2w-1 -> Bridges (w, w-1) then (w-1, w)
    int wx, wy, inst = blockIdx.x;
    if ((a.phase & 1) == 0) {
        wx = wy = a.phase >> 1;
    } else {
        const int w = (a.phase + 1) >> 1;
        const int k = inst >= t2;
        inst -= k * t2;
        wx = k ? w - 1 : w;
        wy = k ? w : w - 1;
    }
    const int jx = inst % tiles, jy = inst / tiles;
    const int wmax = wx > wy ? wx : wy, wmin = wx < wy ? wx : wy;
    const int lo = max(1, (wmax - 1) * h + 1);
    const int hi = min(L, (wmin + 1) * h - 1);
    if (lo > hi) return;

    const int C = b / 2 + R;  // window centre (local): footprints are [C-hw, C+hw)
    const int cx = jx * b + ((wx & 1) ? 0 : b / 2);
    const int cy = jy * b + ((wy & 1) ? 0 : b / 2);
    const int ox = cx - C, oy = cy - C;
    T* g0 = reinterpret_cast<T*>(a.buf0);
    T* g1 = reinterpret_cast<T*>(a.buf1);
    const int BUF = NVAR * P;  // LDS values per level-parity buffer (address arithmetic keeps ds_* access)

    preload_rings<S, T>(lds, BUF, g0, g1, W, P, N, NN, ox, oy, wx, wy, lo, hi, h, C);
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
    for (int lvl = lo; lvl <= hi; ++lvl) {
        const LevelEntry e = tab[lvl - kbase];
        const bool has2 = lvl + 2 <= hi;
        const int hx2 = has2 ? e.hx2 : 0, hy2 = has2 ? e.hy2 : 0;
        const T* prev = lds + ((lvl - 1) & 1) * BUF;
        T* cur = lds + (lvl & 1) * BUF;
        T* gout = (lvl & 1) ? g1 : g0;
        if constexpr (NVAR == 1) {
            heat_level<T>(prev, cur, gout, W, C, e, hx2, hy2, ox, oy, N, (T)a.p[0]);
        } else {
            const int fw = e.fw, cnt = fw * e.fh;
            for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
                const int q = qdiv(i, e.inv_fw);
                const int ly = e.y0 + q, lx = e.x0 + (i - q * fw);
                const int li = ly * W + lx;
                T out[NVAR];
                cell_update<S, T>(prev, cur, li, W, P, lvl, a, out);
#pragma unroll
                for (int v = 0; v < NVAR; ++v) cur[v * P + li] = out[v];
                const int dx = lx - C, dy = ly - C;  // in F(l+2) <=> -hw2 <= d < hw2
                const bool keep = (dx >= -hx2) && (dx < hx2) && (dy >= -hy2) && (dy < hy2);
                if (!keep) {
                    const size_t gi = (size_t)wrapi(oy + ly, N) * N + wrapi(ox + lx, N);
#pragma unroll
                    for (int v = 0; v < NVAR; ++v) gout[v * NN + gi] = out[v];
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ Standard steps

// Heat: one step per launch (Sec. 3.1 Standard).  Block 64 x 4 threads;
// each thread walks STD_ROWS rows of one column, reusing the vertical
// neighbours in registers.
constexpr int STD_ROWS = 8;

template <typename T>
__global__ void __launch_bounds__(256) heat_standard_kernel(const T* __restrict__ in, T* __restrict__ out, int N,
                                                            T r)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y0 = (blockIdx.y * 4 + threadIdx.y) * STD_ROWS;
    if (x >= N || y0 >= N) return;
    const int xm = wrapi(x - 1, N), xp = wrapi(x + 1, N);
    T up = in[(size_t)wrapi(y0 - 1, N) * N + x];
    T c = in[(size_t)y0 * N + x];
#pragma unroll
    for (int k = 0; k < STD_ROWS; ++k) {
        const int y = y0 + k;
        if (y >= N) break;
        const T dn = in[(size_t)wrapi(y + 1, N) * N + x];
        const size_t row = (size_t)y * N;
        out[row + x] = heat_update<T>(c, in[row + xp], in[row + xm], dn, up, r);
        up = c;
        c = dn;
    }
}

// Euler: one full RK2 step per launch.  A TSxTS output tile loads Q^n on the
// tile plus a 4-cell halo into LDS, computes Q* on the tile plus 2 cells,
// then Q^{n+1} on the tile (both stages with the same cell function as the
// swept kernels).
template <typename T>
__global__ void __launch_bounds__(256) euler_standard_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                             StdArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int TS = a.ts, N = a.N;
    const int Wq = TS + 8, Pq = Wq * Wq, Ws = TS + 4, Ps = Ws * Ws;
    T* q = reinterpret_cast<T*>(smem_raw);
    T* qs = q + 4 * Pq;
    const size_t NN = (size_t)N * N;
    const int tx0 = blockIdx.x * TS, ty0 = blockIdx.y * TS;
    const float inv_wq = 1.0f / (float)Wq, inv_ws = 1.0f / (float)Ws, inv_ts = 1.0f / (float)TS;
    for (int i = threadIdx.x; i < Pq; i += blockDim.x) {
        const int ly = qdiv(i, inv_wq), lx = i - ly * Wq;
        const size_t gi = (size_t)wrapi(ty0 - 4 + ly, N) * N + wrapi(tx0 - 4 + lx, N);
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v * Pq + i] = in[v * NN + gi];
    }
    __syncthreads();
    const T gamma = (T)a.p[0];
    for (int i = threadIdx.x; i < Ps; i += blockDim.x) {
        const int ly = qdiv(i, inv_ws), lx = i - ly * Ws;
        const int qi = (ly + 2) * Wq + (lx + 2);
        T o[4];
        euler_cell<T>(q, Pq, Wq, qi, q, Pq, qi, gamma, (T)a.p[1], (T)a.p[2], o);
#pragma unroll
        for (int v = 0; v < 4; ++v) qs[v * Ps + i] = o[v];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TS * TS; i += blockDim.x) {
        const int ly = qdiv(i, inv_ts), lx = i - ly * TS;
        const int si = (ly + 2) * Ws + (lx + 2);
        const int qi = (ly + 4) * Wq + (lx + 4);
        T o[4];
        euler_cell<T>(qs, Ps, Ws, si, q, Pq, qi, gamma, (T)a.p[3], (T)a.p[4], o);
        const size_t gi = (size_t)(ty0 + ly) * N + (tx0 + lx);
#pragma unroll
        for (int v = 0; v < 4; ++v) out[v * NN + gi] = o[v];
    }
}

// --------------------------------------------------------------- reductions
// Fixed-order reductions: block k always sums the same contiguous chunk in
// the same tree order, then one block combines the partials in order, so
// results are reproducible run to run.

template <typename T>
__global__ void __launch_bounds__(256) plane_sum_partials(const T* __restrict__ x, size_t NN, int chunk,
                                                          double* __restrict__ partials)
{
    __shared__ double red[256];
    const int plane = blockIdx.y;
    const size_t begin = (size_t)blockIdx.x * chunk;
    const size_t end = begin + chunk < NN ? begin + chunk : NN;
    const T* p = x + plane * NN;
    double s = 0.0;
    for (size_t i = begin + threadIdx.x; i < end; i += blockDim.x) s += (double)p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[plane * gridDim.x + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) combine_partials(const double* __restrict__ partials, int nparts, int op_max,
                                                        double* __restrict__ out)
{
    __shared__ double red[256];
    const int plane = blockIdx.x;
    double s = op_max ? -INFINITY : 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        const double v = partials[plane * nparts + i];
        s = op_max ? (v > s ? v : s) : s + v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            red[threadIdx.x] = op_max ? (o > red[threadIdx.x] ? o : red[threadIdx.x]) : red[threadIdx.x] + o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[plane] = red[0];
}

// Per-block maximum of the CFL signal rate (|u|+c)/dx + (|v|+c)/dy, in double.
template <typename T>
__global__ void __launch_bounds__(256) cfl_partials(const T* __restrict__ q, size_t NN, int chunk, double gamma,
                                                    double dx, double dy, double* __restrict__ partials)
{
    __shared__ double red[256];
    const size_t begin = (size_t)blockIdx.x * chunk;
    const size_t end = begin + chunk < NN ? begin + chunk : NN;
    double m = -INFINITY;
    for (size_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
        const double rho = (double)q[i], mu = (double)q[NN + i], mv = (double)q[2 * NN + i],
                     E = (double)q[3 * NN + i];
        const double u = mu / rho, v = mv / rho;
        const double p = (gamma - 1.0) * (E - 0.5 * (mu * u + mv * v));
        const double c = sqrt(gamma * p / rho);
        const double s = (fabs(u) + c) / dx + (fabs(v) + c) / dy;
        m = s > m ? s : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x + w] > red[threadIdx.x] ? red[threadIdx.x + w]
                                                                                               : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ launchers

template <class S, typename T>
static hipError_t launch_phase_t(const PhaseArgs& a, int wg, size_t lds, hipStream_t st)
{
    const int t2 = a.tiles * a.tiles;
    const int nblk = (a.phase & 1) ? 2 * t2 : t2;
    hipLaunchKernelGGL((swept_phase_kernel<S, T>), dim3(nblk), dim3(wg), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_phase(int kind, int dtype, const PhaseArgs& a, int wg, size_t lds, hipStream_t st)
{
    if (kind == 0) return dtype == 0 ? launch_phase_t<HeatS, double>(a, wg, lds, st)
                                     : launch_phase_t<HeatS, float>(a, wg, lds, st);
    return dtype == 0 ? launch_phase_t<EulerS, double>(a, wg, lds, st) : launch_phase_t<EulerS, float>(a, wg, lds, st);
}

hipError_t set_phase_lds_limit(int kind, int dtype, size_t lds)
{
    const void* f;
    if (kind == 0) f = dtype == 0 ? (const void*)swept_phase_kernel<HeatS, double> : (const void*)swept_phase_kernel<HeatS, float>;
    else f = dtype == 0 ? (const void*)swept_phase_kernel<EulerS, double> : (const void*)swept_phase_kernel<EulerS, float>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_heat_standard(int dtype, const void* in, void* out, int N, double r, hipStream_t st)
{
    dim3 blk(64, 4), grd((N + 63) / 64, (N + 4 * STD_ROWS - 1) / (4 * STD_ROWS));
    if (dtype == 0)
        hipLaunchKernelGGL(heat_standard_kernel<double>, grd, blk, 0, st, (const double*)in, (double*)out, N, r);
    else
        hipLaunchKernelGGL(heat_standard_kernel<float>, grd, blk, 0, st, (const float*)in, (float*)out, N, (float)r);
    return hipGetLastError();
}

size_t euler_standard_lds(int dtype, int ts)
{
    const size_t s = dtype == 0 ? 8 : 4;
    return 4 * s * ((size_t)(ts + 8) * (ts + 8) + (size_t)(ts + 4) * (ts + 4));
}

hipError_t set_euler_standard_lds_limit(int dtype, size_t lds)
{
    const void* f = dtype == 0 ? (const void*)euler_standard_kernel<double> : (const void*)euler_standard_kernel<float>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_euler_standard(int dtype, const void* in, void* out, const StdArgs& a, hipStream_t st)
{
    dim3 grd(a.N / a.ts, a.N / a.ts);
    const size_t lds = euler_standard_lds(dtype, a.ts);
    if (dtype == 0)
        hipLaunchKernelGGL(euler_standard_kernel<double>, grd, dim3(256), lds, st, (const double*)in, (double*)out, a);
    else
        hipLaunchKernelGGL(euler_standard_kernel<float>, grd, dim3(256), lds, st, (const float*)in, (float*)out, a);
    return hipGetLastError();
}

hipError_t launch_plane_sums(int dtype, const void* x, int nvar, size_t NN, double* partials, int nparts,
                             double* out, hipStream_t st)
{
    const int chunk = (int)((NN + nparts - 1) / nparts);
    if (dtype == 0)
        hipLaunchKernelGGL(plane_sum_partials<double>, dim3(nparts, nvar), dim3(256), 0, st, (const double*)x, NN, chunk,
                           partials);
    else
        hipLaunchKernelGGL(plane_sum_partials<float>, dim3(nparts, nvar), dim3(256), 0, st, (const float*)x, NN, chunk,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(combine_partials, dim3(nvar), dim3(256), 0, st, partials, nparts, 0, out);
    return hipGetLastError();
}

hipError_t launch_cfl_max(int dtype, const void* q, size_t NN, double gamma, double dx, double dy, double* partials,
                          int nparts, double* out, hipStream_t st)
{
    const int chunk = (int)((NN + nparts - 1) / nparts);
    if (dtype == 0)
        hipLaunchKernelGGL(cfl_partials<double>, dim3(nparts), dim3(256), 0, st, (const double*)q, NN, chunk, gamma, dx,
                           dy, partials);
    else
        hipLaunchKernelGGL(cfl_partials<float>, dim3(nparts), dim3(256), 0, st, (const float*)q, NN, chunk, gamma, dx, dy,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(combine_partials, dim3(1), dim3(256), 0, st, partials, nparts, 1, out);
    return hipGetLastError();
}

}  // namespace swept
