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
// Memory protocol (level l of a cell lives in global buffer l mod 2).  For
// each level l of its shape a workgroup
//   1. loads Box(F(l), n) minus F(l-1), at level l-1, from buffer (l-1)%2
//      into LDS buffer (l-1)%2 (F = footprint rectangle of the level);
//   2. computes F(l) into LDS buffer l%2 (Euler's second stage also reads
//      the cell's own level l-2 value from LDS buffer l%2, in place);
//   3. stores the cells of F(l) that are not in F(l+2) to buffer l%2:
//      exactly the values later shapes read.
// The load for l+1 is issued right after the compute of l (it touches only
// cells outside F(l)), so each level costs one barrier.
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

// Load the ring Box(bx0..bx1, by0..by1) minus hole (hx0..hx1, hy0..hy1),
// local window coordinates, from global buffer g (planes of NN values) into
// the LDS buffer l (planes of P values, row stride W).  An empty hole is
// given as hx0 == hx1.
template <int NVAR, typename T>
__device__ __forceinline__ void load_ring(T* __restrict__ l, const T* __restrict__ g, int W, int P, int N, size_t NN,
                                          int ox, int oy, int bx0, int bx1, int by0, int by1, int hx0, int hx1,
                                          int hy0, int hy1)
{
    if (hx0 >= hx1) {  // no hole: the whole box as the top region
        hy0 = hy1 = by1;
        hx0 = hx1 = bx1;
    }
    const int bw = bx1 - bx0;
    const int n_top = bw * (hy0 - by0);
    const int n_bot = bw * (by1 - hy1);
    const int sh = hy1 - hy0;
    const int swl = hx0 - bx0, swr = bx1 - hx1;
    const int n_l = swl * sh, n_r = swr * sh;
    const int total = n_top + n_bot + n_l + n_r;
    const float inv_bw = 1.0f / (float)(bw > 0 ? bw : 1);
    const float inv_l = 1.0f / (float)(swl > 0 ? swl : 1);
    const float inv_r = 1.0f / (float)(swr > 0 ? swr : 1);
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        int lx, ly, k = i;
        if (k < n_top) {
            const int q = qdiv(k, inv_bw);
            ly = by0 + q;
            lx = bx0 + (k - q * bw);
        } else if ((k -= n_top) < n_bot) {
            const int q = qdiv(k, inv_bw);
            ly = hy1 + q;
            lx = bx0 + (k - q * bw);
        } else if ((k -= n_bot) < n_l) {
            const int q = qdiv(k, inv_l);
            ly = hy0 + q;
            lx = bx0 + (k - q * swl);
        } else {
            k -= n_l;
            const int q = qdiv(k, inv_r);
            ly = hy0 + q;
            lx = hx1 + (k - q * swr);
        }
        const int gx = wrapi(ox + lx, N), gy = wrapi(oy + ly, N);
        const size_t gi = (size_t)gy * N + gx;
        const int li = ly * W + lx;
#pragma unroll
        for (int v = 0; v < NVAR; ++v) l[v * P + li] = g[v * NN + gi];
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
    T* g[2] = {reinterpret_cast<T*>(a.buf0), reinterpret_cast<T*>(a.buf1)};
    T* lb[2] = {lds, lds + NVAR * P};

    // first level: whole Box(F(lo), R) at level lo-1
    {
        const int hx = half_width(wx, lo, h, R), hy = half_width(wy, lo, h, R);
        load_ring<NVAR, T>(lb[(lo - 1) & 1], g[(lo - 1) & 1], W, P, N, NN, ox, oy, C - hx - R, C + hx + R,
                           C - hy - R, C + hy + R, 0, 0, 0, 0);
        if (S::TWO_STAGE && (lo & 1) == 0)  // own cells at level lo-2 for the second RK stage
            load_ring<NVAR, T>(lb[lo & 1], g[lo & 1], W, P, N, NN, ox, oy, C - hx, C + hx, C - hy, C + hy, 0, 0,
                               0, 0);
    }
    __syncthreads();

    for (int lvl = lo; lvl <= hi; ++lvl) {
        const int hx = half_width(wx, lvl, h, R), hy = half_width(wy, lvl, h, R);
        const int hx2 = (lvl + 2 <= hi) ? half_width(wx, lvl + 2, h, R) : 0;
        const int hy2 = (lvl + 2 <= hi) ? half_width(wy, lvl + 2, h, R) : 0;
        const int fw = 2 * hx, cnt = fw * 2 * hy;
        const float inv_fw = 1.0f / (float)fw;
        const T* prev = lb[(lvl - 1) & 1];
        T* cur = lb[lvl & 1];
        T* gout = g[lvl & 1];
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            const int q = qdiv(i, inv_fw);
            const int ly = C - hy + q, lx = C - hx + (i - q * fw);
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
        if (lvl < hi) {  // ring for level l+1: Box(F(l+1), R) minus F(l), at level l
            const int nx_ = half_width(wx, lvl + 1, h, R), ny_ = half_width(wy, lvl + 1, h, R);
            load_ring<NVAR, T>(cur, gout, W, P, N, NN, ox, oy, C - nx_ - R, C + nx_ + R, C - ny_ - R, C + ny_ + R,
                               C - hx, C + hx, C - hy, C + hy);
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
