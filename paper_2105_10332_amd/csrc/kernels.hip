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

#include <mutex>

#include "device_common.h"

namespace swept {

// B > 0: heat instantiated for one tile edge (see phase_instance); B = 0: any tile.
template <class S, typename T, int B, bool TAPED = false>
__global__ void __launch_bounds__((max_wg<S, T>())) swept_phase_kernel(PhaseArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    phase_instance<S, T, B, TAPED>(a, blockIdx.x, smem_raw);
}

// ------------------------------------------------------------ Standard steps

// Heat: one step per launch (Sec. 3.1 Standard).  A workgroup of WG threads
// covers WG consecutive columns and ROWS rows: each thread walks the rows of
// its column, keeping the vertical neighbours in registers, so the halo rows
// add 2/ROWS to the reads.  The left and right neighbours come from the
// adjacent lanes by DPP wavefront shifts; only the lanes at a wavefront's
// edge (or next to a column past the grid) load theirs, from cache lines the
// neighbouring wavefront of the same workgroup reads anyway.  The launch takes
// the largest of 512 x 16, 256 x 8 and 128 x 4 that still gives 2048
// workgroups (measured per 500 FP64 steps: 4096^2 22.4 ms with 512 x 16,
// 2048^2 6.5 ms with 256 x 8 against 7.6, 320^2 1.8 ms with 128 x 4 against 3.6).

template <typename T>
__device__ __forceinline__ T lane_shift(T v, bool next)
{
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
        const unsigned l = next ? __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, false)
                                : __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
        const unsigned h = next ? __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, false)
                                : __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
        return __longlong_as_double((long long)(((unsigned long long)h << 32) | l));
    } else {
        const int i = __float_as_int(v);
        return __int_as_float(next ? __builtin_amdgcn_update_dpp(0, i, 0x130, 0xf, 0xf, false)
                                   : __builtin_amdgcn_update_dpp(0, i, 0x138, 0xf, 0xf, false));
    }
}

// BC: 0 periodic; 1 Dirichlet (outside neighbours read bcv); 2 zero flux
// (outside neighbours read the edge cell itself).
template <typename T, int BC, int WG, int ROWS>
__global__ void __launch_bounds__(WG) heat_standard_kernel(const T* __restrict__ in, T* __restrict__ out, int N, T r,
                                                           T bcv)
{
    const int lane = threadIdx.x & 63;
    const int x = blockIdx.x * WG + threadIdx.x;
    const int y0 = blockIdx.y * ROWS;
    const bool live = x < N;
    const int xc = live ? x : N - 1;  // lanes past the grid read a valid column; they store nothing
    const bool own_r = lane < 63 && x + 1 < N;  // lane + 1 holds column x + 1
    const bool own_l = lane > 0;                // lane - 1 holds column x - 1
    const int xm = wrapi(xc - 1, N), xp = wrapi(xc + 1, N);
    T up = in[(size_t)wrapi(y0 - 1, N) * N + xc];
    T c = in[(size_t)y0 * N + xc];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int y = y0 + k;
        if (y >= N) break;
        const size_t row = (size_t)y * N;
        const T dn = in[(size_t)wrapi(y + 1, N) * N + xc];
        T vr = lane_shift(c, true), vl = lane_shift(c, false);
        if (!own_r) vr = in[row + xp];
        if (!own_l) vl = in[row + xm];
        if (live) {
            if constexpr (BC == 0) {
                out[row + x] = heat_update<T>(c, vr, vl, dn, up, r);
            } else {
                const T g = BC == 1 ? bcv : c;
                out[row + x] = heat_update<T>(c, x == N - 1 ? g : vr, x == 0 ? g : vl, y == N - 1 ? g : dn,
                                              y == 0 ? g : up, r);
            }
        }
        up = c;
        c = dn;
    }
}

// Euler: one full RK2 step per launch.  A TSxTS output tile loads Q^n on the
// tile plus a 4-cell halo into LDS (row pitch W + kEulerPad) with the
// pressure of every cell, and runs the same level function as the swept
// kernels twice: Q* (and its pressures) on the tile plus 2 cells, then
// Q^{n+1} on the tile.
template <typename T>
struct TileStore {
    T* out;
    size_t NN;
    int N, gx0, gy0;  // global position of window cell (0, 0)
    __device__ __forceinline__ void operator()(int lx, int ly, const T* v) const
    {
        const size_t gi = (size_t)(gy0 + ly) * N + (gx0 + lx);
#pragma unroll
        for (int c = 0; c < 4; ++c) out[c * NN + gi] = v[c];
    }
};

template <typename T, int V, int BC>
__global__ void __launch_bounds__(256) euler_standard_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                             StdArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int TS = a.ts, N = a.N;
    const int W = TS + 8, PW = W + kEulerPad, P = PW * W, BUF = 4 * P;
    const size_t NN = (size_t)N * N;
    const int tx0 = blockIdx.x * TS, ty0 = blockIdx.y * TS;
    const T gamma = (T)a.p[0], gm1 = gamma - T(1);
    T* q0 = lds;
    T* q1 = lds + BUF;
    T* p0 = lds + 2 * BUF;
    T* p1 = p0 + P;
    const float inv_w = 1.0f / (float)W;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < W * W; i += nthr) {
        const int ly = qdiv(i, inv_w), lx = i - ly * W;
        const size_t gi = (size_t)wrapi(ty0 - 4 + ly, N) * N + wrapi(tx0 - 4 + lx, N);
        T s4[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) s4[v] = in[v * NN + gi];
#pragma unroll
        for (int v = 0; v < 4; ++v) q0[v * P + ly * PW + lx] = s4[v];
        p0[ly * PW + lx] = pressure(s4, gm1);
    }
    __syncthreads();
    const TileStore<T> st{out, NN, N, tx0 - 4, ty0 - 4};
    const int ex = window_edge(tx0 - 4, W, N), ey = window_edge(ty0 - 4, W, N);
    if (BC != 0 && (ex >= 0 || ey >= 0)) {  // a tile at the walls
        euler_level<T, V, NoStore, BC>(q0, q1, p0, p1, PW, P, 2, 2, TS + 4, TS + 4, false, gamma, (T)a.p[1],
                                       (T)a.p[2], NoStore{}, nthr, ex, ey);
        __syncthreads();
        euler_level<T, V, TileStore<T>, BC, false>(q1, q0, p1, p0, PW, P, 4, 4, TS, TS, true, gamma, (T)a.p[3],
                                                   (T)a.p[4], st, nthr, ex, ey);
    } else {
        euler_level<T, V>(q0, q1, p0, p1, PW, P, 2, 2, TS + 4, TS + 4, false, gamma, (T)a.p[1], (T)a.p[2],
                          NoStore{}, nthr);
        __syncthreads();
        euler_level<T, V, TileStore<T>, 0, false>(q1, q0, p1, p0, PW, P, 4, 4, TS, TS, true, gamma, (T)a.p[3],
                                                  (T)a.p[4], st, nthr);
    }
}

// --------------------------------------------------------------- reductions
// Fixed-order reductions: block k always sums the same contiguous chunk in
// the same tree order, then one block combines the partials in order, so
// results are reproducible run to run.

// Maximum that propagates NaN (a non-finite rate must not be skipped by the max).
__device__ __forceinline__ double nan_max(double a, double b) { return (a != a || a > b) ? a : b; }

struct SumOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct MaxOp {
    __device__ double operator()(double a, double b) const { return nan_max(a, b); }
};

// Block reduction of one double per thread: a butterfly over the 64 lanes of
// each wavefront (lane i combines with lane i ^ o, o = 32 ... 1; both partners
// get the same value, so the order is fixed), then thread 0 combines the
// waves' results in wave order.  red holds one value per wave.  The result is
// valid in thread 0.
template <class Op>
__device__ __forceinline__ double block_reduce(double v, Op op, double* red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
    if (threadIdx.x == 0)
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = op(r, red[w]);
    return r;
}

template <typename T>
__global__ void __launch_bounds__(256) plane_sum_partials(const T* __restrict__ x, size_t NN, int chunk,
                                                          double* __restrict__ partials)
{
    __shared__ double red[4];
    const int plane = blockIdx.y;
    const size_t begin = (size_t)blockIdx.x * chunk;
    const size_t end = begin + chunk < NN ? begin + chunk : NN;
    const T* p = x + plane * NN;
    double s = 0.0;
    for (size_t i = begin + threadIdx.x; i < end; i += blockDim.x) s += (double)p[i];
    s = block_reduce(s, SumOp{}, red);
    if (threadIdx.x == 0) partials[plane * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) combine_partials(const double* __restrict__ partials, int nparts, int op_max,
                                                        double* __restrict__ out)
{
    __shared__ double red[4];
    const int plane = blockIdx.x;
    double s = op_max ? -INFINITY : 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        const double v = partials[plane * nparts + i];
        s = op_max ? nan_max(v, s) : s + v;
    }
    s = op_max ? block_reduce(s, MaxOp{}, red) : block_reduce(s, SumOp{}, red);
    if (threadIdx.x == 0) out[plane] = s;
}

// Per-block maximum of the CFL signal rate (|u|+c)/dx + (|v|+c)/dy, in double.
template <typename T>
__global__ void __launch_bounds__(256) cfl_partials(const T* __restrict__ q, size_t NN, int chunk, double gamma,
                                                    double dx, double dy, double* __restrict__ partials)
{
    __shared__ double red[4];
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
        m = nan_max(s, m);
    }
    m = block_reduce(m, MaxOp{}, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = m;
}

// ------------------------------------------------------------------ launchers

// The phase kernel instantiation for a problem: heat at b = 16, 32 or 64
// gets a fixed-tile copy, everything else the runtime-tile one.
template <class S, typename T, bool TAPED = false>
static const void* phase_kernel(int tile)
{
    if constexpr (S::NVAR == 1) {
        if (tile == 64) return (const void*)swept_phase_kernel<S, T, 64, TAPED>;
        if (tile == 32) return (const void*)swept_phase_kernel<S, T, 32, TAPED>;
        if (tile == 16) return (const void*)swept_phase_kernel<S, T, 16, TAPED>;
    }
    return (const void*)swept_phase_kernel<S, T, 0, TAPED>;
}

template <int V, int BC>
static const void* euler_phase_v(int dtype)
{
    return dtype == 0 ? phase_kernel<EulerSV<V, BC>, double>(0) : phase_kernel<EulerSV<V, BC>, float>(0);
}

template <int V>
static const void* euler_phase_kernel(int dtype, int bc)
{
    if (bc == 2) return euler_phase_v<V, 2>(dtype);
    if (bc == 3) return euler_phase_v<V, 3>(dtype);
    return euler_phase_v<V, 0>(dtype);
}

template <int BC>
static const void* heat_phase_kernel(int dtype, int tile, bool taped)
{
    if (taped)  // the first Octahedron of the adjoint's taped cycle (rings by owner)
        return dtype == 0 ? phase_kernel<HeatSV<BC>, double, true>(tile) : phase_kernel<HeatSV<BC>, float, true>(tile);
    return dtype == 0 ? phase_kernel<HeatSV<BC>, double>(tile) : phase_kernel<HeatSV<BC>, float>(tile);
}

// scheme: Euler variant bits; bc: heat boundary.  Each combination is its own
// instantiation, so the periodic minmod kernels carry no test for the others.
static const void* phase_kernel(int kind, int dtype, int tile, int scheme, int bc, bool taped = false)
{
    if (kind == 0) {
        if (bc == 1) return heat_phase_kernel<1>(dtype, tile, taped);
        if (bc == 2) return heat_phase_kernel<2>(dtype, tile, taped);
        return heat_phase_kernel<0>(dtype, tile, taped);
    }
    switch (scheme) {
        case 1: return euler_phase_kernel<1>(dtype, bc);
        case 2: return euler_phase_kernel<2>(dtype, bc);
        case 3: return euler_phase_kernel<3>(dtype, bc);
        default: return euler_phase_kernel<0>(dtype, bc);
    }
}

hipError_t launch_phase(int kind, int dtype, const PhaseArgs& a, int wg, size_t lds, hipStream_t st)
{
    const int per = a.tiles * (a.jrows > 0 ? a.jrows : a.tiles);
    const int nblk = (a.phase & 1) ? 2 * per : per;
    void* args[] = {(void*)&a};
    return hipLaunchKernel(phase_kernel(kind, dtype, a.tile, a.scheme, a.bc, a.q0 != nullptr), dim3(nblk), dim3(wg),
                           args, lds, st);
}

hipError_t set_phase_lds_limit(int kind, int dtype, size_t lds)
{
    hipError_t e = hipSuccess;
    for (int bc = 0; bc < 4; ++bc)  // heat: boundaries 0-2; Euler: boundaries 0, 2, 3 x scheme bits
        for (int v = 0; v < (kind == 0 ? 1 : 4); ++v)
            for (int tile : {0, 16, 32, 64})
                for (int taped = 0; taped < (kind == 0 ? 2 : 1); ++taped)
                    if (e == hipSuccess && !(kind == 0 && bc == 3) && !(kind == 1 && bc == 1))
                        e = hipFuncSetAttribute(phase_kernel(kind, dtype, tile, v, bc, taped != 0),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return e;
}

template <typename T, int BC>
static void heat_standard_launch(const void* in, void* out, int N, double r, double bcv, hipStream_t st)
{
    const auto groups = [N](int wg, int rows) { return (long long)((N + wg - 1) / wg) * ((N + rows - 1) / rows); };
    if (groups(512, 16) >= 2048) {
        dim3 blk(512), grd((N + 511) / 512, (N + 15) / 16);
        hipLaunchKernelGGL((heat_standard_kernel<T, BC, 512, 16>), grd, blk, 0, st, (const T*)in, (T*)out, N, (T)r,
                           (T)bcv);
    } else if (groups(256, 8) >= 2048) {
        dim3 blk(256), grd((N + 255) / 256, (N + 7) / 8);
        hipLaunchKernelGGL((heat_standard_kernel<T, BC, 256, 8>), grd, blk, 0, st, (const T*)in, (T*)out, N, (T)r,
                           (T)bcv);
    } else {
        dim3 blk(128), grd((N + 127) / 128, (N + 3) / 4);
        hipLaunchKernelGGL((heat_standard_kernel<T, BC, 128, 4>), grd, blk, 0, st, (const T*)in, (T*)out, N, (T)r,
                           (T)bcv);
    }
}

hipError_t launch_heat_standard(int dtype, const void* in, void* out, int N, double r, int bc, double bcv,
                                hipStream_t st)
{
    if (dtype == 0) {
        if (bc == 1) heat_standard_launch<double, 1>(in, out, N, r, bcv, st);
        else if (bc == 2) heat_standard_launch<double, 2>(in, out, N, r, bcv, st);
        else heat_standard_launch<double, 0>(in, out, N, r, bcv, st);
    } else {
        if (bc == 1) heat_standard_launch<float, 1>(in, out, N, r, bcv, st);
        else if (bc == 2) heat_standard_launch<float, 2>(in, out, N, r, bcv, st);
        else heat_standard_launch<float, 0>(in, out, N, r, bcv, st);
    }
    return hipGetLastError();
}

size_t euler_standard_lds(int dtype, int ts)
{
    const size_t s = dtype == 0 ? 8 : 4;
    return s * euler_lds_values(ts + 8);
}

size_t euler_phase_lds(int dtype, int tile)
{
    const size_t s = dtype == 0 ? 8 : 4;
    return s * euler_lds_values(tile + 4);
}

template <int V, int BC>
static const void* euler_standard_vb(int dtype)
{
    return dtype == 0 ? (const void*)euler_standard_kernel<double, V, BC>
                      : (const void*)euler_standard_kernel<float, V, BC>;
}

template <int V>
static const void* euler_standard_v(int dtype, int bc)
{
    if (bc == 2) return euler_standard_vb<V, 2>(dtype);
    if (bc == 3) return euler_standard_vb<V, 3>(dtype);
    return euler_standard_vb<V, 0>(dtype);
}

static const void* euler_standard(int dtype, int scheme, int bc)
{
    switch (scheme) {
        case 1: return euler_standard_v<1>(dtype, bc);
        case 2: return euler_standard_v<2>(dtype, bc);
        case 3: return euler_standard_v<3>(dtype, bc);
        default: return euler_standard_v<0>(dtype, bc);
    }
}

hipError_t set_euler_standard_lds_limit(int dtype, size_t lds)
{
    hipError_t e = hipSuccess;
    for (int bc : {0, 2, 3})
        for (int scheme = 0; scheme < 4 && e == hipSuccess; ++scheme)
            e = hipFuncSetAttribute(euler_standard(dtype, scheme, bc), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds);
    return e;
}

hipError_t launch_euler_standard(int dtype, const void* in, void* out, const StdArgs& a, hipStream_t st)
{
    dim3 grd(a.N / a.ts, a.N / a.ts);
    const size_t lds = euler_standard_lds(dtype, a.ts);
    void* args[] = {(void*)&in, (void*)&out, (void*)&a};
    return hipLaunchKernel(euler_standard(dtype, a.scheme, a.bc), grd, dim3(256), args, lds, st);
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

hipError_t launch_combine(const double* partials, int nparts, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(combine_partials, dim3(1), dim3(256), 0, st, partials, nparts, 0, out);
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

// ------------------------------------------------- allocation-free scratch
// Partials and result of the CFL max-reduction of swept_cfl_dt_noalloc: a
// file-scope device array (each GPU holds its own copy until the process
// ends).  In host code its name is only a stand-in, so the device address is
// looked up once per device and kept; kernels get that address.
static __device__ __align__(256) double scratch[kNoAllocParts + 1];

hipError_t noalloc_scratch(double** out)
{
    static std::mutex mu;
    static double* ptr[kNoAllocMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double*>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace swept
