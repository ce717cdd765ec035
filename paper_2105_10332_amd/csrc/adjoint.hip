// adjoint.hip -- the hand-written adjoint of the swept heat advance.
//
// J depends on the final state T^M; given g = dJ/dT^M, the reverse sweep
// lambda^M = g, lambda^m = A^T lambda^{m+1} gives dJ/dT^0 = lambda^0 and
// dJ/dr = sum_{m<M} <lambda^{m+1}, L T^m> (T^{m+1} = A T^m, A = I + r L, L the
// periodic 5-point operator; dJ/dalpha = dJ/dr * dt/dx^2).  A is symmetric,
// so A^T lambda is the same heat update applied to lambda, and the pairing
// is evaluated as <L lambda^{m+1}, T^m>, which needs T^m only at the cell
// where lambda^m is computed.
//
// The forward run is cut into cycles of h = b/2 steps with the flat state at
// each cycle start kept as a checkpoint, and each cycle's forward strips kept
// on the tape: the Up-Pyramid's in P, the Bridges' in Q (the first
// Octahedron reads every ring cell from its owner's buffers).  Backward,
// per cycle:
//   R0, R1, R2 (this file): lambda over the cycle is itself a swept advance
//      of h levels in reversed time k = h - j, starting flat, on the other
//      tiling.  Its k-time Up-Pyramid, Bridges and Down-Pyramid occupy
//      exactly the footprints of the forward Octahedron 1, the forward
//      Bridges (X and Y exchanged) and the forward Up-Pyramid plus level 0.
//      Each reverse workgroup therefore first recomputes the forward T of
//      its footprint in LDS (R0 from P, Q and the checkpoint, the source of
//      each input cell chosen by its owner; R1 from P and the checkpoint; R2
//      from the checkpoint), keeping every level, then runs lambda through
//      the footprint level by level, pairs each lambda update with T at the
//      same cell and level, and stores lambda strips for later reverse
//      shapes with the usual top-two-levels rule.
// Pairing partial sums are reduced per workgroup in double and written to
// one slot each; the host sums the slots in a fixed order.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace swept {

// Forward level of the recompute: F(l) into `cur` (the LDS parity buffer)
// and into the packed all-levels store `pk` (row-major over the footprint).
// BC != 0 (windows that cross the domain edge of a walled problem): a
// neighbour outside the square reads the ghost value (bcv for Dirichlet,
// the cell itself for zero flux), as in the forward phases.
template <typename T, int BC = 0>
__device__ __forceinline__ void heat_level_pack(const T* __restrict__ prev, T* __restrict__ cur, T* __restrict__ pk,
                                                int W, const LevelEntry& e, T r, int ox = 0, int oy = 0, int N = 0,
                                                T bcv = T(0))
{
    const int fw = e.fw, cells = fw * e.fh;
    for (int i = threadIdx.x; i < cells; i += blockDim.x) {
        const int q = qdiv(i, e.inv_fw);
        const int lx = e.x0 + (i - q * fw), ly = e.y0 + q;
        const int li = ly * W + lx;
        const T c = prev[li];
        T v;
        if constexpr (BC != 0) {
            const int gx = wrapi(ox + lx, N), gy = wrapi(oy + ly, N);
            const T gh = BC == 1 ? bcv : c;
            v = heat_update<T>(c, gx == N - 1 ? gh : prev[li + 1], gx == 0 ? gh : prev[li - 1],
                               gy == N - 1 ? gh : prev[li + W], gy == 0 ? gh : prev[li - W], r);
        } else {
            v = heat_update<T>(c, prev[li + 1], prev[li - 1], prev[li + W], prev[li - W], r);
        }
        cur[li] = v;
        pk[i] = v;
    }
}

// Reverse level: lambda on F(k) from lambda at k-1 (`prev`), the pairing
// (L lambda^{k-1}) * T at each cell accumulated in double, and the
// top-two-levels store of lambda.  T comes from the packed store in LDS
// (row-major over the same footprint) or, for the cycle's level 0
// (T_GLOBAL), from the checkpoint in global memory; the two are separate
// instantiations so that each is read with its own load instructions.
// WRAP = false when the window does not cross the periodic boundary.
// Lambda has its own type L (double for both state precisions); T is the
// forward state's type.
//
// Walls (BC != 0, only with WRAP): the walled step is affine, A0 T + r b, with
// A0 the homogeneous walled step (symmetric) and b the Dirichlet ghost terms
// (bcv times the number of outside neighbours).  Lambda runs A0: an outside
// neighbour reads 0 (Dirichlet) or the cell itself (zero flux); the pairing
// <lambda, L0 T + b> adds bcv * (outside neighbours) * lambda at edge cells.
template <typename L, typename T, bool T_GLOBAL, bool WRAP, int BC = 0>
__device__ __forceinline__ double lambda_level(const L* __restrict__ prev, L* __restrict__ cur,
                                               L* __restrict__ gout, const T* __restrict__ tsrc, int W, int C,
                                               const LevelEntry& e, int hx2, int hy2, int ox, int oy, int N, L r,
                                               double bcv = 0.0)
{
    static_assert(BC == 0 || WRAP, "walls are met only by windows that cross the edge");
    const int fw = e.fw, cells = fw * e.fh;
    double acc = 0.0;
    for (int i = threadIdx.x; i < cells; i += blockDim.x) {
        const int q = qdiv(i, e.inv_fw);
        const int lx = e.x0 + (i - q * fw), ly = e.y0 + q;
        const int li = ly * W + lx;
        const L c = prev[li];
        const L two_c = c + c;
        const int gx = WRAP ? wrapi(ox + lx, N) : ox + lx, gy = WRAP ? wrapi(oy + ly, N) : oy + ly;
        L xp = prev[li + 1], xm = prev[li - 1], yp = prev[li + W], ym = prev[li - W];
        int nout = 0;
        if constexpr (BC != 0) {
            const L gh = BC == 1 ? L(0) : c;
            nout = (gx == N - 1) + (gx == 0) + (gy == N - 1) + (gy == 0);
            xp = gx == N - 1 ? gh : xp;
            xm = gx == 0 ? gh : xm;
            yp = gy == N - 1 ? gh : yp;
            ym = gy == 0 ? gh : ym;
        }
        const L dxx = (xp - two_c) + xm;
        const L dyy = (yp - two_c) + ym;
        const L v = (c + r * dxx) + r * dyy;  // the heat update (scheme.h) with its Laplacian kept
        cur[li] = v;
        const T tv = T_GLOBAL ? tsrc[(size_t)gy * N + gx] : tsrc[i];
        acc += ((double)dxx + (double)dyy) * (double)tv;
        if constexpr (BC == 1) acc += bcv * (double)nout * (double)c;
        const int dx = lx - C, dy = ly - C;
        if (!((dx >= -hx2) && (dx < hx2) && (dy >= -hy2) && (dy < hy2))) gout[(size_t)gy * N + gx] = v;
    }
    return acc;
}

// Sum over the workgroup in a fixed pairwise order (any blockDim).
__device__ __forceinline__ double block_sum(double v, double* red)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    red[tid] = v;
    __syncthreads();
    for (int w = 1; w < nt; w <<= 1) {
        if ((tid & (2 * w - 1)) == 0 && tid + w < nt) red[tid] += red[tid + w];
        __syncthreads();
    }
    return red[0];
}

// Byte layout of the adjoint workgroup's LDS (shared by host and device).
// The forward recompute's parity windows, then the lambda parity windows,
// then the reduction scratch use one region in turn (each is dead before the
// next is written); the packed forward levels and their offsets follow.
struct AdjLds {
    size_t pk, offs, total;
};
__host__ __device__ inline AdjLds adjoint_lds_layout(size_t scalar, size_t lscalar, int tile, int pk_max, int wg)
{
    const size_t W = tile + 2;
    const int h = tile / 2;
    const size_t win = (scalar > lscalar ? scalar : lscalar) * 2 * W * W, red = sizeof(double) * wg;
    AdjLds l;
    l.pk = ((win > red ? win : red) + 15) / 16 * 16;
    l.offs = (l.pk + scalar * pk_max + 15) / 16 * 16;
    l.total = l.offs + sizeof(int) * (2 * h + 2);
    return l;
}

// One reverse phase (k-time phase 0, 1 or 2) of a full cycle of h levels.
// LDS: one region of two parity windows (forward T, then lambda, then the
// reduction scratch), the packed forward levels (pk_max values) and their
// offsets.  B > 0 fixes the tile edge at compile time (a.tile must equal
// it), so the window pitch is an immediate LDS offset; B = 0 takes a.tile.
template <typename T, int B, int BC>
__global__ void __launch_bounds__(1024) adjoint_phase_kernel(PhaseArgs a, int pk_max)
{
    using L = double;  // lambda
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = B > 0 ? B : a.tile, h = B > 0 ? B / 2 : a.h, N = a.N;
    const int W = b + 2, P = W * W;
    const size_t NN = (size_t)N * N;
    const int tiles = a.tiles, t2 = tiles * tiles;
    const int nthr = blockDim.x;
    const AdjLds lay = adjoint_lds_layout(sizeof(T), sizeof(L), b, pk_max, nthr);
    T* tpar = reinterpret_cast<T*>(smem_raw);
    L* lpar = reinterpret_cast<L*>(smem_raw);  // the forward windows are dead once every level is packed
    T* pk = reinterpret_cast<T*>(smem_raw + lay.pk);
    int* offs = reinterpret_cast<int*>(smem_raw + lay.offs);  // packed offset of each forward level
    double* red = reinterpret_cast<double*>(smem_raw);  // after the last lambda level

    // k-time shape of this workgroup (same decode as the forward phases)
    int kx, ky, inst = blockIdx.x;
    if ((a.phase & 1) == 0) {
        kx = ky = a.phase >> 1;
    } else {
        const int w = (a.phase + 1) >> 1;
        const int k = inst >= t2;
        inst -= k * t2;
        kx = k ? w - 1 : w;
        ky = k ? w : w - 1;
    }
    const int jx = inst % tiles, jy = inst / tiles;
    const int fx = 1 - kx, fy = 1 - ky;  // forward shape with the same footprints
    const int C = b / 2 + 1;
    // the k-time tiling is the other one (shift), so its centres equal the forward shape's
    const int cx = jx * b + ((fx & 1) ? 0 : b / 2);
    const int cy = jy * b + ((fy & 1) ? 0 : b / 2);
    const int ox = cx - C, oy = cy - C;
    const bool wraps = ox < 0 || oy < 0 || ox + W > N || oy + W > N;  // window crosses the periodic boundary
    const T r = (T)a.p[0];
    const L rl = (L)r;  // lambda runs the transpose of exactly the forward's (T-rounded) operator

    // ---- forward recompute of levels j = 1..h-1 of shape (fx, fy) ----
    const int flo = 1, fhi = h - 1;
    const LevelEntry* ftab;
    int fkbase;
    if (fx == fy) {
        ftab = a.tab;
        fkbase = fx == 0 ? -h : 0;
    } else {
        ftab = a.tab + (fx > fy ? 2 * h : 3 * h);
        fkbase = 0;
    }
    if (threadIdx.x == 0) {
        int o = 0;
        for (int j = flo; j <= fhi; ++j) {
            offs[j] = o;
            const LevelEntry e = ftab[j - fkbase];
            o += e.fw * e.fh;
        }
    }
    {
        const RingSrc<T> src{reinterpret_cast<const T*>(a.buf0), reinterpret_cast<const T*>(a.buf1),
                             reinterpret_cast<const T*>(a.lvl0), reinterpret_cast<const T*>(a.q0),
                             reinterpret_cast<const T*>(a.q1), fx == 1 && fy == 1};
        preload_rings<HeatS, T>(tpar, P, src, W, P, W, N, NN, ox, oy, fx, fy, flo, fhi, h, C, nthr);
    }
    __syncthreads();
    const T bcv = (T)a.p[1];  // Dirichlet ghost value, rounded as the forward phases round it
    // level entries through the constant address space: scalar loads, which no wait for the
    // level's global stores holds up (see phase_instance)
    const ConstLevelEntry* cftab = (const ConstLevelEntry*)(ftab - fkbase);
    for (int j = flo; j <= fhi; ++j) {
        const LevelEntry e = load_entry(cftab + j);
        if (BC != 0 && wraps)
            heat_level_pack<T, BC>(tpar + ((j - 1) & 1) * P, tpar + (j & 1) * P, pk + offs[j], W, e, r, ox, oy, N,
                                   bcv);
        else
            heat_level_pack<T>(tpar + ((j - 1) & 1) * P, tpar + (j & 1) * P, pk + offs[j], W, e, r);
        __syncthreads();
    }

    // ---- reverse sweep in k-time on the same window ----
    const int kmax = kx > ky ? kx : ky, kmin = kx < ky ? kx : ky;
    const int klo = max(1, (kmax - 1) * h + 1);
    const int khi = min(h, (kmin + 1) * h - 1);
    {
        const RingSrc<L> src{reinterpret_cast<const L*>(a.lam0), reinterpret_cast<const L*>(a.lam1),
                             reinterpret_cast<const L*>(a.lam0), nullptr, nullptr, false};
        preload_rings<HeatS, L>(lpar, P, src, W, P, W, N, NN, ox, oy, kx, ky, klo, khi, h, C, nthr);
    }
    const LevelEntry* ktab;
    int kkbase;
    if (kx == ky) {
        ktab = a.tab;
        kkbase = kx == 0 ? -h : (kx - 1) * h;
    } else {
        ktab = a.tab + (kx > ky ? 2 * h : 3 * h);
        kkbase = (kmax - 1) * h;
    }
    __syncthreads();
    L* l0 = reinterpret_cast<L*>(a.lam0);
    L* l1 = reinterpret_cast<L*>(a.lam1);
    double acc = 0.0;
    const ConstLevelEntry* cktab = (const ConstLevelEntry*)(ktab - kkbase);
    for (int k = klo; k <= khi; ++k) {
        const LevelEntry e = load_entry(cktab + k);
        const bool has2 = k + 2 <= khi;
        const int hx2 = has2 ? e.hx2 : 0, hy2 = has2 ? e.hy2 : 0;
        const int j = h - k;
        L* lprev = lpar + ((k - 1) & 1) * P;
        L* lcur = lpar + (k & 1) * P;
        L* gout = (k & 1) ? l1 : l0;
        const T* tglob = reinterpret_cast<const T*>(a.lvl0);
        if (wraps) {
            if (j >= 1)
                acc += lambda_level<L, T, false, true, BC>(lprev, lcur, gout, pk + offs[j], W, C, e, hx2, hy2, ox, oy,
                                                           N, rl, (double)bcv);
            else
                acc += lambda_level<L, T, true, true, BC>(lprev, lcur, gout, tglob, W, C, e, hx2, hy2, ox, oy, N, rl,
                                                          (double)bcv);
        } else {
            if (j >= 1)
                acc += lambda_level<L, T, false, false>(lprev, lcur, gout, pk + offs[j], W, C, e, hx2, hy2, ox, oy, N,
                                                        rl);
            else
                acc += lambda_level<L, T, true, false>(lprev, lcur, gout, tglob, W, C, e, hx2, hy2, ox, oy, N, rl);
        }
        __syncthreads();
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = tot;
}

// Remainder steps (a run whose length is not a multiple of h): one adjoint
// step per launch over the whole grid, lambda_out = A lambda_in (lambda in
// double), with the pairing against the stored forward level T^m; per-block
// partial sums.
// BC: the wall (0 periodic, 1 Dirichlet with ghost value bcv, 2 zero flux),
// handled as in lambda_level.
template <typename T, int BC>
__global__ void __launch_bounds__(256) adjoint_step_kernel(const double* __restrict__ lin, double* __restrict__ lout,
                                                           const T* __restrict__ Tm, int N, double r, double bcv,
                                                           double* __restrict__ partials)
{
    __shared__ double red[256];
    const size_t NN = (size_t)N * N;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < NN; i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / N), x = (int)(i - (size_t)y * N);
        const size_t row = (size_t)y * N;
        const double c = lin[i];
        const double two_c = c + c;
        double xp = lin[row + wrapi(x + 1, N)], xm = lin[row + wrapi(x - 1, N)];
        double yp = lin[(size_t)wrapi(y + 1, N) * N + x], ym = lin[(size_t)wrapi(y - 1, N) * N + x];
        int nout = 0;
        if constexpr (BC != 0) {
            const double gh = BC == 1 ? 0.0 : c;
            nout = (x == N - 1) + (x == 0) + (y == N - 1) + (y == 0);
            xp = x == N - 1 ? gh : xp;
            xm = x == 0 ? gh : xm;
            yp = y == N - 1 ? gh : yp;
            ym = y == 0 ? gh : ym;
        }
        const double dxx = (xp - two_c) + xm;
        const double dyy = (yp - two_c) + ym;
        lout[i] = (c + r * dxx) + r * dyy;
        acc += (dxx + dyy) * (double)Tm[i];
        if constexpr (BC == 1) acc += bcv * (double)nout * c;
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

size_t adjoint_lds(int dtype, int tile, int pk_max, int wg)
{
    return adjoint_lds_layout(dtype == 0 ? 8 : 4, sizeof(double), tile, pk_max, wg).total;
}

// Lambda is kept in double: the seed dJ/dT^M is widened into it and dJ/dT^0
// narrowed out of it in the state's type.
template <typename T>
__global__ void widen_kernel(const T* __restrict__ x, double* __restrict__ y, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

template <typename T>
__global__ void narrow_kernel(const double* __restrict__ x, T* __restrict__ y, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = (T)x[i];
}

hipError_t launch_lambda_convert(int dtype, const void* src, void* dst, size_t n, bool widen, hipStream_t st)
{
    const dim3 grd(1024), blk(256);
    if (widen) {
        if (dtype == 0) hipLaunchKernelGGL(widen_kernel<double>, grd, blk, 0, st, (const double*)src, (double*)dst, n);
        else hipLaunchKernelGGL(widen_kernel<float>, grd, blk, 0, st, (const float*)src, (double*)dst, n);
    } else {
        if (dtype == 0) hipLaunchKernelGGL(narrow_kernel<double>, grd, blk, 0, st, (const double*)src, (double*)dst, n);
        else hipLaunchKernelGGL(narrow_kernel<float>, grd, blk, 0, st, (const double*)src, (float*)dst, n);
    }
    return hipGetLastError();
}

// The reverse kernel for a tile and wall: fixed-tile copies at b = 16 and 32,
// else the runtime-tile one.
template <typename T, int BC>
static const void* adjoint_kernel_bc(int tile)
{
    if (tile == 32) return (const void*)adjoint_phase_kernel<T, 32, BC>;
    if (tile == 16) return (const void*)adjoint_phase_kernel<T, 16, BC>;
    return (const void*)adjoint_phase_kernel<T, 0, BC>;
}

template <typename T>
static const void* adjoint_kernel(int tile, int bc)
{
    if (bc == 1) return adjoint_kernel_bc<T, 1>(tile);
    if (bc == 2) return adjoint_kernel_bc<T, 2>(tile);
    return adjoint_kernel_bc<T, 0>(tile);
}

hipError_t set_adjoint_lds_limit(int dtype, size_t lds)
{
    hipError_t e = hipSuccess;
    for (int bc = 0; bc < 3; ++bc)
        for (int tile : {0, 16, 32})
            if (e == hipSuccess)
                e = hipFuncSetAttribute(dtype == 0 ? adjoint_kernel<double>(tile, bc) : adjoint_kernel<float>(tile, bc),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return e;
}

hipError_t launch_adjoint_phase(int dtype, const PhaseArgs& a, int pk_max, int wg, size_t lds, hipStream_t st)
{
    const int t2 = a.tiles * a.tiles;
    const int nblk = (a.phase & 1) ? 2 * t2 : t2;
    void* args[] = {(void*)&a, (void*)&pk_max};
    return hipLaunchKernel(dtype == 0 ? adjoint_kernel<double>(a.tile, a.bc) : adjoint_kernel<float>(a.tile, a.bc),
                           dim3(nblk), dim3(wg), args, lds, st);
}

template <typename T, int BC>
static void adjoint_step_launch(const void* lin, void* lout, const void* Tm, int N, double r, double bcv,
                                double* partials, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((adjoint_step_kernel<T, BC>), dim3(nblocks), dim3(256), 0, st, (const double*)lin,
                       (double*)lout, (const T*)Tm, N, r, bcv, partials);
}

hipError_t launch_adjoint_step(int dtype, const void* lin, void* lout, const void* Tm, int N, double r, int bc,
                               double bcv, double* partials, int nblocks, hipStream_t st)
{
    // FP32: the forward ran with r and the ghost value rounded to float; lambda runs the
    // transpose of that operator and pairs with those ghosts
    const double rr = dtype == 0 ? r : (double)(float)r, gv = dtype == 0 ? bcv : (double)(float)bcv;
    if (dtype == 0) {
        if (bc == 1) adjoint_step_launch<double, 1>(lin, lout, Tm, N, rr, gv, partials, nblocks, st);
        else if (bc == 2) adjoint_step_launch<double, 2>(lin, lout, Tm, N, rr, gv, partials, nblocks, st);
        else adjoint_step_launch<double, 0>(lin, lout, Tm, N, rr, gv, partials, nblocks, st);
    } else {
        if (bc == 1) adjoint_step_launch<float, 1>(lin, lout, Tm, N, rr, gv, partials, nblocks, st);
        else if (bc == 2) adjoint_step_launch<float, 2>(lin, lout, Tm, N, rr, gv, partials, nblocks, st);
        else adjoint_step_launch<float, 0>(lin, lout, Tm, N, rr, gv, partials, nblocks, st);
    }
    return hipGetLastError();
}

}  // namespace swept
