// launch.h -- internal interface between the C ABI (capi.cpp) and the
// kernels (kernels.hip).  Not installed; the public interface is swept.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace swept {

// Per-level launch geometry of one shape type, precomputed on the host
// (uniform across a workgroup, read with scalar loads).  Footprint
// [x0, x0+fw) x [y0, y0+fh) in window coordinates; hx2/hy2 = half-widths of
// the footprint two levels up (0 past the shape's end); inv_fw = 1.0f/fw for
// the exact float quotient of the flattened cell loop.  Heat maps threads
// onto column pairs: pw = fw/2 pairs per row, each thread walks a vertical
// strip of R rows of one pair, spc = strips per pair column, inv_pw = 1/pw.
// Heat LDS row pitch = window width + kHeatPad values.
constexpr int kHeatPad = 1;

struct LevelEntry {
    int x0, y0, fw, fh, hx2, hy2, pw, R, spc;
    float inv_fw, inv_pw;
    int pad[5];
};

// Level table layout (entries indexed by t, the level within the shape's
// window): Octahedron t = 1..2h-1 at [t] (the Up-Pyramid is its upper half,
// t = l + h); X-Bridge (w, w-1) t = 1..h-1 at [2h + t]; Y-Bridge at [3h + t].
inline int level_table_entries(int h) { return 4 * h; }

// Arguments of one swept phase launch.  p[] holds the scheme constants in
// double: heat {r, Dirichlet ghost value}; Euler {gamma, dt/(2dx), dt/(2dy),
// dt/dx, dt/dy}.
struct PhaseArgs {
    void* buf0;   // level-parity buffer 0 (the caller's state): read and written
    void* buf1;   // level-parity buffer 1 (workspace): read and written
    void* out0;   // where stores go (normally buf0/buf1; the adjoint's Bridges recompute writes elsewhere)
    void* out1;
    const void* lvl0;  // level-0 state (normally buf0)
    const void* q0;    // adjoint only: the Bridges' strips, read by the first Octahedron of a taped cycle
    const void* q1;
    void* lam0;        // adjoint only: lambda level-parity buffers (reversed time)
    void* lam1;
    double* partials;  // adjoint only: one pairing partial sum per workgroup
    int shift;         // adjoint only: 1 = the reversed sweep runs on the other tiling
    int kind;          // batch only: 0 heat, 1 Euler (single-problem launches pick the kernel by template)
    int scheme;        // Euler scheme variant bits (scheme.h); picks the kernel instantiation, 0 for heat
    int bc;            // heat boundary (SWEPT_BC_*); the Dirichlet ghost value is p[1]
    int N;        // cells per side
    int tile;     // b
    int h;        // b / (2n)
    int tiles;    // N / b
    int L;        // final level of this advance
    int phase;    // 0 .. 2*ceil(L/h)
    int jrows;    // heterogeneous advance: only the instances of tile rows jy < jrows (0: all)
    const LevelEntry* tab;  // level table (device memory, see above)
    double p[5];
};

struct StdArgs {
    int N;
    int ts;      // output tile edge of the fused Euler step
    int scheme;  // Euler scheme variant bits (scheme.h)
    int bc;      // Euler walls: 0 periodic, 2 zero gradient, 3 slip
    double p[5];
};

hipError_t launch_phase(int kind, int dtype, const PhaseArgs& a, int wg, size_t lds, hipStream_t st);
hipError_t set_phase_lds_limit(int kind, int dtype, size_t lds);
hipError_t launch_heat_standard(int dtype, const void* in, void* out, int N, double r, int bc, double bcv,
                                hipStream_t st);
size_t euler_standard_lds(int dtype, int ts);
size_t euler_phase_lds(int dtype, int tile);  // LDS bytes of an Euler swept workgroup
hipError_t set_euler_standard_lds_limit(int dtype, size_t lds);
hipError_t launch_euler_standard(int dtype, const void* in, void* out, const StdArgs& a, hipStream_t st);
size_t adjoint_lds(int dtype, int tile, int pk_max, int wg);
hipError_t set_adjoint_lds_limit(int dtype, size_t lds);
hipError_t launch_adjoint_phase(int dtype, const PhaseArgs& a, int pk_max, int wg, size_t lds, hipStream_t st);
hipError_t launch_adjoint_step(int dtype, const void* lin, void* lout, const void* Tm, int N, double r, int bc,
                               double bcv, double* partials, int nblocks, hipStream_t st);
// lambda (double) from/to the state's type: widen = true copies a state-typed
// field into double, false the reverse.
hipError_t launch_lambda_convert(int dtype, const void* src, void* dst, size_t n, bool widen, hipStream_t st);
// Batched persistent launch: every problem's phases in one cooperative
// kernel, global phase g running phase g of every problem that has one.
constexpr int kBatchMax = 256;
// Threads per batch workgroup: the Euler phase bound of the precision (heat
// takes any size), 512 in FP32 and 256 in FP64.
constexpr int batch_wg(int dtype) { return dtype == 0 ? 256 : 512; }
constexpr size_t kBatchStaticLds = 2048;  // >= sizeof(int) * (kBatchMax + 1), the kernel's static array
hipError_t batch_occupancy(int dtype, size_t lds, int* blocks_per_cu);
hipError_t set_batch_lds_limit(int dtype, size_t lds);
hipError_t launch_batch(int dtype, const PhaseArgs* d_args, int count, int nphase_max, long long n_steps, int grid,
                        size_t lds, hipStream_t st, int* ctr);
// Global phase gp alone, as an ordinary launch (the batch's one-launch-per-phase mode).
hipError_t launch_batch_phase(int dtype, const PhaseArgs* d_args, int count, int gp, long long n_steps, int grid,
                              size_t lds, hipStream_t st, int* ctr);
hipError_t launch_combine(const double* partials, int nparts, double* out, hipStream_t st);
hipError_t launch_plane_sums(int dtype, const void* x, int nvar, size_t NN, double* partials, int nparts,
                             double* out, hipStream_t st);
// Scratch of the allocation-free CFL entry point: kNoAllocParts partial maxima
// and one result, in a file-scope device array; *out = its address on the
// current device (looked up once per device).
constexpr int kNoAllocParts = 1024;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch(double** out);
hipError_t launch_cfl_max(int dtype, const void* q, size_t NN, double gamma, double dx, double dy, double* partials,
                          int nparts, double* out, hipStream_t st);

}  // namespace swept
