// launch.h -- internal interface between the C ABI (capi.cpp) and the
// kernels (kernels.hip).  Not installed; the public interface is swept.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace swept {

// Per-level launch geometry of one shape type, precomputed on the host
// (uniform across a workgroup, read with scalar loads).  Footprint
// [x0, x0+fw) x [y0, y0+fh) in window coordinates; hx2/hy2 = half-widths of
// the footprint two levels up (0 past the shape's end); R = cells per thread
// strip and spc = strips per column for the heat strip mapping; inv_fw =
// 1.0f/fw for the exact float quotient.
struct LevelEntry {
    int x0, y0, fw, fh, R, spc, hx2, hy2;
    float inv_fw;
    int pad[3];
};

// Level table layout (entries indexed by t, the level within the shape's
// window): Octahedron t = 1..2h-1 at [t] (the Up-Pyramid is its upper half,
// t = l + h); X-Bridge (w, w-1) t = 1..h-1 at [2h + t]; Y-Bridge at [3h + t].
inline int level_table_entries(int h) { return 4 * h; }

// Arguments of one swept phase launch.  p[] holds the scheme constants in
// double: heat {r}; Euler {gamma, dt/(2dx), dt/(2dy), dt/dx, dt/dy}.
struct PhaseArgs {
    void* buf0;   // level-parity buffer 0 (the caller's state)
    void* buf1;   // level-parity buffer 1 (workspace)
    int N;        // cells per side
    int tile;     // b
    int h;        // b / (2n)
    int tiles;    // N / b
    int L;        // final level of this advance
    int phase;    // 0 .. 2*ceil(L/h)
    const LevelEntry* tab;  // level table (device memory, see above)
    double p[5];
};

struct StdArgs {
    int N;
    int ts;  // output tile edge of the fused Euler step
    double p[5];
};

hipError_t launch_phase(int kind, int dtype, const PhaseArgs& a, int wg, size_t lds, hipStream_t st);
hipError_t set_phase_lds_limit(int kind, int dtype, size_t lds);
hipError_t launch_heat_standard(int dtype, const void* in, void* out, int N, double r, hipStream_t st);
size_t euler_standard_lds(int dtype, int ts);
hipError_t set_euler_standard_lds_limit(int dtype, size_t lds);
hipError_t launch_euler_standard(int dtype, const void* in, void* out, const StdArgs& a, hipStream_t st);
hipError_t launch_plane_sums(int dtype, const void* x, int nvar, size_t NN, double* partials, int nparts,
                             double* out, hipStream_t st);
hipError_t launch_cfl_max(int dtype, const void* q, size_t NN, double gamma, double dx, double dy, double* partials,
                          int nparts, double* out, hipStream_t st);

}  // namespace swept
