// hetero.h -- internal interface of the heterogeneous advance (hetero.cpp):
// the shape instances of every phase are split between the GPU and the host
// cores by tile rows (the GPU share of Eq. 2).  Not installed; the public
// interface is swept.h.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "launch.h"

namespace swept {

struct HeteroSetup {
    int kind, dtype, scheme;  // periodic problems only
    int N, b, h, tiles, nvar, lps, wg;
    size_t lds, state_bytes;
    std::vector<LevelEntry> tab;  // host copy of the level table
    PhaseArgs base;               // the context's phase arguments (device buffers and level table)
    void* d0;                     // level-parity buffer 0 (the caller's state)
    void* d1;                     // level-parity buffer 1 (workspace)
    hipStream_t stream;
    int gpu_rows;  // tile rows 0 .. gpu_rows-1 run on the GPU, the rest on the host cores
    int threads;   // host worker threads
};

struct Hetero;

// hipSuccess, or the HIP error of a failed host allocation or copy.  On any
// error *out is left null and nothing is held.
hipError_t hetero_create(const HeteroSetup& s, Hetero** out);
// n_steps with the split on `stream`; synchronous (the host takes part).
hipError_t hetero_advance(Hetero* h, long long n_steps, hipStream_t stream);
void hetero_destroy(Hetero* h);
// Bytes of pinned host memory the runner holds.
size_t hetero_host_bytes(const Hetero* h);

}  // namespace swept
