// batch.hip -- many swept problems of uneven size in one persistent launch.
//
// The grid is sized to what the GPU holds resident (cooperative launch), and
// every workgroup walks global phases g = 0, 1, ...: in phase g it takes the
// shape instances of phase g of every problem that has one (each problem has
// 1 + 2 ceil(L/h) phases for its own tile and level count) -- grid-stride in
// phase 0, then one at a time from a per-phase atomic counter, so faster
// workgroups take more of the uneven instances -- runs each exactly like the
// single-problem phase kernel, and then waits at a grid barrier.  Problems are
// independent, so one barrier per global phase is the only synchronisation;
// heat and Euler instances share the launch.  The two counters alternate
// between phases: workgroup 0 clears the next phase's counter while the
// current phase runs (nobody touches it then), and the grid barrier
// publishes the clear.
#include <algorithm>

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace swept {

namespace cg = cooperative_groups;

__device__ __forceinline__ int problem_phases(const PhaseArgs& a, long long n_steps)
{
    const long long L = n_steps * (a.kind == 0 ? 1 : 2);
    return L > 0 ? 2 * (int)((L + a.h - 1) / a.h) + 1 : 0;
}

// One shape instance of problem a: the kernel variant its kind, wall and
// scheme bits select (the same device function as the single-problem kernels).
template <typename T>
__device__ __forceinline__ void instance(const PhaseArgs& a, int blk, unsigned char* smem_raw)
{
    if (a.kind == 0) {
        if (a.bc == 1) phase_instance<HeatSV<1>, T>(a, blk, smem_raw);
        else if (a.bc == 2) phase_instance<HeatSV<2>, T>(a, blk, smem_raw);
        else phase_instance<HeatS, T>(a, blk, smem_raw);
    } else {
        switch (a.scheme) {
            case 1: phase_instance<EulerSV<1>, T>(a, blk, smem_raw); break;
            case 2: phase_instance<EulerSV<2>, T>(a, blk, smem_raw); break;
            case 3: phase_instance<EulerSV<3>, T>(a, blk, smem_raw); break;
            default: phase_instance<EulerS, T>(a, blk, smem_raw);
        }
    }
}

// Global phase gp of the batch, run by every workgroup of the grid: the items
// of the phase problem by problem (prefix in pre), then the instances.
template <typename T>
__device__ __forceinline__ void batch_phase(const PhaseArgs* __restrict__ probs, int count, int gp, long long n_steps,
                                            int* ctr, int* pre, int* s_it, unsigned char* smem_raw)
{
    if (threadIdx.x == 0) {  // items of this global phase, problem by problem
        int tot = 0;
        for (int q = 0; q < count; ++q) {
            pre[q] = tot;
            const PhaseArgs& a = probs[q];
            const int t2 = a.tiles * a.tiles;
            if (gp < problem_phases(a, n_steps)) tot += (gp & 1) ? 2 * t2 : t2;
        }
        pre[count] = tot;
        if (blockIdx.x == 0) ctr[(gp + 1) & 1] = 0;  // the next phase's counter is idle during this one
    }
    __syncthreads();
    const int total = pre[count];
    for (int k = 0;; ++k) {
        int it;
        if (gp == 0) {
            it = blockIdx.x + k * gridDim.x;
        } else {
            if (threadIdx.x == 0) *s_it = atomicAdd(&ctr[gp & 1], 1);
            __syncthreads();
            it = *s_it;
        }
        it = __builtin_amdgcn_readfirstlane(it);  // uniform: the instance's arguments come in as scalars
        if (it >= total) break;
        int lo = 0, hi = count;  // largest q with pre[q] <= it
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= it) lo = mid;
            else hi = mid;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        // the problem's arguments through the constant address space, word by word: scalar loads,
        // so neither they nor the level table they point to wait behind the level's global stores
        PhaseArgs a;
        {
            static_assert(sizeof(PhaseArgs) % 4 == 0, "copied in 32-bit words");
            const __attribute__((address_space(4))) unsigned* src =
                (const __attribute__((address_space(4))) unsigned*)(probs + lo);
            unsigned* dst = reinterpret_cast<unsigned*>(&a);
#pragma unroll
            for (int w = 0; w < (int)(sizeof(PhaseArgs) / 4); ++w) dst[w] = src[w];
        }
        a.phase = gp;
        a.L = (int)(n_steps * (a.kind == 0 ? 1 : 2));
        instance<T>(a, it - pre[lo], smem_raw);
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(batch_wg(sizeof(T) == 8 ? 0 : 1))
    batch_kernel(const PhaseArgs* __restrict__ probs, int count, int nphase_max, long long n_steps, int* ctr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int pre[kBatchMax + 1];
    __shared__ int s_it;
    cg::grid_group grid = cg::this_grid();
    for (int gp = 0; gp < nphase_max; ++gp) {
        batch_phase<T>(probs, count, gp, n_steps, ctr, pre, &s_it, smem_raw);
        grid.sync();
    }
}

// One global phase per launch: the same work with stream order in place of the
// grid barrier, for processes that cannot make cooperative launches.  The
// second bound (waves per SIMD) keeps two workgroups per compute unit: left
// free, the compiler gives this kernel half again the registers of the
// cooperative one and one workgroup per CU.
template <typename T>
__global__ void __launch_bounds__(batch_wg(sizeof(T) == 8 ? 0 : 1), batch_wg(sizeof(T) == 8 ? 0 : 1) / 128)
    batch_phase_kernel(const PhaseArgs* __restrict__ probs, int count, int gp, long long n_steps, int* ctr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int pre[kBatchMax + 1];
    __shared__ int s_it;
    batch_phase<T>(probs, count, gp, n_steps, ctr, pre, &s_it, smem_raw);
}

hipError_t batch_occupancy(int dtype, size_t lds, int* blocks_per_cu)
{
    const void* f = dtype == 0 ? (const void*)batch_kernel<double> : (const void*)batch_kernel<float>;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, batch_wg(dtype), lds);
}

hipError_t set_batch_lds_limit(int dtype, size_t lds)
{
    const void* f = dtype == 0 ? (const void*)batch_kernel<double> : (const void*)batch_kernel<float>;
    const void* g = dtype == 0 ? (const void*)batch_phase_kernel<double> : (const void*)batch_phase_kernel<float>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return e;
}

hipError_t launch_batch(int dtype, const PhaseArgs* d_args, int count, int nphase_max, long long n_steps, int grid,
                        size_t lds, hipStream_t st, int* ctr)
{
    void* args[] = {(void*)&d_args, (void*)&count, (void*)&nphase_max, (void*)&n_steps, (void*)&ctr};
    const void* f = dtype == 0 ? (const void*)batch_kernel<double> : (const void*)batch_kernel<float>;
    return hipLaunchCooperativeKernel(f, dim3(grid), dim3(batch_wg(dtype)), args, (unsigned int)lds, st);
}

hipError_t launch_batch_phase(int dtype, const PhaseArgs* d_args, int count, int gp, long long n_steps, int grid,
                              size_t lds, hipStream_t st, int* ctr)
{
    // at most the workgroups this kernel keeps resident (grid is the cooperative kernel's);
    // any grid covers the phase: grid-stride in phase 0, the counter after it
    const void* f = dtype == 0 ? (const void*)batch_phase_kernel<double> : (const void*)batch_phase_kernel<float>;
    int bpc = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, f, batch_wg(dtype), lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (bpc < 1) return hipErrorInvalidConfiguration;
    grid = std::min(grid, bpc * cus);
    if (dtype == 0)
        hipLaunchKernelGGL(batch_phase_kernel<double>, dim3(grid), dim3(batch_wg(dtype)), lds, st, d_args, count, gp,
                           n_steps, ctr);
    else
        hipLaunchKernelGGL(batch_phase_kernel<float>, dim3(grid), dim3(batch_wg(dtype)), lds, st, d_args, count, gp,
                           n_steps, ctr);
    return hipGetLastError();
}

}  // namespace swept
