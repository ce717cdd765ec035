// Stand-ins for the kernel launchers (kernels.hip, adjoint.hip, batch.hip), so
// that the host validation of the C ABI (capi.cpp, hetero.cpp) can be built
// with the host sanitizers without the device code.  Every launcher reports
// hipErrorNotSupported; the validation paths the driver runs never reach one.
// euler_phase_lds is the real size rule (validation uses it).
#include "../../paper_2105_10332_amd/csrc/device_common.h"

namespace swept {
hipError_t launch_phase(int, int, const PhaseArgs&, int, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t set_phase_lds_limit(int, int, size_t) { return hipErrorNotSupported; }
hipError_t launch_heat_standard(int, const void*, void*, int, double, int, double, hipStream_t)
{
    return hipErrorNotSupported;
}
size_t euler_standard_lds(int dtype, int ts) { return (dtype == 0 ? 8 : 4) * euler_lds_values(ts + 8); }
size_t euler_phase_lds(int dtype, int tile) { return (dtype == 0 ? 8 : 4) * euler_lds_values(tile + 4); }
hipError_t set_euler_standard_lds_limit(int, size_t) { return hipErrorNotSupported; }
hipError_t launch_euler_standard(int, const void*, void*, const StdArgs&, hipStream_t) { return hipErrorNotSupported; }
size_t adjoint_lds(int, int, int, int) { return 0; }
hipError_t set_adjoint_lds_limit(int, size_t) { return hipErrorNotSupported; }
hipError_t launch_adjoint_phase(int, const PhaseArgs&, int, int, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_adjoint_step(int, const void*, void*, const void*, int, double, int, double, double*, int,
                               hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t launch_lambda_convert(int, const void*, void*, size_t, bool, hipStream_t) { return hipErrorNotSupported; }
hipError_t batch_occupancy(int, size_t, int*) { return hipErrorNotSupported; }
hipError_t set_batch_lds_limit(int, size_t) { return hipErrorNotSupported; }
hipError_t launch_batch(int, const PhaseArgs*, int, int, long long, int, size_t, hipStream_t, int*)
{
    return hipErrorNotSupported;
}
hipError_t launch_batch_phase(int, const PhaseArgs*, int, int, long long, int, size_t, hipStream_t, int*)
{
    return hipErrorNotSupported;
}
hipError_t launch_combine(const double*, int, double*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_plane_sums(int, const void*, int, size_t, double*, int, double*, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t noalloc_scratch(double**) { return hipErrorNotSupported; }
hipError_t launch_cfl_max(int, const void*, size_t, double, double, double, double*, int, double*, hipStream_t)
{
    return hipErrorNotSupported;
}
}  // namespace swept
