// Host-only stand-ins for the device entry points of kernels.hip, linked
// into the sanitizer builds of the library's host code (runtime, autotuner,
// server), which the CPU tests exercise without a GPU: validation, sizes,
// layouts and the collision-plan walk, and the server's scheduler on a
// caller's executor. Every launch reports that no device is there.
#include "mhc_internal.h"

namespace mhc {

hipError_t launch_trajgen(const Launch &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_collide(const Launch &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_risk(const Launch &, hipStream_t) { return hipErrorNoDevice; }
int collide_blocks_per_cu(int, int, bool, bool) { return 1; }
hipError_t noalloc_scratch_address(int, char **out)
{
    *out = nullptr;
    return hipErrorNoDevice;
}

}  // namespace mhc
