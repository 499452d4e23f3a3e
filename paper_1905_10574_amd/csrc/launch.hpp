// Host-side launchers of the solver kernels (solver.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace trsyl {

hipError_t launch_setup(const Plan &P, hipStream_t s);
hipError_t launch_dag(const Plan &P, int workers, hipStream_t s);
hipError_t launch_fronts(const Plan &P, hipStream_t s);
hipError_t launch_finalize(const Plan &P, hipStream_t s);
hipError_t launch_debug_protect(int which, int count, const double *in, int32_t *out, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace trsyl
