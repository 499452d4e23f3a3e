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

// Device-side tables of a batched solve (all inside the caller's workspace).
struct BatchedLaunch {
    int count;
    const Plan *plans;                 // [count]
    const int32_t *off_structure;      // [count + 1] block offsets per stage
    const int32_t *off_A, *off_B, *off_C, *off_consistency;
    int blocks_structure, blocks_bounds, blocks_consistency;
    const uint64_t *tasks;             // merged task list
    const uint32_t *tprob;             // problem of each task
    int64_t ntasks;
    uint32_t *ticket;
    double *scratch;                   // [workers][kMaxTile * kMaxTile]
    int workers;
};
hipError_t launch_batched(const BatchedLaunch &b, hipStream_t s);

}  // namespace trsyl
