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

// trsyl_robust_noalloc's core (capi.cpp) and its size error.
constexpr int kNoAllocTooLarge = -201;
}  // namespace trsyl
#include "../../include/trsyl.h"
namespace trsyl {
int noalloc_need(int64_t m, int64_t n, const trsyl_opts *opts, size_t *need);
int noalloc_solve(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                  int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info, const trsyl_opts *opts,
                  char *ws, size_t cap, hipStream_t stream);
int check_solve_args(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                     const double *C, int64_t ldc, const int64_t *scale_log2, const int32_t *info);

}  // namespace trsyl
