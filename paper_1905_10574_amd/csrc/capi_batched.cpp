// Batched entry point of include/trsyl.h (filled in by the batched driver).
#include <hip/hip_runtime.h>

#include "../../include/trsyl.h"

extern "C" {

size_t trsyl_batched_workspace_size(int32_t, const int64_t *, const int64_t *, const trsyl_opts *) { return 0; }
int trsyl_robust_batched(int32_t, const int64_t *, const int64_t *, const double *const *, const int64_t *,
                         const double *const *, const int64_t *, double *const *, const int64_t *,
                         int64_t *, double *, int32_t *, const trsyl_opts *, void *, size_t, trsyl_stream_t)
{
    return -100;
}

}  // extern "C"
