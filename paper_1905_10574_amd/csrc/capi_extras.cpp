// Entry points of include/trsyl.h that are not the forward FP64 solve.  Filled in as the
// corresponding drivers land; until then they report "not available" (-100).
#include <hip/hip_runtime.h>

#include "../../include/trsyl.h"

extern "C" {

size_t trsyl_adjoint_workspace_size(int64_t, int64_t, const trsyl_opts *) { return 0; }
int trsyl_robust_adjoint(int64_t, int64_t, const double *, int64_t, const double *, int64_t, double *,
                         int64_t, int64_t *, double *, int32_t *, const trsyl_opts *, void *, size_t,
                         trsyl_stream_t)
{
    return -100;
}
int trsyl_grad(int64_t, int64_t, const double *, int64_t, const double *, int64_t, const double *,
               int64_t, const int64_t *, const double *, int64_t, const int64_t *, double *, int64_t,
               double *, int64_t, double *, int64_t, trsyl_stream_t)
{
    return -100;
}
size_t trsyl_batched_workspace_size(int32_t, const int64_t *, const int64_t *, const trsyl_opts *) { return 0; }
int trsyl_robust_batched(int32_t, const int64_t *, const int64_t *, const double *const *, const int64_t *,
                         const double *const *, const int64_t *, double *const *, const int64_t *,
                         int64_t *, double *, int32_t *, const trsyl_opts *, void *, size_t, trsyl_stream_t)
{
    return -100;
}
size_t trsyl_residual_workspace_size(int64_t, int64_t) { return 0; }
int trsyl_residual(int64_t, int64_t, const double *, int64_t, const double *, int64_t, const double *,
                   int64_t, const int64_t *, const double *, int64_t, double *, void *, size_t,
                   trsyl_stream_t)
{
    return -100;
}

}  // extern "C"
