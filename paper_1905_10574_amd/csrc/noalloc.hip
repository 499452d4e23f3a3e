// trsyl_robust_noalloc (include/trsyl.h): the robust solve for callers that cannot allocate.
//
// The solver state lives in `scratch`, a file-scope device array of TRSYL_NOALLOC_BYTES.  Each GPU
// the library runs on holds its own copy until the process ends.  In host code the array's name
// is a host-side stand-in, not a device address: the device address is taken once per device, with
// that device current, by hipGetSymbolAddress, and only that address is handed to the kernels and
// the fill kernel that clears the state.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/trsyl.h"
#include "launch.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[TRSYL_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// The device address of the current device's `scratch`, or nullptr on a HIP error.
void *scratch_address(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int trsyl_robust_noalloc(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                                    int64_t ldb, double *C, int64_t ldc, int64_t *scale_log2, double *scale,
                                    int32_t *info, const trsyl_opts *opts, trsyl_stream_t stream)
{
    if (int e = trsyl::check_solve_args(m, n, A, lda, B, ldb, C, ldc, scale_log2, info)) return e;
    size_t need = 0;
    if (int e = trsyl::noalloc_need(m, n, opts, &need)) return e;
    if (need > (size_t)TRSYL_NOALLOC_BYTES) return TRSYL_ENOSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -100;
    void *ws = scratch_address(dev);
    if (!ws) return -100;
    return trsyl::noalloc_solve(m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, opts, (char *)ws,
                                (size_t)TRSYL_NOALLOC_BYTES, (hipStream_t)stream);
}
