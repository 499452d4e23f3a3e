// Descriptors and host-side launchers of the kernels in extras.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trsyl {

constexpr int kNormParts = 512;   // partial sums per norm (fixed reduction order)

// Out = cs * Cin + as * Aop Bop (M x N, K inner), with
//   Aop(m, k) = A[m * sAm + k * sAk],  Bop(k, n) = B[k * sBk + n * sBn],
//   triA: Aop is upper quasi-triangular (entries with k < m - 1 are zero and never read),
//   triB: Bop is upper quasi-triangular (entries with k > n + 1 are zero and never read),
//   as = asign 2^(ae0 + ae1 *ep1 + ae2 *ep2),  cs likewise (Cin may be null),
//   the A operand's values are staged times 2^(sa1 *ep1), the B operand's times 2^(sb1 *ep1)
//   (exact power-of-two normalisation that keeps the products in range),
//   mask: zero every output entry outside the quasi-triangular pattern of the square matrix
//         pat (keep i <= j, and i == j + 1 where pat(j+1, j) != 0).
// Cin may equal Out (each entry is read and then written by the same thread).
struct GemmDesc {
    int M, N, K;
    const double *A;
    int64_t sAm, sAk;
    int triA;
    const double *B;
    int64_t sBk, sBn;
    int triB;
    const double *Cin;
    int64_t ldcin;
    double *Out;
    int64_t ldo;
    int sa1, sb1;
    double asign;
    int ae0, ae1, ae2;
    double csign;
    int ce0, ce1, ce2;
    const int64_t *ep1, *ep2;
    int mask;
    const double *pat;
    int64_t ldpat;
    const int32_t *skip;     // optional: when *skip != 0 the kernel does nothing
};

hipError_t launch_quasi_copy(const double *T, int64_t ldt, int n, bool flip, double sign, double *D,
                             hipStream_t s);
hipError_t launch_flip_transpose(const double *A, int64_t lda, int n, double *Ah, hipStream_t s);
hipError_t launch_flip_axes(double *W, int64_t ldw, int m, int n, bool rows, bool cols, hipStream_t s);
hipError_t launch_flip(double *W, int64_t ldw, int m, int n, hipStream_t s);
hipError_t launch_gemm(const GemmDesc &g, hipStream_t s);
hipError_t launch_scale_copy(const double *G, int64_t ldg_, int m, int n, const int64_t *eG,
                             const int64_t *eY, double *dC, int64_t lddc, hipStream_t s);
hipError_t launch_norm(const double *X, int64_t ld, int rows, int cols, int pattern, double *part,
                       int32_t *s, double *t, hipStream_t st, const int32_t *skip = nullptr);
hipError_t launch_neg_exp(const int32_t *s, int64_t *out, hipStream_t st, const int32_t *skip = nullptr);
hipError_t launch_norm_shift(const int32_t *s, const double *t, int64_t *negshift, int64_t *total,
                             hipStream_t st);
hipError_t launch_add_exponent(int64_t *e, double *scale, const int64_t *add, hipStream_t st);
hipError_t launch_residual_final(const int32_t *s5, const double *t5, const int64_t *e, double *out,
                                 hipStream_t st);

hipError_t launch_refine_update(double *Y, int64_t ldy, const double *D, int64_t ldd, int m, int n,
                                const int64_t *eD, const int64_t *negsy, const int32_t *sD, int64_t *e,
                                int32_t *info, const int32_t *infoD, double *scale, hipStream_t st,
                                const int32_t *skip = nullptr, uint32_t *sweeps = nullptr);
hipError_t launch_absmax_exp(const double *X, int64_t ld, int rows, int cols, double *part, int32_t *s,
                             hipStream_t st, const int32_t *skip = nullptr);
// Convergence test of the precision form's sweeps: eq. (9) of the current iterate from the five
// norm pairs (as for trsyl_residual: R' of the scaled iterate, A, B, Ys, C); when it is at most
// tol, *skip is set (and stays set), which turns every later kernel of the refinement into a
// no-op.
hipError_t launch_refine_check(const int32_t *s5, const double *t5, const int64_t *e, double tol, int32_t *skip,
                               hipStream_t st);

}  // namespace trsyl
