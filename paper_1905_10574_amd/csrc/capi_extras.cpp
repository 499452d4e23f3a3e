// Entry points of include/trsyl.h beside the forward, precision-form and batched solves (those
// are in capi.cpp): the adjoint, general-form and Bartels-Stewart solves, the gradient products
// and the eq. (9) residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/trsyl.h"
#include "extras.hpp"
#include "launch.hpp"

using namespace trsyl;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
bool bad_ptr(const void *p) { return p == nullptr; }

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------------------------
// Adjoint: A^T G + G B^T = alpha W.  With P, Q the order reversals, Ah = P A^T P and Bh = Q B^T Q
// are upper quasi-triangular, and Gh = P G Q solves Ah Gh + Gh Bh = alpha P W Q; W is flipped in
// place, solved by the forward driver, and flipped back.  Workspace: the forward workspace, then
// Ah (m x m) and Bh (n x n).
// ---------------------------------------------------------------------------------------------
size_t trsyl_adjoint_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts)
{
    const size_t fw = trsyl_workspace_size(m, n, opts);
    if (fw == 0) return 0;
    return align_up(fw) + align_up(8 * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(m, 1)) +
           align_up(8 * (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(n, 1));
}

int trsyl_robust_adjoint(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                         int64_t ldb, double *W, int64_t ldw, int64_t *scale_log2, double *scale,
                         int32_t *info, const trsyl_opts *opts, void *workspace, size_t ws_bytes,
                         trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && bad_ptr(A)) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (n > 0 && bad_ptr(B)) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (m > 0 && n > 0 && bad_ptr(W)) return -7;
    if (ldw < std::max<int64_t>(1, m)) return -8;
    if (bad_ptr(scale_log2)) return -9;
    if (bad_ptr(info)) return -11;
    const size_t fw = trsyl_workspace_size(m, n, opts);
    if (fw == 0) return -12;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -13;
    if (ws_bytes < trsyl_adjoint_workspace_size(m, n, opts)) return -14;
    if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return -1;
    char *ws = (char *)workspace;
    double *Ah = (double *)(ws + align_up(fw));
    double *Bh = (double *)(ws + align_up(fw) + align_up(8 * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(m, 1)));
    const int mi = (int)m, ni = (int)n;
    if (m > 0 && n > 0) {
        if (launch_flip_transpose(A, lda, mi, Ah, stream) != hipSuccess) return -100;
        if (launch_flip_transpose(B, ldb, ni, Bh, stream) != hipSuccess) return -100;
        if (launch_flip(W, ldw, mi, ni, stream) != hipSuccess) return -100;
    }
    const int rc = trsyl_robust(m, n, Ah, std::max<int64_t>(1, m), Bh, std::max<int64_t>(1, n), W, ldw,
                                scale_log2, scale, info, opts, workspace, fw, stream_);
    if (rc != 0) return rc == -100 ? -100 : -12;
    if (m > 0 && n > 0 && launch_flip(W, ldw, mi, ni, stream) != hipSuccess) return -100;
    return 0;
}

// ---------------------------------------------------------------------------------------------
// Host read-back of a solve's results: waits for the stream, then copies e, alpha and the status
// from device memory.
// ---------------------------------------------------------------------------------------------
int trsyl_sync_result(const int64_t *scale_log2, const double *scale, const int32_t *info,
                      int64_t *e_host, double *scale_host, int32_t *info_host, trsyl_stream_t stream_)
{
    if (bad_ptr(scale_log2)) return -1;
    if (bad_ptr(info)) return -3;
    if (bad_ptr(e_host)) return -4;
    if (bad_ptr(info_host)) return -6;
    if (scale_host && bad_ptr(scale)) return -2;
    hipStream_t stream = (hipStream_t)stream_;
    if (hipStreamSynchronize(stream) != hipSuccess) return -100;
    if (hipMemcpy(e_host, scale_log2, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) return -100;
    if (hipMemcpy(info_host, info, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return -100;
    if (scale_host && hipMemcpy(scale_host, scale, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return -100;
    return 0;
}

// ---------------------------------------------------------------------------------------------
// General form op(A) Y + isgn Y op(B) = alpha C.  A transposed A is reversed as in the adjoint
// (Ah = P A^T P, rows of C reversed), a transposed B likewise (Bh = Q B^T Q, columns of C
// reversed), and isgn = -1 negates the B operand; the forward driver solves
// Ah Yh + Yh (isgn Bh) = alpha Ch and the reversals are undone on the result.  A and B are read
// in place when they need neither.  Workspace: the forward workspace, then Ah (m x m), Bh (n x n).
// ---------------------------------------------------------------------------------------------
static int trans_code(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

size_t trsyl_general_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts)
{
    return trsyl_adjoint_workspace_size(m, n, opts);
}

int trsyl_robust_general(char trana, char tranb, int32_t isgn, int64_t m, int64_t n, const double *A,
                         int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                         int64_t *scale_log2, double *scale, int32_t *info, const trsyl_opts *opts,
                         void *workspace, size_t ws_bytes, trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    const int ta = trans_code(trana), tb = trans_code(tranb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (isgn != 1 && isgn != -1) return -3;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (m > 0 && bad_ptr(A)) return -6;
    if (lda < std::max<int64_t>(1, m)) return -7;
    if (n > 0 && bad_ptr(B)) return -8;
    if (ldb < std::max<int64_t>(1, n)) return -9;
    if (m > 0 && n > 0 && bad_ptr(C)) return -10;
    if (ldc < std::max<int64_t>(1, m)) return -11;
    if (bad_ptr(scale_log2)) return -12;
    if (bad_ptr(info)) return -14;
    const size_t fw = trsyl_workspace_size(m, n, opts);
    if (fw == 0) return -15;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -16;
    if (ws_bytes < trsyl_general_workspace_size(m, n, opts)) return -17;
    if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return -4;
    char *ws = (char *)workspace;
    double *Ah = (double *)(ws + align_up(fw));
    double *Bh = (double *)(ws + align_up(fw) + align_up(8 * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(m, 1)));
    const int mi = (int)m, ni = (int)n;
    const bool work = m > 0 && n > 0;
    const double *Au = A, *Bu = B;
    int64_t ldau = lda, ldbu = ldb;
    if (work && ta) {
        if (launch_quasi_copy(A, lda, mi, true, 1.0, Ah, stream) != hipSuccess) return -100;
        Au = Ah;
        ldau = m;
    }
    if (work && (tb || isgn < 0)) {
        if (launch_quasi_copy(B, ldb, ni, tb != 0, (double)isgn, Bh, stream) != hipSuccess) return -100;
        Bu = Bh;
        ldbu = n;
    }
    if (work && launch_flip_axes(C, ldc, mi, ni, ta != 0, tb != 0, stream) != hipSuccess) return -100;
    const int rc = trsyl_robust(m, n, Au, ldau, Bu, ldbu, C, ldc, scale_log2, scale, info, opts,
                                workspace, fw, stream_);
    if (rc != 0) return rc == -100 ? -100 : -15;
    if (work && launch_flip_axes(C, ldc, mi, ni, ta != 0, tb != 0, stream) != hipSuccess) return -100;
    return 0;
}

// ---------------------------------------------------------------------------------------------
// Bartels-Stewart (Sec. 1): A X + X B = alpha C with A = U At U^T, B = V Bt V^T in real Schur
// form.  Ct = U^T C V (two GEMMs through a workspace panel, the second written over C), the
// robust triangular solve At Y + Y Bt = alpha Ct in place, then X = U Y V^T (two GEMMs).  The
// transforms cannot overflow: with orthogonal U, V every partial sum of a transformed entry is
// bounded by the Frobenius norm of the matrix being transformed (Cauchy-Schwarz), so C and then
// Y enter their first GEMM times the power of two that brings that norm to OMEGA or below, and
// the two shifts are added to the scale exponent.
// Workspace: the forward workspace, one m x n panel, the norm partials and a few scalars.
// ---------------------------------------------------------------------------------------------
size_t trsyl_bartels_stewart_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts)
{
    const size_t fw = trsyl_workspace_size(m, n, opts);
    if (fw == 0) return 0;
    return align_up(fw) + align_up(8 * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(n, 1)) +
           align_up(8 * (size_t)kNormParts) + kAlign;
}

// Out = Aop Bop with the B operand staged times 2^(*bexp) (bexp: device int64)
static hipError_t plain_gemm(int M, int N, int K, const double *A, int64_t sAm, int64_t sAk,
                             const double *B, int64_t sBk, int64_t sBn, const int64_t *bexp, double *Out,
                             int64_t ldo, hipStream_t stream)
{
    GemmDesc g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.sAm = sAm; g.sAk = sAk; g.triA = 0;
    g.B = B; g.sBk = sBk; g.sBn = sBn; g.triB = 0;
    g.Cin = nullptr; g.ldcin = 1;
    g.Out = Out; g.ldo = ldo;
    g.sa1 = 0; g.sb1 = bexp ? 1 : 0;
    g.asign = 1.0; g.ae0 = 0; g.ae1 = 0; g.ae2 = 0;
    g.csign = 0.0; g.ce0 = 0; g.ce1 = 0; g.ce2 = 0;
    g.ep1 = bexp; g.ep2 = bexp;
    g.mask = 0; g.pat = nullptr; g.ldpat = 1;
    return launch_gemm(g, stream);
}

int trsyl_bartels_stewart(int64_t m, int64_t n, const double *U, int64_t ldu, const double *At,
                          int64_t ldat, const double *V, int64_t ldv, const double *Bt, int64_t ldbt,
                          double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
                          const trsyl_opts *opts, void *workspace, size_t ws_bytes,
                          trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && bad_ptr(U)) return -3;
    if (ldu < std::max<int64_t>(1, m)) return -4;
    if (m > 0 && bad_ptr(At)) return -5;
    if (ldat < std::max<int64_t>(1, m)) return -6;
    if (n > 0 && bad_ptr(V)) return -7;
    if (ldv < std::max<int64_t>(1, n)) return -8;
    if (n > 0 && bad_ptr(Bt)) return -9;
    if (ldbt < std::max<int64_t>(1, n)) return -10;
    if (m > 0 && n > 0 && bad_ptr(C)) return -11;
    if (ldc < std::max<int64_t>(1, m)) return -12;
    if (bad_ptr(scale_log2)) return -13;
    if (bad_ptr(info)) return -15;
    const size_t fw = trsyl_workspace_size(m, n, opts);
    if (fw == 0) return -16;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -17;
    if (ws_bytes < trsyl_bartels_stewart_workspace_size(m, n, opts)) return -18;
    if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return -1;
    const int mi = (int)m, ni = (int)n;
    const bool work = m > 0 && n > 0;
    char *ws = (char *)workspace;
    double *P = (double *)(ws + align_up(fw));
    double *part = (double *)(ws + align_up(fw) + align_up(8 * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(n, 1)));
    char *sc = (char *)part + align_up(8 * (size_t)kNormParts);
    int32_t *ns = (int32_t *)sc;                 // norm exponent
    double *nt = (double *)(sc + 8);             // norm sum of squares
    int64_t *neg = (int64_t *)(sc + 16);         // -shift of the operand being transformed
    int64_t *tot = (int64_t *)(sc + 24);         // sum of the shifts
    if (work) {
        if (launch_fill_zero(tot, sizeof(int64_t), stream) != hipSuccess) return -100;
        // P = U^T (2^-s0 C), then C = P V
        if (launch_norm(C, ldc, mi, ni, 0, part, ns, nt, stream) != hipSuccess) return -100;
        if (launch_norm_shift(ns, nt, neg, tot, stream) != hipSuccess) return -100;
        if (plain_gemm(mi, ni, mi, U, ldu, 1, C, 1, ldc, neg, P, mi, stream) != hipSuccess) return -100;
        if (plain_gemm(mi, ni, ni, P, 1, mi, V, 1, ldv, nullptr, C, ldc, stream) != hipSuccess) return -100;
    }
    const int rc = trsyl_robust(m, n, At, ldat, Bt, ldbt, C, ldc, scale_log2, scale, info, opts,
                                workspace, fw, stream_);
    if (rc != 0) return rc == -100 ? -100 : -16;
    if (work) {
        // P = U (2^-s1 Y), then C = P V^T; e += s0 + s1
        if (launch_norm(C, ldc, mi, ni, 0, part, ns, nt, stream) != hipSuccess) return -100;
        if (launch_norm_shift(ns, nt, neg, tot, stream) != hipSuccess) return -100;
        if (plain_gemm(mi, ni, mi, U, 1, ldu, C, 1, ldc, neg, P, mi, stream) != hipSuccess) return -100;
        if (plain_gemm(mi, ni, ni, P, 1, mi, V, ldv, 1, nullptr, C, ldc, stream) != hipSuccess) return -100;
        if (launch_add_exponent(scale_log2, scale, tot, stream) != hipSuccess) return -100;
    }
    return 0;
}

// ---------------------------------------------------------------------------------------------
// Batched adjoint: every problem reversed as in trsyl_robust_adjoint, then one batched forward
// solve.  Workspace: the batched forward workspace, then Ah_p (m_p x m_p) and Bh_p (n_p x n_p)
// for every problem.
// ---------------------------------------------------------------------------------------------
namespace {
size_t adjoint_batched_extra(int32_t count, const int64_t *m, const int64_t *n, std::vector<size_t> *offs)
{
    size_t o = 0;
    for (int p = 0; p < count; ++p) {
        if (offs) offs->push_back(o);
        o = align_up(o + 8 * (size_t)std::max<int64_t>(m[p], 1) * std::max<int64_t>(m[p], 1));
        if (offs) offs->push_back(o);
        o = align_up(o + 8 * (size_t)std::max<int64_t>(n[p], 1) * std::max<int64_t>(n[p], 1));
    }
    return o;
}
}  // namespace

size_t trsyl_adjoint_batched_workspace_size(int32_t count, const int64_t *m, const int64_t *n,
                                            const int32_t *tiles, const trsyl_opts *opts)
{
    if (count < 0 || (count > 0 && (!m || !n))) return 0;
    for (int p = 0; p < count; ++p)
        if (m[p] < 0 || n[p] < 0) return 0;
    const size_t fw = trsyl_batched_workspace_size(count, m, n, tiles, opts);
    if (count > 0 && fw == 0) return 0;
    return align_up(fw) + adjoint_batched_extra(count, m, n, nullptr);
}

int trsyl_robust_adjoint_batched(int32_t count, const int64_t *m, const int64_t *n, const double *const *A,
                                 const int64_t *lda, const double *const *B, const int64_t *ldb,
                                 double *const *W, const int64_t *ldw, const int32_t *tiles,
                                 int64_t *scale_log2, double *scale, int32_t *info, const trsyl_opts *opts,
                                 void *workspace, size_t ws_bytes, trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (count < 0) return -1;
    if (count == 0) return 0;
    if (!m || !n) return -2;
    if (!A || !lda) return -4;
    if (!B || !ldb) return -6;
    if (!W || !ldw) return -8;
    for (int p = 0; p < count; ++p) {
        if (m[p] < 0 || n[p] < 0 || m[p] > (int64_t)INT32_MAX / 2 || n[p] > (int64_t)INT32_MAX / 2) return -2;
        if (m[p] > 0 && bad_ptr(A[p])) return -4;
        if (lda[p] < std::max<int64_t>(1, m[p])) return -5;
        if (n[p] > 0 && bad_ptr(B[p])) return -6;
        if (ldb[p] < std::max<int64_t>(1, n[p])) return -7;
        if (m[p] > 0 && n[p] > 0 && bad_ptr(W[p])) return -8;
        if (ldw[p] < std::max<int64_t>(1, m[p])) return -9;
    }
    const size_t fw = trsyl_batched_workspace_size(count, m, n, tiles, opts);
    if (fw == 0) return -14;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -15;
    if (ws_bytes < trsyl_adjoint_batched_workspace_size(count, m, n, tiles, opts)) return -16;
    char *ws = (char *)workspace;
    std::vector<size_t> offs;
    adjoint_batched_extra(count, m, n, &offs);
    std::vector<const double *> Ah(count), Bh(count);
    std::vector<int64_t> ldah(count), ldbh(count);
    for (int p = 0; p < count; ++p) {
        double *ah = (double *)(ws + align_up(fw) + offs[2 * p]);
        double *bh = (double *)(ws + align_up(fw) + offs[2 * p + 1]);
        Ah[p] = ah;
        Bh[p] = bh;
        ldah[p] = std::max<int64_t>(1, m[p]);
        ldbh[p] = std::max<int64_t>(1, n[p]);
        if (m[p] > 0 && n[p] > 0) {
            if (launch_flip_transpose(A[p], lda[p], (int)m[p], ah, stream) != hipSuccess) return -100;
            if (launch_flip_transpose(B[p], ldb[p], (int)n[p], bh, stream) != hipSuccess) return -100;
            if (launch_flip(W[p], ldw[p], (int)m[p], (int)n[p], stream) != hipSuccess) return -100;
        }
    }
    const int rc = trsyl_robust_batched(count, m, n, Ah.data(), ldah.data(), Bh.data(), ldbh.data(), W, ldw,
                                        tiles, scale_log2, scale, info, opts, workspace, fw, stream_);
    if (rc != 0) return rc;
    for (int p = 0; p < count; ++p)
        if (m[p] > 0 && n[p] > 0 && launch_flip(W[p], ldw[p], (int)m[p], (int)n[p], stream) != hipSuccess)
            return -100;
    return 0;
}

// ---------------------------------------------------------------------------------------------
// Gradient products: with Gt = 2^eG G,
//   dC = 2^-eY Gt,  dA = -Gt Y^T on A's pattern,  dB = -Y^T Gt on B's pattern.
// ---------------------------------------------------------------------------------------------
int trsyl_grad(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
               const double *Y, int64_t ldy, const int64_t *eY, const double *G, int64_t ldg,
               const int64_t *eG, double *dA, int64_t ldda, double *dB, int64_t lddb, double *dC,
               int64_t lddc, trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && bad_ptr(A)) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (n > 0 && bad_ptr(B)) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (m > 0 && n > 0 && bad_ptr(Y)) return -7;
    if (ldy < std::max<int64_t>(1, m)) return -8;
    if (bad_ptr(eY)) return -9;
    if (m > 0 && n > 0 && bad_ptr(G)) return -10;
    if (ldg < std::max<int64_t>(1, m)) return -11;
    if (bad_ptr(eG)) return -12;
    if (m > 0 && bad_ptr(dA)) return -13;
    if (ldda < std::max<int64_t>(1, m)) return -14;
    if (n > 0 && bad_ptr(dB)) return -15;
    if (lddb < std::max<int64_t>(1, n)) return -16;
    if (m > 0 && n > 0 && bad_ptr(dC)) return -17;
    if (lddc < std::max<int64_t>(1, m)) return -18;
    if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return -1;
    const int mi = (int)m, ni = (int)n;
    GemmDesc g{};
    // dA (m x m) = -2^eG sum_k G(i, k) Y(j, k)
    g.M = mi; g.N = mi; g.K = ni;
    g.A = G; g.sAm = 1; g.sAk = ldg; g.triA = 0;
    g.B = Y; g.sBk = ldy; g.sBn = 1; g.triB = 0;
    g.Cin = nullptr; g.ldcin = 1;
    g.Out = dA; g.ldo = ldda;
    g.asign = -1.0; g.ae0 = 0; g.ae1 = 1; g.ae2 = 0; g.ep1 = eG; g.ep2 = eG;
    g.csign = 0.0; g.ce0 = g.ce1 = g.ce2 = 0;
    g.mask = 1; g.pat = A; g.ldpat = lda;
    if (m > 0 && launch_gemm(g, stream) != hipSuccess) return -100;
    // dB (n x n) = -2^eG sum_k Y(k, i) G(k, j)
    g.M = ni; g.N = ni; g.K = mi;
    g.A = Y; g.sAm = ldy; g.sAk = 1;
    g.B = G; g.sBk = 1; g.sBn = ldg;
    g.Out = dB; g.ldo = lddb;
    g.pat = B; g.ldpat = ldb;
    if (n > 0 && launch_gemm(g, stream) != hipSuccess) return -100;
    if (m > 0 && n > 0 && launch_scale_copy(G, ldg, mi, ni, eG, eY, dC, lddc, stream) != hipSuccess) return -100;
    return 0;
}

// ---------------------------------------------------------------------------------------------
// Eq. (9): with 2^sy > max|Y| and Ys = 2^-sy Y (the quotient is invariant under scaling Y and
// alpha together), R = 2^-(e+sy) C - A Ys - Ys B, and
//   out = ||R||_F / ((||A||_F + ||B||_F) ||Ys||_F + ||2^-(e+sy) C||_F),
// every norm carried as 2^s sqrt(t) so nothing overflows.  A and B norms cover their quasi-
// triangular parts (the only entries the solver reads).  Workspace: R (m x n), the partial sums,
// and a few scalars.
// ---------------------------------------------------------------------------------------------
size_t trsyl_residual_workspace_size(int64_t m, int64_t n)
{
    if (m < 0 || n < 0) return 0;
    return align_up(8 * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(n, 1)) +
           align_up(8 * (size_t)kNormParts) + 256;
}

int trsyl_residual(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                   const double *Y, int64_t ldy, const int64_t *e, const double *C, int64_t ldc,
                   double *out, void *workspace, size_t ws_bytes, trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && bad_ptr(A)) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (n > 0 && bad_ptr(B)) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (m > 0 && n > 0 && bad_ptr(Y)) return -7;
    if (ldy < std::max<int64_t>(1, m)) return -8;
    if (bad_ptr(e)) return -9;
    if (m > 0 && n > 0 && bad_ptr(C)) return -10;
    if (ldc < std::max<int64_t>(1, m)) return -11;
    if (bad_ptr(out)) return -12;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -13;
    if (ws_bytes < trsyl_residual_workspace_size(m, n)) return -14;
    if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return -1;
    if (m == 0 || n == 0) return launch_fill_zero(out, sizeof(double), stream) == hipSuccess ? 0 : -100;
    const int mi = (int)m, ni = (int)n;
    char *ws = (char *)workspace;
    double *R = (double *)ws;
    double *part = (double *)(ws + align_up(8 * (size_t)mi * ni));
    char *sc = ws + align_up(8 * (size_t)mi * ni) + align_up(8 * (size_t)kNormParts);
    int32_t *s5 = (int32_t *)sc;               // 5 exponents (R, A, B, Y, C)
    double *t5 = (double *)(sc + 32);          // 5 sums of squares
    int64_t *negsy = (int64_t *)(sc + 80);     // -sy

    if (launch_norm(Y, ldy, mi, ni, 0, part, s5 + 3, t5 + 3, stream) != hipSuccess) return -100;
    if (launch_neg_exp(s5 + 3, negsy, stream) != hipSuccess) return -100;
    GemmDesc g{};
    // R = 2^(-e - sy) C - A Ys
    g.M = mi; g.N = ni; g.K = mi;
    g.A = A; g.sAm = 1; g.sAk = lda; g.triA = 1;
    g.B = Y; g.sBk = 1; g.sBn = ldy; g.triB = 0;
    g.Cin = C; g.ldcin = ldc;
    g.Out = R; g.ldo = mi;
    g.sa1 = 0; g.sb1 = 1;                      // Ys = 2^-sy Y, staged
    g.asign = -1.0; g.ae0 = 0; g.ae1 = 0; g.ae2 = 0;
    g.csign = 1.0; g.ce0 = 0; g.ce1 = 1; g.ce2 = -1;
    g.ep1 = negsy; g.ep2 = e;
    g.mask = 0; g.pat = nullptr; g.ldpat = 1;
    if (launch_gemm(g, stream) != hipSuccess) return -100;
    // R -= Ys B
    g.K = ni;
    g.A = Y; g.sAm = 1; g.sAk = ldy; g.triA = 0;
    g.B = B; g.sBk = 1; g.sBn = ldb; g.triB = 1;
    g.sa1 = 1; g.sb1 = 0;
    g.Cin = R; g.ldcin = mi;
    g.csign = 1.0; g.ce0 = 0; g.ce1 = 0; g.ce2 = 0;
    if (launch_gemm(g, stream) != hipSuccess) return -100;
    if (launch_norm(R, mi, mi, ni, 0, part, s5 + 0, t5 + 0, stream) != hipSuccess) return -100;
    if (launch_norm(A, lda, mi, mi, 1, part, s5 + 1, t5 + 1, stream) != hipSuccess) return -100;
    if (launch_norm(B, ldb, ni, ni, 1, part, s5 + 2, t5 + 2, stream) != hipSuccess) return -100;
    if (launch_norm(C, ldc, mi, ni, 0, part, s5 + 4, t5 + 4, stream) != hipSuccess) return -100;
    if (launch_residual_final(s5, t5, e, out, stream) != hipSuccess) return -100;
    return 0;
}

}  // extern "C"
