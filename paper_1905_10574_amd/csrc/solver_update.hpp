// Tile update task (Algorithm 3, RobustUpdate) as an FP64 MFMA GEMM with power-of-two scaling.
//
// A column update writes target Y_il with the solved tile Y_kl (k > i):
//     D = (delta/gamma) Y_il - A_ik ((delta/alpha) Y_kl)
// a row update writes target Y_kj with Y_kl (l < j):
//     D = (delta/gamma) Y_kj - ((delta/alpha) Y_kl) B_lj
// with eta = min(gamma, alpha), zeta = ProtectUpdate((eta/gamma)||C||, ||A_ik|| or ||B_lj||,
// (eta/alpha)||Y_kl||) and delta = eta zeta, all scales powers of two held as exponents.  The
// printed update applies delta to both factors of the product; since delta^-1 D must equal
// gamma^-1 C - alpha^-1 (A B), delta enters once, through the solved tile.
//
// One task covers a horizontal slab of the target (full rows, so the slab computes its rows'
// exact absolute row sums); the tile's new infinity norm is the maximum over its slabs.
#pragma once
#include "device_common.hpp"
#include "plan.hpp"

namespace trsyl {

struct UpdateLds {
    double rows[kWaves][kMaxSlabRB * 16];
    double red[kWaves];
};

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Maximum over a 512-thread workgroup; every thread receives the result.  `red` holds kWaves
// doubles of shared scratch.  Contains two barriers.
__device__ __forceinline__ double wg_max(double v, double *red)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) r = fmax(r, red[i]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double tile_norm_at(const Plan &P, int T, int version)
{
    const double *p = P.tnorm + ((size_t)(version & 1) * P.pt * P.qt + T) * P.slabs;
    double r = 0.0;
    for (int s = 0; s < P.slabs; ++s) r = fmax(r, p[s]);
    return r;
}
__device__ __forceinline__ int32_t tile_exp_at(const Plan &P, int T, int version)
{
    return P.texp[(size_t)(version & 1) * P.pt * P.qt + T];
}
__device__ __forceinline__ double *tile_norm_slot(const Plan &P, int T, int version)
{
    return P.tnorm + ((size_t)(version & 1) * P.pt * P.qt + T) * P.slabs;
}
__device__ __forceinline__ int32_t *tile_exp_slot(const Plan &P, int T, int version)
{
    return P.texp + (size_t)(version & 1) * P.pt * P.qt + T;
}

// Row-block range of slab `slab` for a tile with `rows` rows.
__device__ __forceinline__ void slab_rows(int rows, int slabs, int slab, int *rb_lo, int *rb_hi)
{
    const int rbt = (rows + 15) >> 4;
    *rb_lo = (int)(((int64_t)slab * rbt) / slabs);
    *rb_hi = (int)(((int64_t)(slab + 1) * rbt) / slabs);
}

// ---------------------------------------------------------------------------------------------
// One wave accumulates acc[rb][cb] += sum_k Aop(m, k) Bop(k, n) for the rows
// m = m0 + 16 rb + (lane & 15) (valid below mlim) and columns n = n0 + 16 cbs[cb] + ... with the
// D^T mapping of device_common.hpp.  Operand values are scaled by 2^shA / 2^shB on load (exact
// powers of two; 0 means no scaling).
// ---------------------------------------------------------------------------------------------
template <int RB, int CB>
__device__ __forceinline__ void wave_gemm(d4 (&acc)[RB][CB], int nrb, int ncb,
                                          const double *Aop, int64_t lda, int m0, int mlim,
                                          const double *Bop, int64_t ldb, const int (&ncol)[CB],
                                          int nlim, int K, int shA, int shB)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    for (int kc = 0; kc < K; kc += 16) {
        double bf[CB][4], af[RB][4];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int nn = ncol[cb] + r;
            const bool nok = (cb < ncb) && (nn < nlim);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kc + 4 * q + j;
                bf[cb][j] = (nok && k < K) ? Bop[(int64_t)nn * ldb + k] : 0.0;
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int mm = m0 + 16 * rb + r;
            const bool mok = (rb < nrb) && (mm < mlim);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kc + 4 * q + j;
                af[rb][j] = (mok && k < K) ? Aop[(int64_t)k * lda + mm] : 0.0;
            }
        }
        if (shA) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int j = 0; j < 4; ++j) af[rb][j] = ldexp(af[rb][j], shA);
        }
        if (shB) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int j = 0; j < 4; ++j) bf[cb][j] = ldexp(bf[cb][j], shB);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    if (rb < nrb && cb < ncb) acc[rb][cb] = mfma16(bf[cb][j], af[rb][j], acc[rb][cb]);
    }
}

// Epilogue of one group of row blocks: D = 2^shC C - acc on the valid entries, and the entries'
// absolute values summed into rowsum[rb] (per lane; the lane's row is m0 + 16 rb + (lane & 15)).
template <int RBg, int CB>
__device__ __forceinline__ void slab_epilogue(const d4 (&acc)[RBg][CB], int nrbg, int m0, int rows,
                                              int cols, const int (&ncol)[CB], int ncb, double *Ct,
                                              int64_t ldc, int shC, double *rowsum)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int rb = 0; rb < RBg; ++rb) {
        const int mm = m0 + 16 * rb + (lane & 15);
        if (rb >= nrbg || mm >= rows) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if (cb >= ncb) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int nn = ncol[cb] + (lane >> 4) + 4 * i;
                if (nn < cols) {
                    double *p = Ct + (int64_t)nn * ldc + mm;
                    double c = *p;
                    if (shC) c = ldexp(c, shC);
                    const double d = c - acc[rb][cb][i];
                    *p = d;
                    rowsum[rb] += fabs(d);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Execute one update slab.  kind: kTaskColUpdate or kTaskRowUpdate.  T target, S source (solved),
// u the update's position in T's order (reads version u of T, writes version u+1).
// ---------------------------------------------------------------------------------------------
__device__ __noinline__ void run_update(const Plan &Pin, int kind_, int T_, int S_, int u_, int slab_,
                                       UpdateLds &L)
{
    const Plan P = uniform_plan(Pin);
    // callee arguments arrive in vector registers: make them (and all that derives from them,
    // including the branches around the barriers below) visibly uniform
    const int kind = uniform(kind_), T = uniform(T_), S = uniform(S_), u = uniform(u_);
    const int slab = uniform(slab_);
    const int ti = T / P.qt, tl = T % P.qt;
    const int si = S / P.qt, sl = S % P.qt;
    const int r0 = P.rowoff[ti], rows = P.rowoff[ti + 1] - r0;
    const int c0 = P.coloff[tl], cols = P.coloff[tl + 1] - c0;

    // scale decision (identical in every slab of this update)
    const int VS = tile_updates(P, S) + 1;
    const int eC = tile_exp_at(P, T, u);
    const int eY = tile_exp_at(P, S, VS);
    const double cn = tile_norm_at(P, T, u);
    const double yn = tile_norm_at(P, S, VS);
    const int emax = eC > eY ? eC : eY;
    const double cs = ldexp(cn, eC - emax), ys = ldexp(yn, eY - emax);
    double tn;
    const double *Aop;
    const double *Bop;
    int64_t lda_, ldb_;
    int K;
    int shA = 0, shB = 0;
    if (kind == kTaskColUpdate) {      // target (ti, tl) -= A(ti, si) * Y(si, tl)
        tn = P.anorm[(size_t)ti * P.pt + si];
        const int k0 = P.rowoff[si];
        K = P.rowoff[si + 1] - k0;
        Aop = P.A + (int64_t)k0 * P.lda + r0;
        lda_ = P.lda;
        Bop = P.C + (int64_t)c0 * P.ldc + k0;
        ldb_ = P.ldc;
    } else {                           // target (ti, tl) -= Y(ti, sl) * B(sl, tl)
        tn = P.bnorm[(size_t)sl * P.qt + tl];
        const int k0 = P.coloff[sl];
        K = P.coloff[sl + 1] - k0;
        Aop = P.C + (int64_t)k0 * P.ldc + r0;
        lda_ = P.ldc;
        Bop = P.B + (int64_t)c0 * P.ldb + k0;
        ldb_ = P.ldb;
    }
    const int s = (kind == kTaskColUpdate) ? protect_update(cs, tn, ys) : protect_update(cs, ys, tn);
    const int enew = emax + s;
    const int shC = eC - enew;        // <= 0
    const int shY = eY - enew;        // <= 0
    if (kind == kTaskColUpdate) shB = shY; else shA = shY;
    if (threadIdx.x == 0 && slab == 0 && (shC != 0 || shY != 0)) atomicAdd(&P.stats[1], 1u);

    int rb_lo, rb_hi;
    slab_rows(rows, P.slabs, slab, &rb_lo, &rb_hi);
    const int nrb = rb_hi - rb_lo;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ncbt = (cols + 15) >> 4;

    constexpr int CB = kMaxColBlocksPerWave;
    int ncol[CB];
    int ncb = 0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int g = w + kWaves * cb;
        ncol[cb] = 16 * g;
        if (g < ncbt) ncb = cb + 1;
    }
    const bool active = rows > 0 && cols > 0 && nrb > 0 && ncb > 0;
    double *Ct = P.C + (int64_t)c0 * P.ldc + r0;
    double rowsum[kMaxSlabRB];
#pragma unroll
    for (int rb = 0; rb < kMaxSlabRB; ++rb) rowsum[rb] = 0.0;

    if (active) {
        // main group: up to four row blocks
        const int n4 = nrb < 4 ? nrb : 4;
        d4 acc[4][CB];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < CB; ++b) acc[a][b] = zero4();
        if (K > 0)
            wave_gemm<4, CB>(acc, n4, ncb, Aop, lda_, 16 * rb_lo, rows, Bop, ldb_, ncol, cols, K, shA, shB);
        slab_epilogue<4, CB>(acc, n4, 16 * rb_lo, rows, cols, ncol, ncb, Ct, P.ldc, shC, rowsum);
        if (nrb > 4) {   // ragged fifth row block of a tile one row longer than nominal
            d4 acc1[1][CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) acc1[0][b] = zero4();
            if (K > 0)
                wave_gemm<1, CB>(acc1, 1, ncb, Aop, lda_, 16 * (rb_lo + 4), rows, Bop, ldb_, ncol, cols, K,
                                 shA, shB);
            slab_epilogue<1, CB>(acc1, 1, 16 * (rb_lo + 4), rows, cols, ncol, ncb, Ct, P.ldc, shC, rowsum + 4);
        }
    }

    // rows: lanes l, l^16, l^32, l^48 share a row; then across the waves through LDS
#pragma unroll
    for (int rb = 0; rb < kMaxSlabRB; ++rb) {
        double v = rowsum[rb];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lane < 16) L.rows[w][rb * 16 + lane] = v;
    }
    __syncthreads();
    double best = 0.0;
    if (threadIdx.x < kMaxSlabRB * 16) {
        double t = 0.0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) t += L.rows[ww][threadIdx.x];
        best = t;
    }
    best = wg_max(best, L.red);
    if (threadIdx.x == 0) {
        tile_norm_slot(P, T, u + 1)[slab] = best;
        *tile_exp_slot(P, T, u + 1) = enew;
    }
}

}  // namespace trsyl
