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

// Leading dimension of the LDS operand stages: 9 column blocks of 16 plus padding that shifts
// consecutive k rows across the LDS banks.
constexpr int kUS = 146;
constexpr int kUK = 16;               // k per stage

// FP64 stages loaded straight into LDS: As[k][m] (k-major, row stride kUS) and Bs[n][k]
// (column-major like the operand, 16 k per column plus one 16-byte pad slot, stride kBS), in a
// ring of kDStages buffers so that two stages are in flight while one is multiplied.
constexpr int kDStages = 3;
constexpr int kBS = 18;
constexpr int kDA = kUK * kUS;        // doubles per A stage
constexpr int kDB = 144 * kBS;        // doubles per B stage
constexpr int kDStage = kDA + kDB;

struct UpdateLds {
    // operand stages.  FP64: kDStages x (As, Bs) as above.  FP32 form: T As[2][kUK][kUS] followed
    // by T Bs[2][kUK][kUS], both k-major, staged through registers.
    double stage[kDStages * kDStage];
    double rs[kWaves][kMaxTile + 3];  // per-wave partial absolute row sums of the slab
    double red[kWaves];
    // multi-term update, per term: the solved tile, its first k (row of A_ik / column of B_lj),
    // its K, 1 for a column update (0: row update) and the exponent shift of the solved tile
    int gS[kMaxGroup], gk0[kMaxGroup], gK[kMaxGroup], gcol[kMaxGroup], gsh[kMaxGroup];
    double gyn[kMaxGroup], gtn[kMaxGroup];   // ||Y_S||_inf of the solved tile, ||A_ik|| or ||B_lj||
};
static_assert(2 * 2 * kUK * kUS <= kDStages * kDStage, "FP32 stages fit the FP64 ring");
template <class T> __device__ __forceinline__ T *stage_A(UpdateLds &L, int buf)
{
    return reinterpret_cast<T *>(L.stage) + (size_t)buf * kUK * kUS;
}
template <class T> __device__ __forceinline__ T *stage_B(UpdateLds &L, int buf)
{
    return reinterpret_cast<T *>(L.stage) + (size_t)(2 + buf) * kUK * kUS;
}

// MFMA accumulator and product per element type.  The FP64 16x16x4 product leaves result element
// t of lane l in row (l >> 4) + 4t of the (transposed) block, the FP32 one in row 4 (l >> 4) + t;
// both in column l & 15.
template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc_t;
    static __device__ __forceinline__ d4 zero() { return zero4(); }
    static __device__ __forceinline__ d4 mac(double b, double a, d4 c) { return mfma16(b, a, c); }
    static __device__ __forceinline__ int col(int q, int t) { return q + 4 * t; }
};
typedef float f4 __attribute__((ext_vector_type(4)));
template <> struct Mfma<float> {
    typedef f4 acc_t;
    static __device__ __forceinline__ f4 zero() { return (f4){0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ f4 mac(float b, float a, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int col(int q, int t) { return 4 * q + t; }
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

// Per-tile state written by other workgroups: read and written at device scope.
__device__ __forceinline__ DevView tnorm_view(const Plan &P)
{
    return dev_view(P.tnorm, (uint64_t)2 * P.pt * P.qt * P.slabs * 8);
}
__device__ __forceinline__ DevView texp_view(const Plan &P)
{
    return dev_view(P.texp, (uint64_t)2 * P.pt * P.qt * 4);
}
__device__ __forceinline__ int64_t tnorm_index(const Plan &P, int T, int version)
{
    return ((int64_t)(version & 1) * P.pt * P.qt + T) * P.slabs;
}
__device__ __forceinline__ int64_t texp_index(const Plan &P, int T, int version)
{
    return (int64_t)(version & 1) * P.pt * P.qt + T;
}
__device__ __forceinline__ double tile_norm_at(const Plan &P, int T, int version)
{
    const DevView v = tnorm_view(P);
    const int64_t b = tnorm_index(P, T, version);
    double r = 0.0;
    for (int s = 0; s < P.slabs; ++s) r = fmax(r, ld_dev(v, b + s));
    return r;
}
__device__ __forceinline__ int32_t tile_exp_at(const Plan &P, int T, int version)
{
    return ld_dev_i32(texp_view(P), texp_index(P, T, version));
}
__device__ __forceinline__ void tile_norm_store(const Plan &P, int T, int version, int slab, double v)
{
    st_dev(tnorm_view(P), tnorm_index(P, T, version) + slab, v);
}
__device__ __forceinline__ void tile_exp_store(const Plan &P, int T, int version, int32_t e)
{
    st_dev_i32(texp_view(P), texp_index(P, T, version), e);
}

// Row-block range of slab `slab` for a tile with `rows` rows.
__device__ __forceinline__ void slab_rows(int rows, int slabs, int slab, int *rb_lo, int *rb_hi)
{
    const int rbt = (rows + 15) >> 4;
    *rb_lo = (int)(((int64_t)slab * rbt) / slabs);
    *rb_hi = (int)(((int64_t)(slab + 1) * rbt) / slabs);
}

// n blocks are covered by groups of 8; a remainder of a single block joins the last group, so
// groups hold at most 9 blocks (a nominal 128 tile that grew by one row is one group).
__device__ __forceinline__ int block_groups(int n) { return n <= 9 ? 1 : (n % 8 == 1 ? n / 8 : (n + 7) / 8); }
__device__ __forceinline__ int group_size(int n, int g, int ng) { return g == ng - 1 ? n - 8 * g : 8; }

// ---------------------------------------------------------------------------------------------
// Stage k-chunk [kc, kc + 16) of both operands of a pass into LDS buffer `buf`:
//   As[k][m] = 2^shA Aop(m0 + m, kc + k) for m < Mp,  Bs[k][n] = 2^shB Bop(kc + k, n0 + n), n < Np,
// zero elsewhere (rows / columns past the pass and k past K), so every MFMA input is finite.
// Aop is column-major with leading dimension lda (consecutive threads read consecutive m), Bop
// column-major with ldb (16 consecutive k per column).  SA / SB select device-scope loads for
// the operand that other workgroups write.  Loads use clamped in-range addresses and a select.
// ---------------------------------------------------------------------------------------------
template <bool SA, bool SB>
struct StageRegs {
    double a[5], b[5];
};

template <bool SA, bool SB>
__device__ __forceinline__ void stage_load(StageRegs<SA, SB> &R, const double *Aop, const DevView &vA,
                                           int64_t lda, int m0, int Mp, const double *Bop,
                                           const DevView &vB, int64_t ldb, int n0, int Np, int kc, int K)
{
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int e = threadIdx.x + kThreads * i;
        if (i == 4 && threadIdx.x >= kUK * 144 - 4 * kThreads) break;     // wave-uniform tail
        {
            const int m = e % 144, k = kc + e / 144;
            const int mc = m < Mp ? m : 0, kk = k < K ? k : K - 1;
            const int64_t idx = (int64_t)kk * lda + m0 + mc;
            double v;
            if constexpr (SA) v = ld_dev(vA, idx);
            else v = ldg(Aop + idx);
            R.a[i] = (m < Mp && k < K) ? v : 0.0;
        }
        {
            const int k = kc + (e & 15), n = e >> 4;
            const int nc_ = n < Np ? n : 0, kk = k < K ? k : K - 1;
            const int64_t idx = (int64_t)(n0 + nc_) * ldb + kk;
            double v;
            if constexpr (SB) v = ld_dev(vB, idx);
            else v = ldg(Bop + idx);
            R.b[i] = (n < Np && k < K) ? v : 0.0;
        }
    }
}

template <class T, bool SA, bool SB>
__device__ __forceinline__ void stage_store(const StageRegs<SA, SB> &R, UpdateLds &L, int buf,
                                            int shA, int shB)
{
    T *As = stage_A<T>(L, buf), *Bs = stage_B<T>(L, buf);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int e = threadIdx.x + kThreads * i;
        if (i == 4 && threadIdx.x >= kUK * 144 - 4 * kThreads) break;
        As[(e / 144) * kUS + e % 144] = (T)(shA ? ldexp(R.a[i], shA) : R.a[i]);
        Bs[(e & 15) * kUS + (e >> 4)] = (T)(shB ? ldexp(R.b[i], shB) : R.b[i]);
    }
}

// Target block (brow, bcol) of a pass, in the MFMA result layout: lane (r, q) holds rows
// m0 + 16 brow + r and columns n0 + 16 bcol + q + 4i.  Loads use clamped in-range addresses.
template <class T>
__device__ __forceinline__ void load_target(double (&cv)[4], const DevView &Ct, int64_t ldc, int m0,
                                            int Mp, int n0, int Np, int brow, int bcol)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int mm = m0 + 16 * brow + r;
    const int mmc = mm < m0 + Mp ? mm : m0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nn = n0 + 16 * bcol + Mfma<T>::col(q, i);
        const int nnc = nn < n0 + Np ? nn : n0;
        cv[i] = ld_dev(Ct, (int64_t)nnc * ldc + mmc);
    }
}

// D = 2^shC C - acc on the valid entries of the block, stored at device scope; the block's
// absolute row sums are added to rs[row - rbase] (row tile-relative).
template <class T>
__device__ __forceinline__ void store_target(const double (&cv)[4], const typename Mfma<T>::acc_t &ac,
                                             int shC, int shP, const DevView &Ct, int64_t ldc, int m0,
                                             int Mp, int n0, int Np, int brow, int bcol, double *rs,
                                             int rbase)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int mm = m0 + 16 * brow + r;
    const bool mok = mm < m0 + Mp;
    double rsum = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nn = n0 + 16 * bcol + Mfma<T>::col(q, i);
        if (mok && nn < n0 + Np) {
            const double c = shC ? ldexp(cv[i], shC) : cv[i];
            const double p = shP ? ldexp((double)ac[i], shP) : (double)ac[i];
            const double d = c - p;
            st_dev(Ct, (int64_t)nn * ldc + mm, d);
            rsum += fabs(d);
        }
    }
    rsum += __shfl_xor(rsum, 16);
    rsum += __shfl_xor(rsum, 32);
    if (q == 0 && mok) rs[mm - rbase] += rsum;
}

// ---------------------------------------------------------------------------------------------
// Execute one update slab.  kind: kTaskColUpdate or kTaskRowUpdate.  T target, S source (solved),
// u the update's position in T's order (reads version u of T, writes version u+1).
//
// The slab's row blocks x the tile's column blocks are covered in passes of at most 9 x 9
// blocks of 16 x 16.  In a pass, wave w = 4 wr + wc owns the 4 x 2 blocks rows 4wr.., columns
// 2wc.. of the first 8 x 8, and a share of the ninth block row / column (at most three
// blocks), all accumulated with v_mfma_f64_16x16x4 from LDS stages of 16 k that are double
// buffered: the next stage's global loads are in flight while the current stage's MFMAs run.
// ---------------------------------------------------------------------------------------------
// T = double: operands staged as they are (times 2^shA, 2^shB), product used as computed (shP
// = 0).  T = float: operands staged times 2^shA, 2^shB chosen to normalise them into FP32's range,
// product taken back by 2^shP; every scale is an exact power of two.
template <bool COL, class T>
__device__ __forceinline__ void update_passes(const Plan &P, const double *Aop, int64_t lda,
                                              const double *Bop, int64_t ldb, int K, int shA,
                                              int shB, int shP, int shC, double *Ct, int rows,
                                              int cols, int rb_lo, int nrb, UpdateLds &L,
                                              uint64_t *ustamp)
{
    typedef typename Mfma<T>::acc_t acc_t;
    constexpr bool SA = !COL, SB = COL;     // the solved tile Y_S is the shared operand
    const int w = uniform((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int wr = w >> 2, wc = w & 3;
    const int ncbt = (cols + 15) >> 4;
    const int ngr = block_groups(nrb), ngc = block_groups(ncbt);
    const int nkc = (K + kUK - 1) / kUK;
    const DevView vA = dev_view(Aop, lda, rows, K), vB = dev_view(Bop, ldb, K, cols);
    const DevView vC = dev_view(Ct, P.ldc, rows, cols);
    for (int gr = 0; gr < ngr; ++gr) {
        for (int gc = 0; gc < ngc; ++gc) {
            const int R = group_size(nrb, gr, ngr), Cc = group_size(ncbt, gc, ngc);
            const int m0 = 16 * (rb_lo + 8 * gr), n0 = 16 * 8 * gc;
            const int Mp = (m0 + 16 * R < rows ? m0 + 16 * R : rows) - m0;
            const int Np = (n0 + 16 * Cc < cols ? n0 + 16 * Cc : cols) - n0;
            const int R8 = R < 8 ? R : 8, C8 = Cc < 8 ? Cc : 8;
            // this wave's main blocks and extra blocks (ninth block row, then ninth column)
            const int nrm = R8 - 4 * wr < 0 ? 0 : (R8 - 4 * wr > 4 ? 4 : R8 - 4 * wr);
            const int ncm = C8 - 2 * wc < 0 ? 0 : (C8 - 2 * wc > 2 ? 2 : C8 - 2 * wc);
            const int xrow = R == 9 ? Cc : 0;
            const int nx = xrow + (Cc == 9 ? R8 : 0);
            int xr[3], xc[3];
            int nxw = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int e = w + kWaves * j;
                xr[j] = e < xrow ? 8 : e - xrow;
                xc[j] = e < xrow ? e : 8;
                if (e < nx) nxw = j + 1;
            }
            acc_t acc[4][2], accx[3];
#pragma unroll
            for (int a = 0; a < 4; ++a) { acc[a][0] = Mfma<T>::zero(); acc[a][1] = Mfma<T>::zero(); }
#pragma unroll
            for (int j = 0; j < 3; ++j) accx[j] = Mfma<T>::zero();

            StageRegs<SA, SB> SR;
            stage_load<SA, SB>(SR, Aop, vA, lda, m0, Mp, Bop, vB, ldb, n0, Np, 0, K);
            stage_store<T, SA, SB>(SR, L, 0, shA, shB);
            __syncthreads();
            if (ustamp && threadIdx.x == 0 && gr == 0 && gc == 0) ustamp[2] = wall_clock64();
            for (int c = 0; c < nkc; ++c) {
                const int buf = c & 1;
                const bool more = c + 1 < nkc;
                if (more) stage_load<SA, SB>(SR, Aop, vA, lda, m0, Mp, Bop, vB, ldb, n0, Np, kUK * (c + 1), K);
                const T *As = stage_A<T>(L, buf), *Bs = stage_B<T>(L, buf);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 4 * q + j;
                    T av[4], bv[2];
#pragma unroll
                    for (int a = 0; a < 4; ++a) av[a] = As[k * kUS + 16 * (4 * wr + a) + r];
#pragma unroll
                    for (int b = 0; b < 2; ++b) bv[b] = Bs[k * kUS + 16 * (2 * wc + b) + r];
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            if (a < nrm && b < ncm) acc[a][b] = Mfma<T>::mac(bv[b], av[a], acc[a][b]);
#pragma unroll
                    for (int x = 0; x < 3; ++x)
                        if (x < nxw)
                            accx[x] = Mfma<T>::mac(Bs[k * kUS + 16 * xc[x] + r], As[k * kUS + 16 * xr[x] + r], accx[x]);
                }
                if (more) stage_store<T, SA, SB>(SR, L, buf ^ 1, shA, shB);
                __syncthreads();
            }

            if (ustamp && threadIdx.x == 0 && gr == 0 && gc == 0) ustamp[3] = wall_clock64();
            // epilogue: D = 2^shC C - acc, row sums into this wave's partials
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                double cm[4][4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    if (a < nrm && b < ncm) load_target<T>(cm[a], vC, P.ldc, m0, Mp, n0, Np, 4 * wr + a, 2 * wc + b);
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    if (a < nrm && b < ncm)
                        store_target<T>(cm[a], acc[a][b], shC, shP, vC, P.ldc, m0, Mp, n0, Np, 4 * wr + a,
                                        2 * wc + b, L.rs[w], 16 * rb_lo);
            }
            double cx[3][4];
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (x < nxw) load_target<T>(cx[x], vC, P.ldc, m0, Mp, n0, Np, xr[x], xc[x]);
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (x < nxw)
                    store_target<T>(cx[x], accx[x], shC, shP, vC, P.ldc, m0, Mp, n0, Np, xr[x], xc[x], L.rs[w], 16 * rb_lo);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// FP64 passes with direct-to-LDS operand stages (gfx950 global_load_lds_dwordx4: lane l of a wave
// writes the 16 bytes it loads to LDS at base + 16 l, without passing through registers).
//
// A stage (16 k) is issued by every wave: A rows k = 2w, 2w + 1 (one instruction for m < 128 and
// one of 8 lanes for m = 128..143), and B slots 64 i + lane for i = w, w + 8, w + 16 (< 21): slot
// s covers column n = s / 9, k = 2 (s % 9) .. + 1, with s % 9 == 8 the pad.  Lanes whose k range
// lies at or beyond K, whose column is past the pass, or that fill a pad read 16 bytes of zeros;
// when K is odd the B slot holding k = K - 1 also reads zeros and that one value is written into
// LDS separately (a 16-byte read would cross the source tile).  A rows past the pass are loaded
// (they only feed output rows that are not stored) or read as zeros.
//
// Waits are explicit: loads return in issue order, so `s_waitcnt vmcnt(n)` with n the loads issued
// after a stage completes it.  The barriers between stages wait only for LDS traffic (a workgroup
// fence would also wait for the two stages still in flight).
// ---------------------------------------------------------------------------------------------
// Target block (brow, bcol) of a pass loaded into an FP64 accumulator in the MFMA result layout
// (element i of lane (r, q): row m0 + 16 brow + r, column n0 + 16 bcol + q + 4 i); entries past
// the pass read as zero.
__device__ __forceinline__ void load_target_acc(d4 &acc, const DevView &Ct, int64_t ldc, int m0, int Mp, int n0,
                                                int Np, int brow, int bcol)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int mm = m0 + 16 * brow + r;
    const bool mok = mm < m0 + Mp;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nn = n0 + 16 * bcol + q + 4 * i;
        const bool ok = mok && nn < n0 + Np;
        const double v = ld_dev(Ct, (int64_t)(ok ? nn : n0) * ldc + (ok ? mm : m0));
        acc[i] = ok ? v : 0.0;
    }
}
// -2^sh x, element by element (sh <= 0: an exact power-of-two scaling, the target's share of
// Algorithm 3's delta / gamma)
__device__ __forceinline__ d4 neg_scale4(d4 x, int sh)
{
    d4 y;
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = -(sh ? ldexp(x[i], sh) : x[i]);
    return y;
}
// The target block's values as load_target_acc leaves them, but loaded from clamped in-range
// addresses without the masking select, so that the loads of all blocks are in flight together
// (a select right after each block's loads makes the compiler wait for them, one round trip per
// block); the masking happens in neg_scale4_masked, after every load has been issued.
__device__ __forceinline__ void load_target_raw(d4 &acc, const DevView &Ct, int64_t ldc, int m0, int Mp, int n0,
                                                int Np, int brow, int bcol)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int mm = m0 + 16 * brow + r;
    const bool mok = mm < m0 + Mp;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nn = n0 + 16 * bcol + q + 4 * i;
        const bool ok = mok && nn < n0 + Np;
        acc[i] = ld_dev(Ct, (int64_t)(ok ? nn : n0) * ldc + (ok ? mm : m0));
    }
}
__device__ __forceinline__ d4 neg_scale4_masked(d4 x, int sh, int m0, int Mp, int n0, int Np, int brow, int bcol)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const bool mok = m0 + 16 * brow + r < m0 + Mp;
    d4 y;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool ok = mok && n0 + 16 * bcol + q + 4 * i < n0 + Np;
        y[i] = ok ? -(sh ? ldexp(x[i], sh) : x[i]) : 0.0;
    }
    return y;
}
// Stores D = -acc on the valid entries of the block (device scope) and adds the block's absolute
// row sums to rs[row - rbase].
__device__ __forceinline__ void store_neg_acc(const d4 &acc, const DevView &Ct, int64_t ldc, int m0, int Mp, int n0,
                                              int Np, int brow, int bcol, double *rs, int rbase)
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int mm = m0 + 16 * brow + r;
    const bool mok = mm < m0 + Mp;
    double rsum = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nn = n0 + 16 * bcol + q + 4 * i;
        if (mok && nn < n0 + Np) {
            const double d = -acc[i];
            st_dev(Ct, (int64_t)nn * ldc + mm, d);
            rsum += fabs(d);
        }
    }
    rsum += __shfl_xor(rsum, 16);
    rsum += __shfl_xor(rsum, 32);
    if (q == 0 && mok) rs[mm - rbase] += rsum;
}

__device__ __align__(16) const double g_zero16[2] = {0.0, 0.0};

typedef __attribute__((address_space(1))) const void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

// s_waitcnt vmcnt(n) (0 <= n < 16) leaving the other counters alone.  n is wave-uniform.
__device__ __forceinline__ void wait_vm(int n)
{
#define TRSYL_VM(N) case N: __builtin_amdgcn_s_waitcnt((N) | (0x7 << 4) | (0xF << 8)); break;
    switch (n) {
        TRSYL_VM(0) TRSYL_VM(1) TRSYL_VM(2) TRSYL_VM(3) TRSYL_VM(4) TRSYL_VM(5) TRSYL_VM(6)
        TRSYL_VM(7) TRSYL_VM(8) TRSYL_VM(9) TRSYL_VM(10) TRSYL_VM(11) TRSYL_VM(12) TRSYL_VM(13)
        TRSYL_VM(14)
        default: __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xF << 8)); break;
    }
#undef TRSYL_VM
}

// Workgroup barrier that orders LDS traffic only: this wave's LDS accesses have completed, and the
// compiler moves no memory access across it.  Global loads in flight stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xF | (0x7 << 4) | (0x0 << 8) | (0x3 << 14));   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ double *dstage_A(UpdateLds &L, int buf) { return L.stage + (size_t)buf * kDStage; }
__device__ __forceinline__ double *dstage_B(UpdateLds &L, int buf) { return L.stage + (size_t)buf * kDStage + kDA; }

// Issue stage kc (k in [kc, kc + 16)) of a pass into ring buffer `buf`.  PA / PB: cache policy
// of the A / B operand (device scope for the solved tile, which other workgroups write).
template <int PA, int PB>
__device__ __forceinline__ void dma_stage(UpdateLds &L, int buf, const double *Aop, int64_t lda, int m0, int Mp,
                                          bool tailA, const double *Bop, int64_t ldb, int n0, int Np, int kc, int K)
{
    const int w = uniform((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    double *stA = dstage_A(L, buf), *stB = dstage_B(L, buf);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int kr = 2 * w + h, k = kc + kr;
        const bool kin = k < K;
        {
            const int m = 2 * lane;
            const double *src = (kin && m < Mp) ? Aop + (int64_t)k * lda + m0 + m : g_zero16;
            __builtin_amdgcn_global_load_lds((gvoid_t *)src, (lvoid_t *)(stA + kr * kUS), 16, 0, PA);
        }
        if (tailA) {
            if (lane < 8) {
                const int m = 128 + 2 * lane;
                const double *src = (kin && m < Mp) ? Aop + (int64_t)k * lda + m0 + m : g_zero16;
                __builtin_amdgcn_global_load_lds((gvoid_t *)src, (lvoid_t *)(stA + kr * kUS + 128), 16, 0, PA);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int i = w + 8 * t;
        if (i < 21) {
            const int s = 64 * i + lane;
            const int n = s / 9, j = s - 9 * n;
            const int k = kc + 2 * j;
            const bool ok = j < 8 && n < Np && k + 1 < K;
            const double *src = ok ? Bop + (int64_t)(n0 + n) * ldb + k : g_zero16;
            if (i < 20 || lane < 16)
                __builtin_amdgcn_global_load_lds((gvoid_t *)src, (lvoid_t *)(stB + 128 * i), 16, 0, PB);
        }
    }
}

// One term of an FP64 update pass: Aop (rows x K, column-major, ld lda) times Bop (K x cols,
// column-major, ld ldb).  The solved tile -- the B operand of a column update, the A operand of a
// row update -- is read at device scope (other workgroups write it) and enters the product times
// 2^shY; the A / B panels keep the default cache policy, so that they stay in the XCD's L2 across
// the many updates that read them.
struct UpdTerm {
    const double *Aop;
    int64_t lda;
    const double *Bop;
    int64_t ldb;
    int K, col, shY;
};

// Issue stage kc (k in [kc, kc + 16)) of term tm into ring buffer `buf`.  KIND: 1 every term is a
// column update, 2 every term a row update (the policies are then fixed at compile time), 0 mixed.
template <int KIND>
__device__ __forceinline__ void term_stage(UpdateLds &L, int buf, const UpdTerm &tm, int m0, int Mp, bool tailA,
                                           int n0, int Np, int kc)
{
    if (KIND == 0 ? tm.col != 0 : KIND == 1)
        dma_stage<0, kPolicyDevice>(L, buf, tm.Aop, tm.lda, m0, Mp, tailA, tm.Bop, tm.ldb, n0, Np, kc, tm.K);
    else
        dma_stage<kPolicyDevice, 0>(L, buf, tm.Aop, tm.lda, m0, Mp, tailA, tm.Bop, tm.ldb, n0, Np, kc, tm.K);
}

// k = K - 1 of B column n0 + threadIdx.x (threads below Np): the stage loads k in pairs, so an odd
// K's last k is staged separately.
__device__ __forceinline__ double term_fix(const UpdTerm &tm, int n0, int Np)
{
    if ((int)threadIdx.x >= Np) return 0.0;
    const int64_t idx = (int64_t)(n0 + threadIdx.x) * tm.ldb + (tm.K - 1);
    if (tm.col) return ld_dev(dev_view(tm.Bop, tm.ldb, tm.K, n0 + Np), idx);
    return ldg(tm.Bop + idx);
}

// Cursors over the concatenated stages of g terms: term t, first k of the stage kc; terms with
// K = 0 contribute no stage.  A term is fetched only when a cursor enters it, and each cursor
// keeps only what its side of the loop needs (the issuing side the operands, the multiplying
// side the term's K, kind and shift), to spare registers in the stage loop.
struct IssueCursor {
    int t, kc, K, col;
    const double *Aop, *Bop;
    int64_t lda, ldb;
    __device__ __forceinline__ void set(const UpdTerm &x)
    {
        K = x.K; col = x.col; Aop = x.Aop; Bop = x.Bop; lda = x.lda; ldb = x.ldb;
    }
    __device__ __forceinline__ UpdTerm term() const { return UpdTerm{Aop, lda, Bop, ldb, K, col, 0}; }
};
struct ProcCursor {
    int t, kc, K, col, shY;
    __device__ __forceinline__ void set(const UpdTerm &x) { K = x.K; col = x.col; shY = x.shY; }
};
template <class C, class Term>
__device__ __forceinline__ void cursor_start(C &c, int g, Term term)
{
    c.t = 0;
    c.kc = 0;
    c.set(term(0));
    while (c.t < g && c.kc >= c.K) {
        ++c.t;
        if (c.t < g) c.set(term(c.t));
    }
}
template <class C, class Term>
__device__ __forceinline__ void cursor_next(C &c, int g, Term term)
{
    c.kc += kUK;
    while (c.t < g && c.kc >= c.K) {
        ++c.t;
        c.kc = 0;
        if (c.t < g) c.set(term(c.t));
    }
}

// One update slab in FP64 over g terms (a single update: g = 1), the terms' K dimensions
// concatenated into one stream of 16-k stages:
//     D = 2^shC C - sum_t 2^shY_t Aop_t Bop_t.
// `term(t)` returns term t (its shY valid once `decide` has run); `decide` runs the scale decision
// and returns shC; it is called once, after the first pass's first two stages have been issued,
// so that its loads overlap theirs, and leaves the shifts it stores visible to every wave (the
// stage cursor fetches them right after it returns).  See update_passes for the block layout of the waves.
// SIMPLE: one pass of 8 x 8 blocks (113..128 rows and columns), for which the extra block
// row/column and the pass loop compile away (fewer live registers, so the set-up does not spill).
template <bool SIMPLE, int KIND, class Term, class Decide>
__device__ __forceinline__ void update_stream_f64(const Plan &P, int g, Term term, double *Ct, int rows, int cols,
                                                  int rb_lo, int nrb, UpdateLds &L, uint64_t *ustamp, Decide decide)
{
    const int w = uniform((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int wr = w >> 2, wc = w & 3;
    const int ncbt = SIMPLE ? 8 : (cols + 15) >> 4;
    const int ngr = SIMPLE ? 1 : block_groups(nrb), ngc = SIMPLE ? 1 : block_groups(ncbt);
    int nkc = 0;
    for (int t = 0; t < g; ++t) nkc += (term(t).K + kUK - 1) / kUK;
    nkc = uniform(nkc);
    const DevView vC = dev_view(Ct, P.ldc, rows, cols);
    const int nB = w < 5 ? 3 : 2;
    int shC = 0;
    bool decided = false;
    for (int gr = 0; gr < ngr; ++gr) {
        for (int gc = 0; gc < ngc; ++gc) {
            const int R = SIMPLE ? 8 : group_size(nrb, gr, ngr), Cc = SIMPLE ? 8 : group_size(ncbt, gc, ngc);
            const int m0 = 16 * (rb_lo + 8 * gr), n0 = 16 * 8 * gc;
            const int Mp = (m0 + 16 * R < rows ? m0 + 16 * R : rows) - m0;
            const int Np = (n0 + 16 * Cc < cols ? n0 + 16 * Cc : cols) - n0;
            const int R8 = R < 8 ? R : 8, C8 = Cc < 8 ? Cc : 8;
            const int nrm = R8 - 4 * wr < 0 ? 0 : (R8 - 4 * wr > 4 ? 4 : R8 - 4 * wr);
            const int ncm = C8 - 2 * wc < 0 ? 0 : (C8 - 2 * wc > 2 ? 2 : C8 - 2 * wc);
            const int xrow = R == 9 ? Cc : 0;
            const int nx = xrow + (Cc == 9 ? R8 : 0);
            int xr[3], xc[3];
            int nxw = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int e = w + kWaves * j;
                xr[j] = e < xrow ? 8 : e - xrow;
                xc[j] = e < xrow ? e : 8;
                if (e < nx) nxw = j + 1;
            }
            const bool tailA = SIMPLE ? false : uniform(Mp > 128 ? 1 : 0) != 0;
            const bool full = nrm == 4 && ncm == 2;              // all eight main blocks live
            const int Lw = 2 + (tailA ? 2 : 0) + nB;             // DMA loads per stage of this wave
            // every wave has left the previous pass's buffers
            lds_barrier();
            // the target's blocks go straight into the accumulators (issued first, so that they,
            // the first two operand stages and the scale decision share one round trip); the
            // product is then accumulated onto -2^shC C and the result is the negated sum
            d4 acc[4][2], accx[3];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    acc[a][b] = zero4();
                    if (a < nrm && b < ncm) load_target_raw(acc[a][b], vC, P.ldc, m0, Mp, n0, Np, 4 * wr + a, 2 * wc + b);
                }
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                accx[x] = zero4();
                if (x < nxw) load_target_raw(accx[x], vC, P.ldc, m0, Mp, n0, Np, xr[x], xc[x]);
            }
            // stages in flight and their odd-K values (one per ring parity)
            IssueCursor is;
            cursor_start(is, g, term);
            double fx0 = 0.0, fx1 = 0.0;
            for (int c = 0; c < 2 && c < nkc; ++c) {
                const UpdTerm tm = is.term();
                term_stage<KIND>(L, c, tm, m0, Mp, tailA, n0, Np, is.kc);
                if (uniform((tm.K & 1) && is.kc + kUK >= tm.K ? 1 : 0)) {
                    if (c == 0) fx0 = term_fix(tm, n0, Np); else fx1 = term_fix(tm, n0, Np);
                }
                cursor_next(is, g, term);
            }
            if (!decided) {
                shC = uniform(decide());
                decided = true;
            }
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    acc[a][b] = neg_scale4_masked(acc[a][b], shC, m0, Mp, n0, Np, 4 * wr + a, 2 * wc + b);
#pragma unroll
            for (int x = 0; x < 3; ++x) accx[x] = neg_scale4_masked(accx[x], shC, m0, Mp, n0, Np, xr[x], xc[x]);
            if (ustamp && threadIdx.x == 0 && gr == 0 && gc == 0) ustamp[2] = wall_clock64();
            ProcCursor ps;
            cursor_start(ps, g, term);
            for (int c = 0; c < nkc; ++c) {
                const int buf = c % kDStages;
                wait_vm(c + 1 < nkc ? Lw : 0);
                lds_barrier();
                const int shY = uniform(ps.shY);
                const bool pcol = KIND == 0 ? ps.col != 0 : KIND == 1;
                const bool lastodd = uniform((ps.K & 1) && ps.kc + kUK >= ps.K ? 1 : 0) != 0;
                if (shY != 0) {
                    // the solved tile enters the product times 2^shY (Algorithm 3's delta / alpha)
                    double *sh = pcol ? dstage_B(L, buf) : dstage_A(L, buf);
                    const int cnt = pcol ? kDB : kDA;
                    for (int t = threadIdx.x; t < cnt; t += kThreads) sh[t] = ldexp(sh[t], shY);
                    if (lastodd) lds_barrier();
                }
                if (lastodd) {
                    const double fix = (c & 1) ? fx1 : fx0;
                    if ((int)threadIdx.x < Np)
                        dstage_B(L, buf)[threadIdx.x * kBS + (ps.K - 1 - ps.kc)] = (pcol && shY) ? ldexp(fix, shY) : fix;
                }
                if (shY != 0 || lastodd) lds_barrier();
                if (c + 2 < nkc) {
                    const UpdTerm tn = is.term();
                    term_stage<KIND>(L, (c + 2) % kDStages, tn, m0, Mp, tailA, n0, Np, is.kc);
                    if (uniform((tn.K & 1) && is.kc + kUK >= tn.K ? 1 : 0)) {
                        if (c & 1) fx1 = term_fix(tn, n0, Np); else fx0 = term_fix(tn, n0, Np);
                    }
                    cursor_next(is, g, term);
                }
                const double *As = dstage_A(L, buf), *Bs = dstage_B(L, buf);
                // this lane's 4 k of each of its B column blocks are adjacent: two 16-byte reads
                double bq[2][4];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double2 *bp = reinterpret_cast<const double2 *>(Bs + (16 * (2 * wc + b) + r) * kBS + 4 * q);
                    const double2 x0 = bp[0], x1 = bp[1];
                    bq[b][0] = x0.x; bq[b][1] = x0.y; bq[b][2] = x1.x; bq[b][3] = x1.y;
                }
                if (full) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = 4 * q + j;
                        double av[4];
#pragma unroll
                        for (int a = 0; a < 4; ++a) av[a] = As[k * kUS + 16 * (4 * wr + a) + r];
#pragma unroll
                        for (int a = 0; a < 4; ++a)
#pragma unroll
                            for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bq[b][j], av[a], acc[a][b]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = 4 * q + j;
                        double av[4];
#pragma unroll
                        for (int a = 0; a < 4; ++a) av[a] = As[k * kUS + 16 * (4 * wr + a) + r];
#pragma unroll
                        for (int a = 0; a < 4; ++a)
#pragma unroll
                            for (int b = 0; b < 2; ++b)
                                if (a < nrm && b < ncm) acc[a][b] = mfma16(bq[b][j], av[a], acc[a][b]);
                    }
                }
                if (nxw > 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = 4 * q + j;
#pragma unroll
                        for (int x = 0; x < 3; ++x)
                            if (x < nxw)
                                accx[x] = mfma16(Bs[(16 * xc[x] + r) * kBS + k], As[k * kUS + 16 * xr[x] + r], accx[x]);
                    }
                }
                cursor_next(ps, g, term);
            }
            if (ustamp && threadIdx.x == 0 && gr == 0 && gc == 0) ustamp[3] = wall_clock64();
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    if (a < nrm && b < ncm)
                        store_neg_acc(acc[a][b], vC, P.ldc, m0, Mp, n0, Np, 4 * wr + a, 2 * wc + b, L.rs[w], 16 * rb_lo);
#pragma unroll
            for (int x = 0; x < 3; ++x)
                if (x < nxw) store_neg_acc(accx[x], vC, P.ldc, m0, Mp, n0, Np, xr[x], xc[x], L.rs[w], 16 * rb_lo);
        }
    }
}

__device__ __noinline__ void run_update(const Plan &Pin, int kind_, int T_, int S_, int u_, int slab_,
                                       UpdateLds &L, uint64_t *ustamp)
{
    const Plan P = uniform_plan(Pin);
    if (ustamp && threadIdx.x == 0) ustamp[0] = wall_clock64();
    // callee arguments arrive in vector registers: make them (and all that derives from them,
    // including the branches around the barriers below) visibly uniform
    const int kind = uniform(kind_), T = uniform(T_), S = uniform(S_), u = uniform(u_);
    const int slab = uniform(slab_);
    const int ti = T / P.qt, tl = T % P.qt;
    const int si = S / P.qt, sl = S % P.qt;
    const int r0 = uniform(P.rowoff[ti]), rows = uniform(P.rowoff[ti + 1]) - r0;
    const int c0 = uniform(P.coloff[tl]), cols = uniform(P.coloff[tl + 1]) - c0;

    const bool colu = kind == kTaskColUpdate;
    const int K = colu ? uniform(P.rowoff[si + 1] - P.rowoff[si]) : uniform(P.coloff[sl + 1] - P.coloff[sl]);
    const double tn = colu ? P.anorm[(size_t)ti * P.pt + si] : P.bnorm[(size_t)sl * P.qt + tl];
    const int VS = tile_updates(P, S) + 1;

    // scale decision (identical in every slab of this update): returns (shC, shY) and sets enew
    int enew = 0;
    double yn = 0.0;
    auto decide = [&]() -> int2 {
        const int eC = tile_exp_at(P, T, u);
        const int eY = tile_exp_at(P, S, VS);
        const double cn = tile_norm_at(P, T, u);
        yn = tile_norm_at(P, S, VS);
        const int emax = eC > eY ? eC : eY;
        const double cs = ldexp(cn, eC - emax), ys = ldexp(yn, eY - emax);
        const int sp = colu ? protect_update(cs, tn, ys) : protect_update(cs, ys, tn);
        enew = uniform(emax + sp);
        const int shC_ = uniform(eC - enew);       // <= 0
        const int shY_ = uniform(eY - enew);       // <= 0
        if (threadIdx.x == 0 && slab == 0 && (shC_ != 0 || shY_ != 0)) atomicAdd(&P.stats[1], 1u);
        return make_int2(shC_, shY_);
    };

    int rb_lo, rb_hi;
    slab_rows(rows, P.slabs, slab, &rb_lo, &rb_hi);
    const int nrb = rb_hi - rb_lo;
    double *Ct = P.C + (int64_t)c0 * P.ldc + r0;
    for (int t = threadIdx.x; t < kWaves * (kMaxTile + 3); t += kThreads) (&L.rs[0][0])[t] = 0.0;
    __syncthreads();
    if (ustamp && threadIdx.x == 0) ustamp[1] = wall_clock64();

    const bool gemm = rows > 0 && cols > 0 && nrb > 0 && K > 0;
    const int k0 = colu ? uniform(P.rowoff[si]) : uniform(P.coloff[sl]);
    const double *Aop = colu ? P.A + (int64_t)k0 * P.lda + r0 : P.C + (int64_t)k0 * P.ldc + r0;
    const double *Bop = colu ? P.C + (int64_t)c0 * P.ldc + k0 : P.B + (int64_t)c0 * P.ldb + k0;
    const int64_t lda_ = colu ? P.lda : P.ldc, ldb_ = colu ? P.ldc : P.ldb;
    int shC = 0;
    if (gemm && !(P.flags & kFlagF32Updates)) {
        // FP64: the decision runs inside, overlapped with the first operand stages
        int shY = 0;
        const UpdTerm one{uniptr(Aop), uni64(lda_), uniptr(Bop), uni64(ldb_), K, colu ? 1 : 0, 0};
        auto term = [&](int) -> UpdTerm { UpdTerm x = one; x.shY = shY; return x; };
        auto dec = [&]() -> int { const int2 d = decide(); shC = d.x; shY = d.y; return d.x; };
        const bool simple = uniform(nrb == 8 && ((cols + 15) >> 4) == 8 ? 1 : 0) != 0;
        if (colu) {
            if (simple) update_stream_f64<true, 1>(P, 1, term, Ct, rows, cols, rb_lo, nrb, L, ustamp, dec);
            else update_stream_f64<false, 1>(P, 1, term, Ct, rows, cols, rb_lo, nrb, L, ustamp, dec);
        } else {
            if (simple) update_stream_f64<true, 2>(P, 1, term, Ct, rows, cols, rb_lo, nrb, L, ustamp, dec);
            else update_stream_f64<false, 2>(P, 1, term, Ct, rows, cols, rb_lo, nrb, L, ustamp, dec);
        }
    } else {
        const int2 d = decide();
        shC = uniform(d.x);
        const int shY = uniform(d.y);
        if (gemm) {
            // normalise both operands to entries below 1 (their infinity norms bound every entry)
            // and take the product back by the shifts plus the update's scale of Y_S
            const int sT = tn > 0.0 ? -(ilogb(tn) + 1) : 0;
            const int sY = yn > 0.0 ? -(ilogb(yn) + 1) : 0;
            const int shP = uniform(shY - sT - sY);
            if (colu)
                update_passes<true, float>(P, Aop, lda_, Bop, ldb_, K, sT, sY, shP, shC, Ct, rows, cols, rb_lo, nrb, L, ustamp);
            else
                update_passes<false, float>(P, Aop, lda_, Bop, ldb_, K, sY, sT, shP, shC, Ct, rows, cols, rb_lo, nrb, L, ustamp);
        } else if (rows > 0 && cols > 0 && nrb > 0) {
            // an empty source (a tile emptied by a boundary that dodged a 2x2 block) leaves the
            // product out, but the target still moves to the common exponent and its next
            // version still needs its exact row sums
            const int srows = (16 * rb_hi < rows ? 16 * rb_hi : rows) - 16 * rb_lo;
            for (int t = threadIdx.x; t < srows; t += kThreads) {
                double rs = 0.0;
                const DevView vC = dev_view(Ct, P.ldc, rows, cols);
                for (int nn = 0; nn < cols; ++nn) {
                    const int64_t idx = (int64_t)nn * P.ldc + 16 * rb_lo + t;
                    double d = ld_dev(vC, idx);
                    if (shC != 0) {
                        d = ldexp(d, shC);
                        st_dev(vC, idx, d);
                    }
                    rs += fabs(d);
                }
                L.rs[0][t] = rs;
            }
        }
    }
    __syncthreads();
    if (ustamp && threadIdx.x == 0) ustamp[4] = wall_clock64();
    double best = 0.0;
    const int srows = (16 * rb_hi < rows ? 16 * rb_hi : rows) - 16 * rb_lo;
    for (int t = threadIdx.x; t < srows; t += kThreads) {
        double tot = 0.0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) tot += L.rs[ww][t];
        best = fmax(best, tot);
    }
    best = wg_max(best, L.red);
    if (threadIdx.x == 0) {
        tile_norm_store(P, T, u + 1, slab, best);
        tile_exp_store(P, T, u + 1, enew);
    }
    if (ustamp && threadIdx.x == 0) ustamp[5] = wall_clock64();
}

// ---------------------------------------------------------------------------------------------
// Multi-term update task: the g consecutive updates u0 .. u0 + g - 1 of target T (sources in the
// order of update_index) applied in one pass,
//     D = 2^shC C - sum_t 2^shY_t Aop_t Bop_t,
// with Aop_t Bop_t = A_ik Y_kl (column source) or Y_ij B_jl (row source).  One scale decision
// covers all terms: every operand is first brought to the common exponent emax (the largest of
// the target's and the solved tiles'), then the smallest s >= 0 with
//     2^-s (||C|| 2^(eC-emax) + sum_t ||A_t|| ||Y_t|| 2^(eY_t-emax)) <= OMEGA
// is chosen (ProtectUpdate of Algorithm 3 with the sum of the terms' bounds, which bounds every
// partial sum of the product as well), so that D = 2^-(emax+s) times the updated block.  The
// K dimensions of the terms are concatenated into one stream of 16-k stages; the target is
// read and written once.  Runs as one workgroup over the whole tile (one slab).
// ---------------------------------------------------------------------------------------------

// Sum over a 512-thread workgroup; every thread receives the result.  Two barriers.
__device__ __forceinline__ double wg_sum(double v, double *red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) r += red[i];
    __syncthreads();
    return r;
}

__device__ __noinline__ void run_update_group(const Plan &Pin, int T_, int u0_, int g_, UpdateLds &L,
                                             uint64_t *ustamp)
{
    const Plan P = uniform_plan(Pin);
    if (ustamp && threadIdx.x == 0) ustamp[0] = wall_clock64();
    const int T = uniform(T_), u0 = uniform(u0_), g = uniform(g_);
    const int ti = T / P.qt, tl = T % P.qt;
    const int r0 = uniform(P.rowoff[ti]), rows = uniform(P.rowoff[ti + 1]) - r0;
    const int c0 = uniform(P.coloff[tl]), cols = uniform(P.coloff[tl + 1]) - c0;
    // the term table, with each term's share of the scale decision (gsh holds the solved tile's
    // exponent until the decision replaces it by the shift)
    const int t = threadIdx.x;
    if (t < g) {
        int ks, ls;
        update_source(P.pt, ti, tl, u0 + t, &ks, &ls);
        const int S = ks * P.qt + ls;
        const bool col = ls == tl;
        const int k0 = col ? P.rowoff[ks] : P.coloff[ls];
        L.gS[t] = S;
        L.gk0[t] = k0;
        L.gK[t] = (col ? P.rowoff[ks + 1] : P.coloff[ls + 1]) - k0;
        L.gcol[t] = col ? 1 : 0;
        const int VS = tile_updates(P, S) + 1;
        L.gsh[t] = tile_exp_at(P, S, VS);
        L.gyn[t] = tile_norm_at(P, S, VS);
        L.gtn[t] = col ? P.anorm[(size_t)ti * P.pt + ks] : P.bnorm[(size_t)ls * P.qt + tl];
    }
    const int eC = uniform(tile_exp_at(P, T, u0));
    const double cn = unid(tile_norm_at(P, T, u0));
    for (int i = threadIdx.x; i < kWaves * (kMaxTile + 3); i += kThreads) (&L.rs[0][0])[i] = 0.0;
    __syncthreads();
    if ((P.flags & kFlagF32Updates) || rows <= 0 || cols <= 0) {
        // the FP32 form (and an empty target): the terms one after another
        for (int s = 0; s < g; ++s) {
            const int kind = uniform(L.gcol[s]) ? kTaskColUpdate : kTaskRowUpdate;
            run_update(P, kind, T, uniform(L.gS[s]), u0 + s, 0, L, ustamp);
            // this term's stores (the tile, its norm and exponent) are visible to the next term
            __builtin_amdgcn_s_waitcnt(0);
            __threadfence();
            __syncthreads();
        }
        return;
    }
    if (ustamp && threadIdx.x == 0) ustamp[1] = wall_clock64();
    // (captures only the operand bases, so that the plan's fields need not stay live in the loop)
    const double *Ab = P.A + r0, *Yc = P.C + (int64_t)c0 * P.ldc, *Yr = P.C + r0;
    const double *Bb = P.B + (int64_t)c0 * P.ldb;
    const int64_t lda = P.lda, ldc = P.ldc, ldb = P.ldb;
    UpdateLds *Lp = &L;
    auto term = [=](int s) -> UpdTerm {
        UpdTerm x;
        const int k0 = uniform(Lp->gk0[s]);
        x.K = uniform(Lp->gK[s]);
        x.col = uniform(Lp->gcol[s]);
        x.shY = uniform(Lp->gsh[s]);
        if (x.col) {
            x.Aop = Ab + (int64_t)k0 * lda; x.lda = lda;
            x.Bop = Yc + k0; x.ldb = ldc;
        } else {
            x.Aop = Yr + (int64_t)k0 * ldc; x.lda = ldc;
            x.Bop = Bb + k0; x.ldb = ldb;
        }
        return x;
    };
    // the scale decision over all terms: common exponent, then the bound at that exponent
    int enew = 0;
    auto dec = [&]() -> int {
        const int eY = t < g ? L.gsh[t] : 0;
        const double yn = t < g ? L.gyn[t] : 0.0, tn = t < g ? L.gtn[t] : 0.0;
        const int eYmax = (int)wg_max(t < g ? (double)eY : (double)eC, L.red);
        const int emax = uniform(eYmax > eC ? eYmax : eC);
        double m = 0.0;
        int E = INT32_MIN;
        if (t < g) {
            const double ys = ldexp(yn, eY - emax);
            if (tn != 0.0 && ys != 0.0) {
                const int ea = ilogb(tn), ey = ilogb(ys);
                m = ldexp(tn, -ea) * ldexp(ys, -ey);   // [1, 4)
                E = ea + ey;
            }
        } else if (t == kThreads - 1) {
            const double cs = ldexp(cn, eC - emax);
            if (cs != 0.0) {
                E = ilogb(cs);
                m = ldexp(cs, -E);
            }
        }
        const double Ed = wg_max(E == INT32_MIN ? -1.0e300 : (double)E, L.red);
        int sh = 0;
        if (uniform(Ed > -1.0e299 ? 1 : 0)) {
            // sum_t m_t 2^(E_t - Es) <= 4 (g + 1): no overflow; the margin covers its rounding
            const int Es = (int)Ed;
            const double sum = wg_sum(m != 0.0 ? ldexp(m, E - Es) : 0.0, L.red) * (1.0 + 0x1p-40);
            int cl = ilogb(sum);
            if (sum != ldexp(1.0, cl)) cl += 1;
            sh = cl + Es - 1022;
            if (sh < 0) sh = 0;
        }
        enew = uniform(emax + sh);
        if (t < g) L.gsh[t] = eY - enew;
        // every wave reads the shifts (the stage cursor fetches them next): a wave that read a
        // stale shift would take a different number of barriers in the stage loop
        __syncthreads();
        return eC - enew;
    };
    int rb_lo, rb_hi;
    slab_rows(rows, 1, 0, &rb_lo, &rb_hi);
    const int nrb = rb_hi - rb_lo;
    double *Ct = P.C + (int64_t)c0 * P.ldc + r0;
    const bool simple = uniform(nrb == 8 && ((cols + 15) >> 4) == 8 ? 1 : 0) != 0;
    if (simple) update_stream_f64<true, 0>(P, g, term, Ct, rows, cols, rb_lo, nrb, L, ustamp, dec);
    else update_stream_f64<false, 0>(P, g, term, Ct, rows, cols, rb_lo, nrb, L, ustamp, dec);
    __syncthreads();
    if (ustamp && threadIdx.x == 0) ustamp[4] = wall_clock64();
    if (threadIdx.x == 0) {
        // scaling events: every term of a group whose decision rescaled the target or a solved tile
        bool scaled = eC != enew;
        for (int s = 0; s < g; ++s) scaled = scaled || L.gsh[s] != 0;
        if (scaled) atomicAdd(&P.stats[1], (unsigned)g);
    }
    double best = 0.0;
    for (int i = threadIdx.x; i < rows; i += kThreads) {
        double tot = 0.0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) tot += L.rs[ww][i];
        best = fmax(best, tot);
    }
    best = wg_max(best, L.red);
    if (threadIdx.x == 0) {
        tile_norm_store(P, T, u0 + g, 0, best);
        tile_exp_store(P, T, u0 + g, enew);
    }
    if (ustamp && threadIdx.x == 0) ustamp[5] = wall_clock64();
}

}  // namespace trsyl
