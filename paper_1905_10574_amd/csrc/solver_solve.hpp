// Tile solve task: RobustSyl (Algorithm 2) on one tile  A_kk Y + Y B_ll = beta Y_kl.
//
// Speculative path.  The tile is cut into leaves of ~15 x 15 (a leaf boundary that would split a
// 2x2 diagonal block moves down by one row/column, so leaves are at most 16 x 16).  Leaves are
// processed by anti-diagonal fronts.  Each leaf's right-hand side is accumulated with MFMA GEMMs
// over everything already solved below it and left of it (split over idle waves on narrow
// fronts, partial sums reduced in a fixed order), then one wave solves the leaf by a wavefront
// over its 1x1/2x2 blocks.  No scaling is applied.  Instead every value that is stored (tile
// input, accumulated right-hand sides, right-hand sides after every block update, solved
// blocks) is checked against Tc = OMEGA / (64 + 8 (||A_kk||_inf + ||B_ll||_1 + ||B_ll||_inf)),
// and every pivot of a small solve must be at least smin.  Passing the check certifies that
// Algorithm 2, with ProtectUpdate fed the (valid, if pessimistic) upper bounds 2 Tc for Y-norms
// and the tile norms for the A/B panels, would choose beta = gamma_1 = gamma_2 = 1 at every
// step, that no guard inside the small solves would fire (their partial sums stay below
// (8 + 3 max|K|) Tc <= OMEGA), and that every partial sum of the GEMMs stays below OMEGA:
// Algorithm 2 then performs exactly this computation up to the order of rounding, with beta = 1.
//
// Fallback.  If the certificate fails, the tile is restored and Algorithm 2 runs as printed:
// block columns left to right, block rows bottom to top, whole-tile rescaling by beta, gamma_1,
// gamma_2 with exact Y-norms.
#pragma once
#include "device_common.hpp"
#include "plan.hpp"
#include "solver_update.hpp"
#include "solver_leaf.hpp"

namespace trsyl {

// Optional phase timestamps of the tile solve (built with -DTRSYL_PHASE_STAMPS): 80 wall-clock
// words per tile, stored after the per-task trace records.
#ifdef TRSYL_PHASE_STAMPS
#define TRSYL_STAMP(ptr, idx) \
    do { if ((ptr) && threadIdx.x == 0 && (idx) < 80) (ptr)[idx] = wall_clock64(); } while (0)
#else
#define TRSYL_STAMP(ptr, idx) do { (void)(ptr); } while (0)
#endif

// Partial-sum slots: the GEMM phase's items of the current front (at most max(kWaves, leaves),
// at most kEarlySet when the front takes part in early partials), then two sets of kEarlySet
// slots for the early partials of the next front (see tile_solve_fast).
constexpr int kEarlySet = 9;
constexpr int kMaxParts = kMaxLeaves > 3 * kEarlySet ? kMaxLeaves : 3 * kEarlySet;

struct SolveLds {
    LeafLds leaf[kWaves];
    LeafShape rs[kMaxLeaves], cs[kMaxLeaves];   // shapes of the tile's row and column leaves
    double part[kMaxParts][16 * kLd];   // split-K partial sums of the leaf GEMMs
    int la[kMaxLeaves + 1], lb[kMaxLeaves + 1];
    int nla, nlb;
    int fail;
    int ectr;            // next early-partial item (an LDS work counter)
    int tguess, tnext;   // leaf-tiled solve: growth shift to start from, and this front's largest
    union {
        struct {   // Algorithm 2 on the whole tile
            int as[kMaxTile + 1], bs[kMaxTile + 1];
            double anorm_above[kMaxTile];
            double bnorm_right[kMaxTile];
            double z[4];
            int zinfo[4];
        };
        struct {   // the leaf-tiled robust solve: per leaf (I, J) at [I * kMaxLeaves + J]
            int eL[kMaxLeaves * kMaxLeaves];        // scale exponent: the leaf holds 2^-e X_IJ
            double nL[kMaxLeaves * kMaxLeaves];     // ||Y_IJ||_inf of the stored leaf
            double nC[kMaxLeaves * kMaxLeaves];     // ||C_IJ||_inf of the tile's right-hand side
            double aN[kMaxLeaves * kMaxLeaves];     // ||A_IK||_inf, leaf blocks of A_kk (I <= K)
            double bN[kMaxLeaves * kMaxLeaves];     // ||B_LJ||_inf, leaf blocks of B_ll (L <= J)
            uint8_t rowleaf[kMaxTile + 1], colleaf[kMaxTile + 1];
        };
    };
    double red[kWaves];
};

// Leaf boundaries of the diagonal tiles A_kk (mr rows) and B_ll (nc rows), computed by one wave:
// nominal multiples of kLeaf, each moved down by one where T(b, b-1) != 0 so that no 2x2 block is
// split.  A moved boundary that reaches the tile end is dropped.  Lanes 0..31 handle A, lanes
// 32..63 handle B; the valid boundaries of each side form a prefix of the candidates.
__device__ inline void leaf_offsets_wave(const double *Ad, int64_t lda, int mr, const double *Bd,
                                         int64_t ldb, int nc, int *la, int *lb, int *nla, int *nlb)
{
    const int lane = threadIdx.x & 63;
    const bool isB = lane >= 32;
    const int k = lane & 31;
    const double *T = isB ? Bd : Ad;
    const int64_t ld = isB ? ldb : lda;
    const int len = isB ? nc : mr;
    const int b = (k + 1) * kLeaf;
    bool valid = false;
    int bb = 0;
    if (k < kMaxLeaves && b < len) {
        bb = (ldg(T + (int64_t)(b - 1) * ld + b) != 0.0) ? b + 1 : b;
        valid = bb < len;
    }
    const uint64_t mask = __ballot(valid);
    const int na = 1 + __popcll(mask & 0xFFFFFFFFull), nb = 1 + __popcll(mask >> 32);
    if (valid) (isB ? lb : la)[k + 1] = bb;
    if (lane == 0) { la[0] = 0; la[na] = mr; *nla = na; }
    if (lane == 32) { lb[0] = 0; lb[nb] = nc; *nlb = nb; }
}

// The shapes of every row leaf (of A_kk) and column leaf (of B_ll), one wave per leaf, ready
// after the closing barrier.
__device__ inline void leaf_shapes(const Plan &P, const double *Ad, const double *Bd, SolveLds &L, int nla, int nlb)
{
    const int w = uniform((int)(threadIdx.x >> 6));
    for (int I = w; I < nla; I += kWaves)
        leaf_shape_wave(Ad, P.lda, L.la[I], L.la[I + 1] - L.la[I], false, L.rs[I]);
    for (int J = w; J < nlb; J += kWaves)
        leaf_shape_wave(Bd, P.ldb, L.lb[J], L.lb[J + 1] - L.lb[J], true, L.cs[J]);
    __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// One wave accumulates acc += Aop(0:nr, k) Bop(k, 0:ncl) over k in [k0, k1), 32 k at a time, the
// next 32-k chunk's operands in flight while the current chunk's MFMAs run.  Lane (r, q) holds
// k = kc + 4q + j and kc + 16 + 4q + j for j < 4 (the MFMA's k-permutation, see mfma16).  Loads
// use clamped in-range addresses; out-of-range operands are replaced by zeros after the load.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void leaf_gemm(d4 &acc, const double *Aop, int64_t lda, int nr,
                                          const double *Bop, int64_t ldb, int ncl, int k0, int k1)
{
    const int lane = lane_here();
    const int r = lane & 15, q = lane >> 4;
    if (k0 >= k1) return;
    const bool va = r < nr, vb = r < ncl;
    const double *Ar = Aop + (va ? r : 0);
    const double *Bc = Bop + (int64_t)(vb ? r : 0) * ldb;
    double af[8], bf[8];
    // the lane's 4 k of each half of a chunk are adjacent in a column of Bop: two 16-byte loads
    // per half for a chunk that lies below k1 (global memory needs only 8-byte alignment)
    auto load = [&](int kc, double (&a)[8], double (&b)[8]) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kc + 16 * (j >> 2) + 4 * q + (j & 3);
            const int kk = k < k1 ? k : k0;
            a[j] = ldg(Ar + (int64_t)kk * lda);
        }
        if (uniform(kc + 32 <= k1 ? 1 : 0)) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int kq = kc + 16 * h + 4 * q;
                double2 x0, x1;
                __builtin_memcpy(&x0, (const gdouble *)(Bc + kq), 16);
                __builtin_memcpy(&x1, (const gdouble *)(Bc + kq + 2), 16);
                b[4 * h + 0] = x0.x; b[4 * h + 1] = x0.y; b[4 * h + 2] = x1.x; b[4 * h + 3] = x1.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kc + 16 * (j >> 2) + 4 * q + (j & 3);
                b[j] = ldg(Bc + (k < k1 ? k : k0));
            }
        }
    };
    load(k0, af, bf);
    for (int kc = k0; kc < k1; kc += 32) {
        double an[8], bn[8];
        if (kc + 32 < k1) load(kc + 32, an, bn);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kc + 16 * (j >> 2) + 4 * q + (j & 3);
            const bool kin = k < k1;
            acc = mfma16((vb && kin) ? bf[j] : 0.0, (va && kin) ? af[j] : 0.0, acc);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) { af[j] = an[j]; bf[j] = bn[j]; }
    }
}

// Two GEMM terms of at most 16 k each, A1 B1 over k in [0, k1) and A2 B2 over k in [k20, k21),
// added to acc with all their loads issued before the first MFMA (one memory round trip).  A term
// with an empty range issues no load.  Operand layouts as in leaf_gemm.
__device__ __forceinline__ void leaf_gemm_pair(d4 &acc, const double *A1, int64_t lda1, const double *B1,
                                               int64_t ldb1, int k1, const double *A2, int64_t lda2,
                                               const double *B2, int64_t ldb2, int k20, int k21, int nr, int ncl)
{
    const int lane = lane_here();
    const int r = lane & 15, q = lane >> 4;
    const bool va = r < nr, vb = r < ncl;
    const int has1 = uniform(k1 > 0 ? 1 : 0), has2 = uniform(k21 > k20 ? 1 : 0);
    double a1[4], b1[4], a2[4], b2[4];
    if (has1) {
        const double *Ar = A1 + (va ? r : 0);
        const double *Bc = B1 + (int64_t)(vb ? r : 0) * ldb1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * q + j, kk = k < k1 ? k : 0;
            a1[j] = ldg(Ar + (int64_t)kk * lda1);
            b1[j] = ldg(Bc + kk);
        }
    }
    if (has2) {
        const double *Ar = A2 + (va ? r : 0);
        const double *Bc = B2 + (int64_t)(vb ? r : 0) * ldb2;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k20 + 4 * q + j, kk = k < k21 ? k : k20;
            a2[j] = ldg(Ar + (int64_t)kk * lda2);
            b2[j] = ldg(Bc + kk);
        }
    }
    if (has1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool kin = 4 * q + j < k1;
            acc = mfma16((vb && kin) ? b1[j] : 0.0, (va && kin) ? a1[j] : 0.0, acc);
        }
    }
    if (has2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool kin = k20 + 4 * q + j < k21;
            acc = mfma16((vb && kin) ? b2[j] : 0.0, (va && kin) ? a2[j] : 0.0, acc);
        }
    }
}

// Loads the inputs of leaf (I, J) that do not depend on other leaves: its diagonal blocks into
// LL.Al / LL.Bl and its right-hand side into registers (lane (m, n0): entries (m, n0 + 4i)).
__device__ __forceinline__ void leaf_inputs(const Plan &P, const double *Ad, const double *Bd,
                                            const DevView &Y, const SolveLds &L, LeafLds &LL,
                                            int I, int J, double (&rhs)[4])
{
    const int lane = lane_here();
    const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
    const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
        const bool in = mm < nr && nn < ncl;
        const double v = ld_dev(Y, (int64_t)(lc0 + (in ? nn : 0)) * P.ldc + lr0 + (in ? mm : 0));
        rhs[i] = in ? v : 0.0;
    }
#pragma unroll
    for (int t0 = 0; t0 < 256; t0 += 64) {
        const int t = t0 + lane, rr = t & 15, cc = t >> 4;
        const bool ia = rr < nr && cc < nr && rr <= cc + 1;
        const bool ib = rr < ncl && cc < ncl && rr <= cc + 1;
        const double va = ldg(Ad + (int64_t)(lr0 + (ia ? cc : 0)) * P.lda + lr0 + (ia ? rr : 0));
        const double vb = ldg(Bd + (int64_t)(lc0 + (ib ? cc : 0)) * P.ldb + lc0 + (ib ? rr : 0));
        LL.Al[cc * kLd + rr] = ia ? va : 0.0;
        LL.Bl[cc * kLd + rr] = ib ? vb : 0.0;
    }
}

// ---------------------------------------------------------------------------------------------
// Speculative tile solve.  Y (ld ldc) holds the right-hand side and is only read; the solution
// is written to S (ld mr).  Returns 1 if certified (S holds Y with beta = 1).
// ---------------------------------------------------------------------------------------------
__device__ int tile_solve_fast(const Plan &P, const double *Ad, const double *Bd, const DevView &Y,
                               double *S, int mr_, int nc_, double smin, double Tc, SolveLds &L,
                               uint64_t *stamp)
{
    const int mr = uniform(mr_), nc = uniform(nc_);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // warm the caches with the upper parts of A_kk and B_ll (one load per 128-byte line); the
    // values are consumed by an empty asm at the end so the loads are kept
    double warm = 0.0;
    {
        const int la = (mr + 15) >> 4, lb = (nc + 15) >> 4;
        for (int t = threadIdx.x; t < mr * la + nc * lb; t += kThreads) {
            if (t < mr * la) {
                const int cc = t / la, rr = 16 * (t % la);
                if (rr <= cc + 1) warm += ldg(Ad + (int64_t)cc * P.lda + rr);
            } else {
                const int u = t - mr * la, cc = u / lb, rr = 16 * (u % lb);
                if (rr <= cc + 1) warm += ldg(Bd + (int64_t)cc * P.ldb + rr);
            }
        }
    }
    if (w == 0) leaf_offsets_wave(Ad, P.lda, mr, Bd, P.ldb, nc, L.la, L.lb, &L.nla, &L.nlb);
    if (threadIdx.x == 0) L.fail = 0;
    if (lane < 33) {                                 // zero row / column 16 of the leaf buffers
        const int o = lane < 17 ? lane * kLd + 16 : 16 * kLd + (lane - 17);
        L.leaf[w].R[o] = 0.0;
        L.leaf[w].Al[o] = 0.0;
        L.leaf[w].Bl[o] = 0.0;
    }
    __syncthreads();
    const int nla = uniform(L.nla), nlb = uniform(L.nlb);
    leaf_shapes(P, Ad, Bd, L, nla, nlb);
    const int64_t lds = mr;
    LeafLds &LL = L.leaf[w];
    int ok = 1;
    const int nfr = nla + nlb - 1;
    // Early partial sums.  While a front's leaves are solved, every wave without a leaf left
    // (at once when it has none) takes items from an LDS counter: a part of a next-front leaf's
    // right-hand-side GEMM over the leaves solved on earlier fronts (rows below the neighbour
    // below, columns left of the neighbour to the left), into the set of kEarlySet slots after
    // the current front's.  The next front's GEMM phase then only reads its two neighbours,
    // solved on the front just finished.  The two sets alternate by front parity: one is read
    // while the other is written.  Fronts of more than kEarlySet leaves take no part.
    int early = 0, ebase = kEarlySet, epe = 1;
    if (threadIdx.x == 0) L.ectr = 0;
    for (int d = 0; d < nfr; ++d) {
        const int jlo = d - (nla - 1) > 0 ? d - (nla - 1) : 0;
        const int jhi = d < nlb - 1 ? d : nlb - 1;
        const int nleaf = jhi - jlo + 1;
        const int use_early = uniform(early);
        // the GEMM phase's items per leaf, their slots li * parts + p
        const int split = use_early && 2 * nleaf <= kWaves ? 1 : 0;      // neighbour terms apart
        const int parts = use_early ? 1 + split : (nleaf >= kWaves ? 1 : kWaves / nleaf);
        double rhs[4];
        if (w < nleaf) leaf_inputs(P, Ad, Bd, Y, L, LL, nla - 1 - (d - (jlo + w)), jlo + w, rhs);
        // phase A: partial right-hand-side GEMMs, work item = leaf * parts + part
        for (int item = w; item < nleaf * parts; item += kWaves) {
            const int J = jlo + item / parts, part = item % parts;
            const int I = nla - 1 - (d - J);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
            const int kb = L.la[I + 1];
            d4 acc = zero4();
            if (use_early) {
                // the neighbour below (rows of leaf I + 1) and the one to the left (columns of
                // leaf J - 1), both solved on front d - 1; with split, one per item
                const int kb1 = (!split || part == 0) && I + 1 < nla ? L.la[I + 2] - kb : 0;
                const int kl0 = (!split || part == 1) && J > 0 ? L.lb[J - 1] : lc0;
                leaf_gemm_pair(acc, Ad + (int64_t)kb * P.lda + lr0, P.lda, S + (int64_t)lc0 * lds + kb, lds, kb1,
                               S + lr0, lds, Bd + (int64_t)lc0 * P.ldb, P.ldb, kl0, lc0, nr, ncl);
            } else {
                const int K1 = mr - kb, K2 = lc0;               // rows below, columns left
                const int nch = (K1 + 15) / 16 + (K2 + 15) / 16;
                const int c0 = (int)(((int64_t)part * nch) / parts), c1 = (int)(((int64_t)(part + 1) * nch) / parts);
                const int n1 = (K1 + 15) / 16;                  // chunks of the first term
                // first term: A(I, below) Y(below, J), chunks [c0, min(c1, n1))
                if (c0 < n1)
                    leaf_gemm(acc, Ad + (int64_t)kb * P.lda + lr0, P.lda, nr, S + (int64_t)lc0 * lds + kb,
                              lds, ncl, 16 * c0, c1 < n1 ? 16 * c1 : K1);
                // second term: Y(I, left) B(left, J), chunks [max(c0, n1), c1) shifted by n1
                if (c1 > n1) {
                    const int s0 = (c0 > n1 ? c0 : n1) - n1, s1 = c1 - n1;
                    leaf_gemm(acc, S + lr0, lds, nr, Bd + (int64_t)lc0 * P.ldb, P.ldb, ncl, 16 * s0,
                              16 * s1 < K2 ? 16 * s1 : K2);
                }
            }
            double *pp = L.part[item];
#pragma unroll
            for (int i = 0; i < 4; ++i) pp[((lane >> 4) + 4 * i) * kLd + (lane & 15)] = acc[i];
        }
        __syncthreads();
        TRSYL_STAMP(stamp, 4 + 2 * d);
        // the next front's early partials: kEarlySet items at most, pe parts per leaf
        const int d1 = d + 1;
        const int jlo1 = d1 - (nla - 1) > 0 ? d1 - (nla - 1) : 0;
        const int jhi1 = d1 < nlb - 1 ? d1 : nlb - 1;
        const int nleaf1 = d1 < nfr ? jhi1 - jlo1 + 1 : 0;
        const int next_early = uniform(nleaf1 > 0 && nleaf1 <= kEarlySet && nleaf <= kEarlySet ? 1 : 0);
        const int pe = next_early ? kEarlySet / nleaf1 : 1;
        const int nbase = kEarlySet * (1 + (d1 & 1));
        // phase B: wave k takes leaves k, k + 8, ...: fills its buffer with the leaf's right-hand
        // side minus the partial sums (added in order), solves the leaf and stores it to S.
        for (int li = w; li < nleaf; li += kWaves) {
            const int J = jlo + li, I = nla - 1 - (d - J);
            if (li >= kWaves) leaf_inputs(P, Ad, Bd, Y, L, LL, I, J, rhs);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
            const int lane = lane_here();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                double v = 0.0;
                if (mm < nr && nn < ncl) {
                    double g = 0.0;
                    for (int p = 0; p < parts; ++p) g += L.part[li * parts + p][nn * kLd + mm];
                    if (use_early)
                        for (int p = 0; p < epe; ++p) g += L.part[ebase + li * epe + p][nn * kLd + mm];
                    v = rhs[i] - g;
                    if (!(fabs(rhs[i]) <= Tc) || !(fabs(v) <= Tc)) ok = 0;
                }
                LL.R[nn * kLd + mm] = v;
            }
            wave_sync_lds();
            if (li == 0) TRSYL_STAMP(stamp, 40 + 2 * d);
            const LeafPatch PT = leaf_setup(LL, L.rs[I], L.cs[J], smin);
            if (li == 0 && d < 6) TRSYL_STAMP(stamp, 74 + d);
            if (!PT.ok) ok = 0;
            if (!leaf_solve(LL, PT, L.rs[I], L.cs[J], nr, ncl, Tc)) ok = 0;
            if (li == 0) TRSYL_STAMP(stamp, 41 + 2 * d);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                if (mm < nr && nn < ncl) stg(S + (int64_t)(lc0 + nn) * lds + lr0 + mm, LL.R[nn * kLd + mm]);
            }
        }
        if (next_early) {
            // items it = leaf * pe + part over the ranges solved on fronts up to d - 1: rows from
            // leaf I + 2 on, columns before leaf J - 1, in 16-k chunks split evenly over pe parts
            for (;;) {
                int it = 0;
                if (lane == 0) it = atomicAdd(&L.ectr, 1);
                it = __builtin_amdgcn_readfirstlane(it);
                if (it >= nleaf1 * pe) break;
                const int J = jlo1 + it / pe, part = it % pe;
                const int I = nla - 1 - (d1 - J);
                const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
                const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
                const int kb = L.la[I + 1];
                const int k1o = I + 1 < nla ? L.la[I + 2] - kb : 0, K1 = mr - kb;   // rows [k1o, K1)
                const int K2 = J > 0 ? L.lb[J - 1] : 0;                            // columns [0, K2)
                const int n1 = (K1 - k1o + 15) / 16;
                const int nch = n1 + (K2 + 15) / 16;
                const int c0 = (int)(((int64_t)part * nch) / pe), c1 = (int)(((int64_t)(part + 1) * nch) / pe);
                d4 acc = zero4();
                if (c0 < n1)
                    leaf_gemm(acc, Ad + (int64_t)kb * P.lda + lr0, P.lda, nr, S + (int64_t)lc0 * lds + kb,
                              lds, ncl, k1o + 16 * c0, c1 < n1 ? k1o + 16 * c1 : K1);
                if (c1 > n1) {
                    const int s0 = (c0 > n1 ? c0 : n1) - n1, s1 = c1 - n1;
                    leaf_gemm(acc, S + lr0, lds, nr, Bd + (int64_t)lc0 * P.ldb, P.ldb, ncl, 16 * s0,
                              16 * s1 < K2 ? 16 * s1 : K2);
                }
                // four stores written out: inside the work loop the compiler leaves a loop here
                // rolled, with a dynamic index into the accumulator
                double *pp = L.part[nbase + it] + (lane >> 4) * kLd + (lane & 15);
                pp[0] = acc[0];
                pp[4 * kLd] = acc[1];
                pp[8 * kLd] = acc[2];
                pp[12 * kLd] = acc[3];
            }
        }
        if (!ok) L.fail = 1;
        __threadfence_block();
        __syncthreads();
        TRSYL_STAMP(stamp, 5 + 2 * d);
        if (threadIdx.x == 0) L.ectr = 0;   // read again only after the next front's barrier
        early = next_early;
        ebase = nbase;
        epe = pe;
        if (uniform(L.fail)) break;
    }
    asm volatile("" ::"v"(warm));
    __syncthreads();
    return uniform(L.fail) ? 0 : 1;
}

// ---------------------------------------------------------------------------------------------
// Leaf-tiled robust tile solve: Algorithm 4 one level down, with the tile's leaves as tiles.
// Leaf (I, J) carries a scale exponent e_IJ (the stored leaf is 2^-e_IJ times the solution block
// X_IJ).  Its right-hand side C_IJ - sum_K A_IK X_KJ - sum_L X_IL B_LJ is formed at
// e_IJ = max(0, e of the sources) + s, with s >= 0 the smallest shift such that
//   2^-s (||C_IJ|| 2^-emax + sum_K ||A_IK|| ||Y_KJ|| 2^(e_KJ-emax) + sum_L ||Y_IL|| ||B_LJ|| 2^(e_IL-emax))
// is at most Tc (the bound of Algorithm 3's ProtectUpdate summed over all the update's terms,
// which also bounds every partial sum); each source enters multiplied by the exact power of two
// 2^(e_src - e_IJ) as it is loaded.  The leaf is solved by the unscaled leaf solve; if a value
// exceeds Tc, the right-hand side is divided by a further power of two chosen from the largest
// magnitude seen (a linear rescaling) and the leaf is solved again.  At the end every leaf is
// brought to the largest exponent (the consistency scaling of Algorithm 4) and that exponent is
// returned: the scratch tile then holds 2^-e X with beta = 2^-e.  Returns -1 when a pivot falls
// below smin or a leaf cannot be brought into range; the caller then runs Algorithm 2.
// ---------------------------------------------------------------------------------------------
constexpr int kML = kMaxLeaves;

__device__ __forceinline__ void lds_max_nonneg(double *p, double v)
{
    atomicMax((unsigned long long *)p, (unsigned long long)__double_as_longlong(v));
}

// Row-sum norms of the leaf blocks of a rows x cols matrix (only columns c >= r - 1 of row r when
// upper), max-reduced per (row leaf, column leaf) into out[I * kML + J].  Thread t takes the
// (row, column leaf) items t, t + kThreads, ... with the row running fastest, so a column's rows
// are read by consecutive threads; X(r, c) = get(r, c).
template <class Get>
__device__ __forceinline__ void leaf_block_norms(int rows, int cols, bool upper, const uint8_t *rleaf,
                                                 const int *cb, int ncb, double *out, Get get)
{
    for (int it = threadIdx.x; it < rows * ncb; it += kThreads) {
        const int r = it % rows, J = it / rows;
        int c = cb[J];
        const int c1 = cb[J + 1] < cols ? cb[J + 1] : cols;
        if (upper && c < r - 1) c = r - 1;
        double s = 0.0;
        for (; c < c1; ++c) s += fabs(get(r, c));
        lds_max_nonneg(&out[rleaf[r] * kML + J], s);
    }
}

// e_IJ from the LDS state of the solved sources (see above).
__device__ __forceinline__ int leaf_exponent(const SolveLds &L, int I, int J, int nla, double Tc)
{
    int emax = 0;
    for (int K = I + 1; K < nla; ++K) emax = max(emax, L.eL[K * kML + J]);
    for (int Lc = 0; Lc < J; ++Lc) emax = max(emax, L.eL[I * kML + Lc]);
    // the bound times 2^-64 (every factor below 2^(1024-32), so nothing overflows)
    double b = ldexp(L.nC[I * kML + J], -emax - 64);
    for (int K = I + 1; K < nla; ++K)
        b += ldexp(L.aN[I * kML + K], -32) * ldexp(L.nL[K * kML + J], L.eL[K * kML + J] - emax - 32);
    for (int Lc = 0; Lc < J; ++Lc)
        b += ldexp(L.nL[I * kML + Lc], L.eL[I * kML + Lc] - emax - 32) * ldexp(L.bN[Lc * kML + J], -32);
    const double t = ldexp(Tc, -64);
    int s = 0;
    if (b > t) {
        // start from the exponent difference when both are finite and nonzero; the loop is
        // bounded whatever the values (2200 shifts take any double below any positive t)
        if (t > 0.0 && b <= 0x1.fffffffffffffp1023) s = max(ilogb(b) - ilogb(t), 0);
        while (s < 2200 && ldexp(b, -s) > t) ++s;
    }
    return emax + s;
}

// As leaf_gemm, with the solved-tile operand (the A operand when scale_a, else the B operand)
// multiplied on load by the exact power of two 2^(eL[kleaf[kbase + k] * mul + add] - e_t).
__device__ __forceinline__ void leaf_gemm_scaled(d4 &acc, const double *Aop, int64_t lda, int nr,
                                                 const double *Bop, int64_t ldb, int ncl, int k0, int k1,
                                                 bool scale_a, const uint8_t *kleaf, int kbase, int mul,
                                                 int add, const int *eL, int e_t)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    if (k0 >= k1) return;
    const bool va = r < nr, vb = r < ncl;
    const double *Ar = Aop + (va ? r : 0);
    const double *Bc = Bop + (int64_t)(vb ? r : 0) * ldb;
    for (int kc = k0; kc < k1; kc += 32) {
        double af[8], bf[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kc + 16 * (j >> 2) + 4 * q + (j & 3);
            const int kk = k < k1 ? k : k0;
            const int ex = eL[kleaf[kbase + kk] * mul + add] - e_t;
            const double a = ldg(Ar + (int64_t)kk * lda), b = ldg(Bc + kk);
            af[j] = scale_a ? ldexp(a, ex) : a;
            bf[j] = scale_a ? b : ldexp(b, ex);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kc + 16 * (j >> 2) + 4 * q + (j & 3);
            const bool kin = k < k1;
            acc = mfma16((vb && kin) ? bf[j] : 0.0, (va && kin) ? af[j] : 0.0, acc);
        }
    }
}

__device__ int tile_solve_scaled(const Plan &P, const double *Ad, const double *Bd, const DevView &Y,
                                 double *S, int mr_, int nc_, double smin, double Tc, SolveLds &L,
                                 uint64_t *stamp)
{
    const int mr = uniform(mr_), nc = uniform(nc_);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (w == 0) leaf_offsets_wave(Ad, P.lda, mr, Bd, P.ldb, nc, L.la, L.lb, &L.nla, &L.nlb);
    if (threadIdx.x == 0) {
        L.fail = 0;
        L.tguess = 0;
        L.tnext = 0;
    }
    if (lane < 33) {                                 // zero row / column 16 of the leaf buffers
        const int o = lane < 17 ? lane * kLd + 16 : 16 * kLd + (lane - 17);
        L.leaf[w].R[o] = 0.0;
        L.leaf[w].Al[o] = 0.0;
        L.leaf[w].Bl[o] = 0.0;
    }
    for (int t = threadIdx.x; t < kML * kML; t += kThreads) {
        L.eL[t] = 0;
        L.nL[t] = 0.0;
        L.nC[t] = 0.0;
        L.aN[t] = 0.0;
        L.bN[t] = 0.0;
    }
    __syncthreads();
    const int nla = uniform(L.nla), nlb = uniform(L.nlb);
    leaf_shapes(P, Ad, Bd, L, nla, nlb);
    for (int r = threadIdx.x; r < mr; r += kThreads) {
        int I = 0;
        while (L.la[I + 1] <= r) ++I;
        L.rowleaf[r] = (uint8_t)I;
    }
    for (int c = threadIdx.x; c < nc; c += kThreads) {
        int J = 0;
        while (L.lb[J + 1] <= c) ++J;
        L.colleaf[c] = (uint8_t)J;
    }
    __syncthreads();
    leaf_block_norms(mr, nc, false, L.rowleaf, L.lb, nlb, L.nC,
                     [&](int r, int c) { return ld_dev(Y, (int64_t)c * P.ldc + r); });
    leaf_block_norms(mr, mr, true, L.rowleaf, L.la, nla, L.aN,
                     [&](int r, int c) { return ldg(Ad + (int64_t)c * P.lda + r); });
    leaf_block_norms(nc, nc, true, L.colleaf, L.lb, nlb, L.bN,
                     [&](int r, int c) { return ldg(Bd + (int64_t)c * P.ldb + r); });
    __syncthreads();
    const int64_t lds = mr;
    LeafLds &LL = L.leaf[w];
    int ok = 1;
    for (int d = 0; d < nla + nlb - 1; ++d) {
        const int jlo = d - (nla - 1) > 0 ? d - (nla - 1) : 0;
        const int jhi = d < nlb - 1 ? d : nlb - 1;
        const int nleaf = jhi - jlo + 1;
        const int parts = nleaf >= kWaves ? 1 : kWaves / nleaf;
        double rhs[4];
        if (w < nleaf) leaf_inputs(P, Ad, Bd, Y, L, LL, nla - 1 - (d - (jlo + w)), jlo + w, rhs);
        // phase A: scaled partial right-hand-side GEMMs
        for (int item = w; item < nleaf * parts; item += kWaves) {
            const int J = jlo + item / parts, part = item % parts;
            const int I = nla - 1 - (d - J);
            const int e_t = leaf_exponent(L, I, J, nla, Tc);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
            const int kb = L.la[I + 1];
            const int K1 = mr - kb, K2 = lc0;
            const int nch = (K1 + 15) / 16 + (K2 + 15) / 16;
            const int c0 = (int)(((int64_t)part * nch) / parts), c1 = (int)(((int64_t)(part + 1) * nch) / parts);
            const int n1 = (K1 + 15) / 16;
            d4 acc = zero4();
            if (c0 < n1)       // A(I, below) (2^(e_KJ - e) Y(below, J)): row leaf K of source row kb + k
                leaf_gemm_scaled(acc, Ad + (int64_t)kb * P.lda + lr0, P.lda, nr, S + (int64_t)lc0 * lds + kb,
                                 lds, ncl, 16 * c0, c1 < n1 ? 16 * c1 : K1, false, L.rowleaf, kb, kML, J,
                                 L.eL, e_t);
            if (c1 > n1) {     // (2^(e_IL - e) Y(I, left)) B(left, J): column leaf of source column k
                const int s0 = (c0 > n1 ? c0 : n1) - n1, s1 = c1 - n1;
                leaf_gemm_scaled(acc, S + lr0, lds, nr, Bd + (int64_t)lc0 * P.ldb, P.ldb, ncl, 16 * s0,
                                 16 * s1 < K2 ? 16 * s1 : K2, true, L.colleaf, 0, 1, I * kML, L.eL, e_t);
            }
            double *pp = L.part[item];
#pragma unroll
            for (int i = 0; i < 4; ++i) pp[((lane >> 4) + 4 * i) * kLd + (lane & 15)] = acc[i];
        }
        __syncthreads();
        TRSYL_STAMP(stamp, 4 + 2 * d);
        // phase B: each wave fills, solves (with power-of-two retries) and stores its leaves
        for (int li = w; li < nleaf; li += kWaves) {
            const int J = jlo + li, I = nla - 1 - (d - J);
            if (li >= kWaves) leaf_inputs(P, Ad, Bd, Y, L, LL, I, J, rhs);
            int e = leaf_exponent(L, I, J, nla, Tc);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
            // the first try is scaled by the largest growth shift the previous front needed (a
            // guess: the leaf's own growth is unknown until it is solved once)
            int t = uniform(L.tguess);
            double v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                v[i] = 0.0;
                if (mm < nr && nn < ncl) {
                    double g = 0.0;
                    for (int p = 0; p < parts; ++p) g += L.part[li * parts + p][nn * kLd + mm];
                    v[i] = ldexp(rhs[i], -e) - g;
                    if (!(fabs(v[i]) <= Tc)) ok = 0;
                }
                LL.R[nn * kLd + mm] = ldexp(v[i], -t);
            }
            wave_sync_lds();
            if (li == 0) TRSYL_STAMP(stamp, 40 + 2 * d);
            const LeafPatch PT = leaf_setup(LL, L.rs[I], L.cs[J], smin);
            if (!PT.ok) ok = 0;
            bool done = false, blind = t > 0;
            for (int attempt = 0; attempt < 8 && uniform(__all(ok)); ++attempt) {
                double vm;
                if (!leaf_solve(LL, PT, L.rs[I], L.cs[J], nr, ncl, Tc, &vm)) ok = 0;
                vm = wave_max(vm);
                if (vm <= Tc) {
                    // after a blind shift (a guessed one, or the previous try overflowed), move
                    // the largest value back up to about Tc / 4 so the leaf is not scaled further
                    // than needed (never below the shift the bound chose)
                    const int gap = vm > 0.0 ? ilogb(Tc) - ilogb(vm) - 2 : 0;
                    const int tn = t - gap > 0 ? t - gap : 0;
                    if (!(blind && gap > 8 && tn != t)) { done = true; break; }
                    blind = false;
                    t = tn;
                } else {
                    // linear in the right-hand side: shift it so the largest value lands below
                    // Tc / 2; an overflowed try gives no magnitude, so shift blindly
                    blind = !(vm <= 0x1.fffffffffffffp+1023);
                    t += blind ? 256 : max(1, ilogb(vm) - ilogb(Tc) + 2);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                    LL.R[nn * kLd + mm] = ldexp(v[i], -t);
                }
                wave_sync_lds();
            }
            if (!done) ok = 0;
            e += t;
            if (lane == 0 && t > 0) atomicMax(&L.tnext, t);
            if (li == 0) TRSYL_STAMP(stamp, 41 + 2 * d);
            // the leaf's infinity norm
            double rs = 0.0;
            if (lane < nr)
                for (int cc = 0; cc < ncl; ++cc) rs += fabs(LL.R[cc * kLd + lane]);
            rs = wave_max(rs);
            if (lane == 0) {
                L.eL[I * kML + J] = e;
                L.nL[I * kML + J] = rs;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                if (mm < nr && nn < ncl) stg(S + (int64_t)(lc0 + nn) * lds + lr0 + mm, LL.R[nn * kLd + mm]);
            }
        }
        if (!ok) L.fail = 1;
        __threadfence_block();
        __syncthreads();
        TRSYL_STAMP(stamp, 5 + 2 * d);
        if (uniform(L.fail)) break;
        if (threadIdx.x == 0) {      // read after the next front's first barrier
            L.tguess = L.tnext;
            L.tnext = 0;
        }
    }
    __syncthreads();
    if (uniform(L.fail)) return -1;
    // consistency: every leaf to the largest exponent
    int et = 0;
    for (int I = 0; I < nla; ++I)
        for (int J = 0; J < nlb; ++J) et = max(et, L.eL[I * kML + J]);
    et = uniform(et);
    for (int t = threadIdx.x; t < mr * nc; t += kThreads) {
        const int rr = t % mr, cc = t / mr;
        const int ex = L.eL[L.rowleaf[rr] * kML + L.colleaf[cc]] - et;
        if (ex != 0) {
            double *p = S + (int64_t)cc * lds + rr;
            stg(p, ldexp(ldg(p), ex));
        }
    }
    __threadfence_block();
    __syncthreads();
    return et;
}

// ---------------------------------------------------------------------------------------------
// ||Y||_inf of an mr x nc tile read from src (ld lsrc), optionally copying it to dst (ld ldst)
// on the way.  Thread t sums row t % mr over the columns congruent to t / mr, so consecutive
// threads read consecutive rows; the partial row sums meet in LDS.  dst, when given, is shared
// with other workgroups and written with device-scope stores.
// ---------------------------------------------------------------------------------------------
__device__ double tile_norm_copy(const double *src, int64_t lsrc, const DevView *dst, int64_t ldst,
                                 int mr, int nc, SolveLds &L)
{
    double *part = &L.part[0][0];                    // kThreads doubles of scratch
    const int g = mr <= kThreads ? kThreads / mr : 1;
    const int t = threadIdx.x, rr = t % mr, p = t / mr;
    double s = 0.0;
    if (p < g) {
        // eight columns' loads issued before their stores (a store may alias a later load, so
        // one column at a time would cost a memory round trip each); the sum keeps column order
        for (int c0 = p; c0 < nc; c0 += 8 * g) {
            double v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int cc = c0 + j * g;
                v[j] = cc < nc ? ldg(src + (int64_t)cc * lsrc + rr) : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int cc = c0 + j * g;
                if (cc < nc) {
                    if (dst) st_dev(*dst, (int64_t)cc * ldst + rr, v[j]);
                    s += fabs(v[j]);
                }
            }
        }
    }
    part[t] = s;
    __syncthreads();
    double v = 0.0;
    if (t < mr) {
        double rs = 0.0;
        for (int u = 0; u < g; ++u) rs += part[u * mr + t];
        v = rs;
    }
    __syncthreads();
    return wg_max(v, L.red);
}

// The smallest s >= 0 with 2^-s ||Y||_inf <= OMEGA for an mr x nc tile (ld ldy) whose entries are
// at most OMEGA each: row sums are formed from 2^-16 |y|, which cannot overflow.
__device__ int tile_excess_shift(const double *Y, int64_t ldy, int mr, int nc, SolveLds &L)
{
    double g = 0.0;
    for (int r = threadIdx.x; r < mr; r += kThreads) {
        double t = 0.0;
        for (int c = 0; c < nc; ++c) t += ldexp(fabs(ldg(Y + (int64_t)c * ldy + r)), -16);
        g = fmax(g, t);
    }
    g = wg_max(g, L.red);
    int s = 0;
    while (s < 2200 && ldexp(g, 16 - s) > kOmega) ++s;
    return s;
}

// ---------------------------------------------------------------------------------------------
// Algorithm 2 as printed, on one tile, by the whole workgroup.  Returns the exponent of beta.
// ---------------------------------------------------------------------------------------------
__device__ void scale_tile(double *Y, int64_t ldc, int mr, int nc, int s)
{
    for (int t = threadIdx.x; t < mr * nc; t += kThreads) {
        const int rr = t % mr, cc = t / mr;
        double *p = Y + (int64_t)cc * ldc + rr;
        *p = ldexp(*p, -s);
    }
    __threadfence_block();
    __syncthreads();
}

__device__ int tile_solve_robust(const Plan &P, const double *Ad, const double *Bd, double *Y, int64_t ldy,
                                 int mr_, int nc_, double smin, SolveLds &L, int *pert)
{
    const int mr = uniform(mr_), nc = uniform(nc_);
    const int tid = threadIdx.x;
    if (tid == 0) {
        int na = 0, i = 0;
        while (i < mr) {
            L.as[na++] = i;
            i += (i + 1 < mr && Ad[(int64_t)i * P.lda + i + 1] != 0.0) ? 2 : 1;
        }
        L.as[na] = mr;
        L.nla = na;
        int nb = 0;
        i = 0;
        while (i < nc) {
            L.bs[nb++] = i;
            i += (i + 1 < nc && Bd[(int64_t)i * P.ldb + i + 1] != 0.0) ? 2 : 1;
        }
        L.bs[nb] = nc;
        L.nlb = nb;
    }
    __syncthreads();
    const int na = uniform(L.nla), nb = uniform(L.nlb);
    // ||A(0:as[k], block k)||_inf and max_{j>l} ||B(block l, block j)||_inf
    for (int k = tid; k < na; k += kThreads) {
        const int c0 = L.as[k], c1 = L.as[k + 1];
        double best = 0.0;
        for (int r = 0; r < c0; ++r) {
            double s = 0.0;
            for (int cc = c0; cc < c1; ++cc) s += fabs(Ad[(int64_t)cc * P.lda + r]);
            best = fmax(best, s);
        }
        L.anorm_above[k] = best;
    }
    for (int l = tid; l < nb; l += kThreads) {
        const int r0 = L.bs[l], r1 = L.bs[l + 1];
        double best = 0.0;
        for (int j = l + 1; j < nb; ++j) {
            for (int r = r0; r < r1; ++r) {
                double s = 0.0;
                for (int cc = L.bs[j]; cc < L.bs[j + 1]; ++cc) s += fabs(Bd[(int64_t)cc * P.ldb + r]);
                best = fmax(best, s);
            }
        }
        L.bnorm_right[l] = best;
    }
    __syncthreads();
    int e = 0;
    for (int lb = 0; lb < nb; ++lb) {
        const int cb0 = uniform(L.bs[lb]), cb1 = uniform(L.bs[lb + 1]), csz = cb1 - cb0;
        for (int ka = na - 1; ka >= 0; --ka) {
            const int ra0 = uniform(L.as[ka]), ra1 = uniform(L.as[ka + 1]), rsz = ra1 - ra0;
            if (tid == 0) {
                double a[4], b[4], z[4];
                for (int t = 0; t < 4; ++t) {
                    const int p = t & 1, pp = t >> 1;
                    a[t] = (p < rsz && pp < rsz) ? Ad[(int64_t)(ra0 + pp) * P.lda + ra0 + p] : 0.0;
                    b[t] = (p < csz && pp < csz) ? Bd[(int64_t)(cb0 + pp) * P.ldb + cb0 + p] : 0.0;
                    z[t] = (p < rsz && pp < csz) ? Y[(int64_t)(cb0 + pp) * ldy + ra0 + p] : 0.0;
                }
                const int sb = small_solve(rsz, csz, a, b, z, smin, pert);
                for (int t = 0; t < 4; ++t) L.z[t] = z[t];
                L.zinfo[0] = sb;
            }
            __syncthreads();
            const int sb = uniform(L.zinfo[0]);
            if (sb) { scale_tile(Y, ldy, mr, nc, sb); e += sb; }     // Y <- beta Y
            if (tid == 0) {
                for (int t = 0; t < 4; ++t) {
                    const int p = t & 1, pp = t >> 1;
                    if (p < rsz && pp < csz) Y[(int64_t)(cb0 + pp) * ldy + ra0 + p] = L.z[t];
                }
            }
            __threadfence_block();
            __syncthreads();
            auto znorm = [&]() {
                double best = 0.0;
                for (int p = 0; p < rsz; ++p) {
                    double s = 0.0;
                    for (int pp = 0; pp < csz; ++pp) s += fabs(Y[(int64_t)(cb0 + pp) * ldy + ra0 + p]);
                    best = fmax(best, s);
                }
                return best;
            };
            if (ra0 > 0) {                                               // column update
                double v = 0.0;
                for (int r = tid; r < ra0; r += kThreads) {
                    double s = 0.0;
                    for (int cc = cb0; cc < cb1; ++cc) s += fabs(Y[(int64_t)cc * ldy + r]);
                    v = fmax(v, s);
                }
                const double ynorm = wg_max(v, L.red);
                const int s1 = uniform(protect_update(ynorm, L.anorm_above[ka], znorm()));
                if (s1) { scale_tile(Y, ldy, mr, nc, s1); e += s1; }
                for (int r = tid; r < ra0; r += kThreads) {
                    for (int cc = cb0; cc < cb1; ++cc) {
                        double acc = Y[(int64_t)cc * ldy + r];
                        for (int rr = ra0; rr < ra1; ++rr)
                            acc = fma(-Ad[(int64_t)rr * P.lda + r], Y[(int64_t)cc * ldy + rr], acc);
                        Y[(int64_t)cc * ldy + r] = acc;
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
            if (lb + 1 < nb) {                                           // row update
                double v = 0.0;
                for (int j = lb + 1 + tid; j < nb; j += kThreads) {
                    for (int p = ra0; p < ra1; ++p) {
                        double s = 0.0;
                        for (int cc = L.bs[j]; cc < L.bs[j + 1]; ++cc) s += fabs(Y[(int64_t)cc * ldy + p]);
                        v = fmax(v, s);
                    }
                }
                const double ynorm = wg_max(v, L.red);
                const int s2 = uniform(protect_update(ynorm, znorm(), L.bnorm_right[lb]));
                if (s2) { scale_tile(Y, ldy, mr, nc, s2); e += s2; }
                for (int cc = cb1 + tid; cc < nc; cc += kThreads) {
                    for (int p = ra0; p < ra1; ++p) {
                        double acc = Y[(int64_t)cc * ldy + p];
                        for (int c2 = cb0; c2 < cb1; ++c2)
                            acc = fma(-Y[(int64_t)c2 * ldy + p], Bd[(int64_t)cc * P.ldb + c2], acc);
                        Y[(int64_t)cc * ldy + p] = acc;
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
    }
    return e;
}

// ---------------------------------------------------------------------------------------------
// Solve task for tile T (after all of its updates; reads version U, writes version U + 1).
// ---------------------------------------------------------------------------------------------
__device__ __noinline__ void run_solve(const Plan &Pin, int T_, double *scratch_, SolveLds &L)
{
    const Plan P = uniform_plan(Pin);
    double *scratch = uniptr(scratch_);
    const int T = uniform(T_);     // see run_update: keep barrier-enclosing branches uniform
    const int ti = T / P.qt, tl = T % P.qt;
    const int r0 = uniform(P.rowoff[ti]), mr = uniform(P.rowoff[ti + 1]) - r0;
    const int c0 = uniform(P.coloff[tl]), nc = uniform(P.coloff[tl + 1]) - c0;
    const int U = tile_updates(P, T);
    const int e_in = tile_exp_at(P, T, U);
    int e_syl = 0;
    double nrm = 0.0;
    int pert = 0;
#ifdef TRSYL_PHASE_STAMPS
    uint64_t *stamp = P.trace ? P.trace + 4 * (size_t)max_tasks(P) + 80 * (size_t)T : nullptr;
#else
    uint64_t *stamp = nullptr;
#endif
    TRSYL_STAMP(stamp, 0);
    if (mr > 0 && nc > 0) {
        const double *Ad = P.A + (int64_t)r0 * P.lda + r0;
        const double *Bd = P.B + (int64_t)c0 * P.ldb + c0;
        double *Y = P.C + (int64_t)c0 * P.ldc + r0;
        // the pivot floor and the certificate's bound are the same in every lane: kept in
        // scalar registers
        double smin = 0x1p-52 * (*P.gmax);
        if (smin < 0x1p-1022) smin = 0x1p-1022;
        smin = unid(smin);
        const double dA = P.anorm[(size_t)ti * P.pt + ti];
        const double dB = P.bnorm[(size_t)tl * P.qt + tl];
        const double dB1 = P.bdiag1[tl];
        // OMEGA / (64 + 8 (dA + dB1 + dB)), formed with every term halved (the same quotient,
        // rounding included): with dA, dB <= OMEGA the sum overflows only if the 1-norm dB1 does,
        // and then Tc = 0 keeps the speculative paths off
        const double Tc = unid((kOmega * 0x1p-4) / (4.0 + ((0.5 * dA + 0.5 * dB1) + 0.5 * dB)));
        const DevView vY = dev_view(Y, P.ldc, mr, nc);
        int done = 0;
        // the unguarded small solves assume unscaled Kronecker entries: max|A|,|B| < 2^1016, and
        // the certificate a bound of at least one (below it, tile norms within a few powers of two
        // of OMEGA, values of order one would fail it or force the leaf-tiled solve to rescale;
        // Algorithm 2 as printed needs no such margin).  The tests are made wave-uniform: both
        // branches below enclose barriers.  A tile
        // whose updates already had to scale it (e_in > 0) goes straight to the leaf-tiled robust
        // solve: growth upstream predicts growth inside the tile, where the speculative attempt
        // would run several fronts before its certificate fails.  e_in is fixed by the update
        // order, so the choice (and the result) does not depend on timing.
        const int spec = uniform(!(P.flags & kFlagRobustSolve) && *P.gmax < 0x1p1016 && Tc >= 1.0 ? 1 : 0);
        const int try_fast = uniform(spec && e_in == 0 ? 1 : 0);
        if (try_fast)
            done = uniform(tile_solve_fast(P, Ad, Bd, vY, scratch, mr, nc, smin, Tc, L, stamp));
        TRSYL_STAMP(stamp, 2);
        if (!done && spec) {
            // the leaf-tiled robust solve (the fast path left Y untouched)
            if (threadIdx.x == 0) atomicAdd(&P.stats[2], 1u);
            const int es = uniform(tile_solve_scaled(P, Ad, Bd, vY, scratch, mr, nc, smin, Tc, L, stamp));
            if (es >= 0) {
                e_syl = es;
                done = 1;
            }
        }
        if (!done) {
            // Algorithm 2 on a private copy of the tile (the fast paths left Y untouched)
            if (threadIdx.x == 0) atomicAdd(&P.stats[0], 1u);
            for (int t = threadIdx.x; t < mr * nc; t += kThreads) {
                const int rr = t % mr, cc = t / mr;
                scratch[t] = ld_dev(vY, (int64_t)cc * P.ldc + rr);
            }
            __threadfence_block();
            __syncthreads();
            e_syl = tile_solve_robust(P, Ad, Bd, scratch, mr, mr, nc, smin, L, &pert);
        }
        nrm = tile_norm_copy(scratch, mr, &vY, P.ldc, mr, nc, L);   // publish the tile, exact norm
        // Algorithm 2 bounds the tile's 1x1 / 2x2 blocks only; Algorithm 4 needs ||Y_kl||_inf <=
        // OMEGA (its postcondition and Algorithm 3's precondition).  A tile above it (or whose
        // row sums overflowed) is scaled by the smallest power of two that restores the bound,
        // folded into the tile's scale, and published again.
        if (uniform(!(nrm <= kOmega) ? 1 : 0)) {
            const int sx = uniform(tile_excess_shift(scratch, mr, mr, nc, L));
            scale_tile(scratch, mr, mr, nc, sx);
            nrm = tile_norm_copy(scratch, mr, &vY, P.ldc, mr, nc, L);
            e_syl += sx;
        }
        TRSYL_STAMP(stamp, 3);
    }
    if (pert) set_status(P.status, kPerturbed);
    if (threadIdx.x == 0) {
        tile_norm_store(P, T, U + 1, 0, nrm);
        for (int s = 1; s < P.slabs; ++s) tile_norm_store(P, T, U + 1, s, 0.0);
        tile_exp_store(P, T, U + 1, e_in + e_syl);
    }
}

}  // namespace trsyl
