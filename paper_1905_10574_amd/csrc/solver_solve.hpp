// Tile solve task: RobustSyl (Algorithm 2) on one tile  A_kk Y + Y B_ll = beta Y_kl.
//
// Speculative path.  The tile is cut into leaves of ~15 x 15 (a leaf boundary that would split a
// 2x2 diagonal block moves down by one row/column, so leaves are at most 16 x 16).  Leaves are
// processed by anti-diagonal fronts; each wave takes whole leaves: it accumulates the leaf's
// right-hand side with one MFMA GEMM over everything already solved below it and left of it,
// then solves the leaf by a wavefront over its 1x1/2x2 blocks.  No scaling is applied; instead
// every value that is stored (right-hand sides after accumulation and after every block
// update, solved blocks) is checked against a threshold Tc, and every small solve must need no
// guard.  With Tc = OMEGA / (2 + 2||A_kk||_inf + 2||B_ll||_1 + 2||B_ll||_inf), passing the check
// certifies that every ProtectUpdate of Algorithm 2, fed with the upper bounds 2 Tc for the
// Y-norms and the tile norms for the A/B panels, returns 1, and that every partial sum stays
// below OMEGA; Algorithm 2 with those (valid, if pessimistic) bounds then performs exactly this
// computation up to the order of rounding, with beta = 1.
//
// Fallback.  If the certificate fails, the tile is restored and Algorithm 2 runs as printed:
// block columns left to right, block rows bottom to top, whole-tile rescaling by beta, gamma_1,
// gamma_2 with exact Y-norms.
#pragma once
#include "device_common.hpp"
#include "plan.hpp"
#include "solver_update.hpp"

namespace trsyl {

constexpr int kLd = 17;   // leading dimension of the per-wave 16x16 LDS buffers

struct LeafLds {
    double R[16 * kLd];
    double Al[16 * kLd];
    double Bl[16 * kLd];
    int rI[16], cJ[16], rst[17], cst[17];
};

struct SolveLds {
    LeafLds leaf[kWaves];
    int la[kMaxLeaves + 1], lb[kMaxLeaves + 1];
    int nla, nlb;
    int fail;
    // fallback
    int as[kMaxTile + 1], bs[kMaxTile + 1];
    double anorm_above[kMaxTile];
    double bnorm_right[kMaxTile];
    double z[4];
    int zinfo[4];
    double red[kWaves];
};

// Leaf boundaries of a diagonal tile with `len` rows: nominal multiples of kLeaf, moved down by
// one where T(b, b-1) != 0.  Returns the leaf count; off[count] = len.
__device__ inline int leaf_offsets(const double *T, int64_t ld, int len, int *off)
{
    int cnt = 0;
    off[cnt++] = 0;
    for (int b = kLeaf; b < len; b += kLeaf) {
        int bb = (T[(int64_t)(b - 1) * ld + b] != 0.0) ? b + 1 : b;
        if (bb >= len) break;
        off[cnt++] = bb;
    }
    off[cnt] = len;
    return cnt;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------------------------
// Leaf solve (one wave): A_l Y + Y B_l = R on a leaf of nr x nc <= 16 x 16 held in L.R (ld 17),
// with A_l, B_l in L.Al, L.Bl.  Block anti-diagonals; the lane owning a block's top-left entry
// solves it, then every pending entry takes the contributions of the blocks just solved in its
// block column (below) and block row (left).  Lane (c = lane & 15, q = lane >> 4) owns rows
// q, q+4, q+8, q+12 of column c.  Returns 1 if the certificate held.
// ---------------------------------------------------------------------------------------------
__device__ int leaf_solve(LeafLds &L, int nr, int nc, double smin, double Tc, int *pert)
{
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, q = lane >> 4;
    // block structure from the subdiagonals (ballot over rows / columns)
    const bool rstart = (lane < nr) && (lane == 0 || L.Al[(lane - 1) * kLd + lane] == 0.0);
    const bool cstart = (lane < nc) && (lane == 0 || L.Bl[(lane - 1) * kLd + lane] == 0.0);
    const uint64_t rmask = __ballot(rstart), cmask = __ballot(cstart);
    const int na = __popcll(rmask), nb = __popcll(cmask);
    if (lane < nr) L.rI[lane] = __popcll(rmask & ((2ull << lane) - 1)) - 1;
    if (lane < nc) L.cJ[lane] = __popcll(cmask & ((2ull << lane) - 1)) - 1;
    if (rstart) L.rst[__popcll(rmask & ((1ull << lane) - 1))] = lane;
    if (cstart) L.cst[__popcll(cmask & ((1ull << lane) - 1))] = lane;
    if (lane == 0) { L.rst[na] = nr; L.cst[nb] = nc; }
    wave_sync_lds();

    int ok = 1;
    double acc[4];
    int Ir[4];
    const int Jc = (c < nc) ? L.cJ[c] : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = q + 4 * i;
        acc[i] = (r < nr && c < nc) ? L.R[c * kLd + r] : 0.0;
        Ir[i] = (r < nr) ? L.rI[r] : 0;
    }
    const int steps = na + nb - 1;
    for (int s = 0; s < steps; ++s) {
        // publish right-hand sides of the blocks finalised at this step
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = q + 4 * i;
            if (r < nr && c < nc && (na - 1 - Ir[i]) + Jc == s) L.R[c * kLd + r] = acc[i];
        }
        wave_sync_lds();
        // owners solve their block
        if (c < nc && c == L.cst[Jc]) {
            const int I = na - 1 - (s - Jc);
            if (I >= 0 && I < na && (L.rst[I] & 3) == q) {
                const int ra = L.rst[I], rsz = L.rst[I + 1] - ra;
                const int csz = L.cst[Jc + 1] - c;
                double a[4], b[4], z[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int p = t & 1, pp = t >> 1;   // column-major 2x2: (p, pp)
                    a[t] = (p < rsz && pp < rsz) ? L.Al[(ra + pp) * kLd + ra + p] : 0.0;
                    b[t] = (p < csz && pp < csz) ? L.Bl[(c + pp) * kLd + c + p] : 0.0;
                    z[t] = (p < rsz && pp < csz) ? L.R[(c + pp) * kLd + ra + p] : 0.0;
                }
                const int sb = small_solve(rsz, csz, a, b, z, smin, pert);
                if (sb != 0) ok = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int p = t & 1, pp = t >> 1;
                    if (p < rsz && pp < csz) {
                        if (!(fabs(z[t]) <= Tc)) ok = 0;
                        L.R[(c + pp) * kLd + ra + p] = z[t];
                    }
                }
            }
        }
        wave_sync_lds();
        // contributions of the blocks solved at step s
        const int Is = na - 1 - (s - Jc);              // solved block in my block column
        const bool colsrc = (c < nc) && Is >= 0 && Is < na;
        const int rs0 = colsrc ? L.rst[Is] : 0, rs1 = colsrc ? L.rst[Is + 1] : 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = q + 4 * i;
            if (r >= nr || c >= nc) continue;
            if ((na - 1 - Ir[i]) + Jc <= s) continue;     // final (or finalised now)
            double v = acc[i];
            if (colsrc && Is > Ir[i]) {
                for (int rr = rs0; rr < rs1; ++rr) v = fma(-L.Al[rr * kLd + r], L.R[c * kLd + rr], v);
            }
            const int Js = s - (na - 1 - Ir[i]);       // solved block in my block row
            if (Js >= 0 && Js < Jc) {
                const int cs0 = L.cst[Js], cs1 = L.cst[Js + 1];
                for (int cc = cs0; cc < cs1; ++cc) v = fma(-L.R[cc * kLd + r], L.Bl[c * kLd + cc], v);
            }
            if (!(fabs(v) <= Tc)) ok = 0;
            acc[i] = v;
        }
    }
    wave_sync_lds();
    return ok;
}

// ---------------------------------------------------------------------------------------------
// Speculative tile solve.  Returns 1 if certified (tile holds Y with beta = 1).
// ---------------------------------------------------------------------------------------------
__device__ int tile_solve_fast(const Plan &P, const double *Ad, const double *Bd, double *Y,
                               int mr_, int nc_, double smin, double Tc, SolveLds &L, int *pert)
{
    const int mr = uniform(mr_), nc = uniform(nc_);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        L.nla = leaf_offsets(Ad, P.lda, mr, L.la);
        L.nlb = leaf_offsets(Bd, P.ldb, nc, L.lb);
        L.fail = 0;
    }
    __syncthreads();
    const int nla = uniform(L.nla), nlb = uniform(L.nlb);
    LeafLds &LL = L.leaf[w];
    int ok = 1;
    for (int d = 0; d < nla + nlb - 1; ++d) {
        const int jlo = d - (nla - 1) > 0 ? d - (nla - 1) : 0;
        const int jhi = d < nlb - 1 ? d : nlb - 1;
        for (int J = jlo + w; J <= jhi; J += kWaves) {
            const int I = nla - 1 - (d - J);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
            // right-hand side: R = Y_IJ - A(I, below) Y(below, J) - Y(I, left) B(left, J)
            d4 acc[1][1] = {{zero4()}};
            const int ncol[1] = {0};
            const int kb = L.la[I + 1];
            if (mr - kb > 0)
                wave_gemm<1, 1>(acc, 1, 1, Ad + (int64_t)kb * P.lda + lr0, P.lda, 0, nr,
                                Y + (int64_t)lc0 * P.ldc + kb, P.ldc, ncol, ncl, mr - kb, 0, 0);
            if (lc0 > 0)
                wave_gemm<1, 1>(acc, 1, 1, Y + lr0, P.ldc, 0, nr,
                                Bd + (int64_t)lc0 * P.ldb, P.ldb, ncol, ncl, lc0, 0, 0);
            // R into LDS (lane holds rows lane & 15, columns (lane >> 4) + 4 i)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                double v = 0.0;
                if (mm < nr && nn < ncl) {
                    v = Y[(int64_t)(lc0 + nn) * P.ldc + lr0 + mm] - acc[0][0][i];
                    if (!(fabs(v) <= Tc)) ok = 0;
                }
                LL.R[nn * kLd + mm] = v;
            }
            // leaf diagonal blocks of A and B (quasi-triangular part only)
            for (int t = lane; t < 256; t += 64) {
                const int rr = t & 15, cc = t >> 4;
                LL.Al[cc * kLd + rr] = (rr < nr && cc < nr && rr <= cc + 1)
                                           ? Ad[(int64_t)(lr0 + cc) * P.lda + lr0 + rr] : 0.0;
                LL.Bl[cc * kLd + rr] = (rr < ncl && cc < ncl && rr <= cc + 1)
                                           ? Bd[(int64_t)(lc0 + cc) * P.ldb + lc0 + rr] : 0.0;
            }
            wave_sync_lds();
            if (!leaf_solve(LL, nr, ncl, smin, Tc, pert)) ok = 0;
            // write the solved leaf back (lane -> row lane & 15 for coalescing)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                if (mm < nr && nn < ncl) Y[(int64_t)(lc0 + nn) * P.ldc + lr0 + mm] = LL.R[nn * kLd + mm];
            }
            wave_sync_lds();
        }
        if (!ok) L.fail = 1;
        __threadfence_block();
        __syncthreads();
        if (uniform(L.fail)) break;
    }
    __syncthreads();
    return uniform(L.fail) ? 0 : 1;
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

__device__ int tile_solve_robust(const Plan &P, const double *Ad, const double *Bd, double *Y,
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
                    z[t] = (p < rsz && pp < csz) ? Y[(int64_t)(cb0 + pp) * P.ldc + ra0 + p] : 0.0;
                }
                const int sb = small_solve(rsz, csz, a, b, z, smin, pert);
                for (int t = 0; t < 4; ++t) L.z[t] = z[t];
                L.zinfo[0] = sb;
            }
            __syncthreads();
            const int sb = uniform(L.zinfo[0]);
            if (sb) { scale_tile(Y, P.ldc, mr, nc, sb); e += sb; }     // Y <- beta Y
            if (tid == 0) {
                for (int t = 0; t < 4; ++t) {
                    const int p = t & 1, pp = t >> 1;
                    if (p < rsz && pp < csz) Y[(int64_t)(cb0 + pp) * P.ldc + ra0 + p] = L.z[t];
                }
            }
            __threadfence_block();
            __syncthreads();
            auto znorm = [&]() {
                double best = 0.0;
                for (int p = 0; p < rsz; ++p) {
                    double s = 0.0;
                    for (int pp = 0; pp < csz; ++pp) s += fabs(Y[(int64_t)(cb0 + pp) * P.ldc + ra0 + p]);
                    best = fmax(best, s);
                }
                return best;
            };
            if (ra0 > 0) {                                               // column update
                double v = 0.0;
                for (int r = tid; r < ra0; r += kThreads) {
                    double s = 0.0;
                    for (int cc = cb0; cc < cb1; ++cc) s += fabs(Y[(int64_t)cc * P.ldc + r]);
                    v = fmax(v, s);
                }
                const double ynorm = wg_max(v, L.red);
                const int s1 = uniform(protect_update(ynorm, L.anorm_above[ka], znorm()));
                if (s1) { scale_tile(Y, P.ldc, mr, nc, s1); e += s1; }
                for (int r = tid; r < ra0; r += kThreads) {
                    for (int cc = cb0; cc < cb1; ++cc) {
                        double acc = Y[(int64_t)cc * P.ldc + r];
                        for (int rr = ra0; rr < ra1; ++rr)
                            acc = fma(-Ad[(int64_t)rr * P.lda + r], Y[(int64_t)cc * P.ldc + rr], acc);
                        Y[(int64_t)cc * P.ldc + r] = acc;
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
                        for (int cc = L.bs[j]; cc < L.bs[j + 1]; ++cc) s += fabs(Y[(int64_t)cc * P.ldc + p]);
                        v = fmax(v, s);
                    }
                }
                const double ynorm = wg_max(v, L.red);
                const int s2 = uniform(protect_update(ynorm, znorm(), L.bnorm_right[lb]));
                if (s2) { scale_tile(Y, P.ldc, mr, nc, s2); e += s2; }
                for (int cc = cb1 + tid; cc < nc; cc += kThreads) {
                    for (int p = ra0; p < ra1; ++p) {
                        double acc = Y[(int64_t)cc * P.ldc + p];
                        for (int c2 = cb0; c2 < cb1; ++c2)
                            acc = fma(-Y[(int64_t)c2 * P.ldc + p], Bd[(int64_t)cc * P.ldb + c2], acc);
                        Y[(int64_t)cc * P.ldc + p] = acc;
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
    const int r0 = P.rowoff[ti], mr = P.rowoff[ti + 1] - r0;
    const int c0 = P.coloff[tl], nc = P.coloff[tl + 1] - c0;
    const int U = tile_updates(P, T);
    const int e_in = tile_exp_at(P, T, U);
    int e_syl = 0;
    double nrm = 0.0;
    int pert = 0;
    if (mr > 0 && nc > 0) {
        const double *Ad = P.A + (int64_t)r0 * P.lda + r0;
        const double *Bd = P.B + (int64_t)c0 * P.ldb + c0;
        double *Y = P.C + (int64_t)c0 * P.ldc + r0;
        double smin = 0x1p-52 * (*P.gmax);
        if (smin < 0x1p-1022) smin = 0x1p-1022;
        const double dA = P.anorm[(size_t)ti * P.pt + ti];
        const double dB = P.bnorm[(size_t)tl * P.qt + tl];
        const double dB1 = P.bdiag1[tl];
        const double Tc = kOmega / (2.0 + 2.0 * dA + 2.0 * dB1 + 2.0 * dB);
        int done = 0;
        if (!(P.flags & 1)) {
            int big = 0;     // the certificate's partial-sum bound needs |input| <= Tc too
            for (int t = threadIdx.x; t < mr * nc; t += kThreads) {
                const int rr = t % mr, cc = t / mr;
                const double v = Y[(int64_t)cc * P.ldc + rr];
                scratch[t] = v;
                if (!(fabs(v) <= Tc)) big = 1;
            }
            __threadfence_block();
            big = uniform(__syncthreads_or(big));
            if (!big) done = uniform(tile_solve_fast(P, Ad, Bd, Y, mr, nc, smin, Tc, L, &pert));
            if (!done) {
                for (int t = threadIdx.x; t < mr * nc; t += kThreads) {
                    const int rr = t % mr, cc = t / mr;
                    Y[(int64_t)cc * P.ldc + rr] = scratch[t];
                }
                __threadfence_block();
                __syncthreads();
                pert = 0;
            }
        }
        if (!done) {
            if (threadIdx.x == 0) atomicAdd(&P.stats[0], 1u);
            e_syl = tile_solve_robust(P, Ad, Bd, Y, mr, nc, smin, L, &pert);
        }
        // exact ||Y_kl||_inf
        double v = 0.0;
        for (int rr = threadIdx.x; rr < mr; rr += kThreads) {
            double s = 0.0;
            for (int cc = 0; cc < nc; ++cc) s += fabs(Y[(int64_t)cc * P.ldc + rr]);
            v = fmax(v, s);
        }
        nrm = wg_max(v, L.red);
    }
    if (pert) set_status(P.status, kPerturbed);
    if (threadIdx.x == 0) {
        double *ns = tile_norm_slot(P, T, U + 1);
        ns[0] = nrm;
        for (int s = 1; s < P.slabs; ++s) ns[s] = 0.0;
        *tile_exp_slot(P, T, U + 1) = e_in + e_syl;
    }
}

}  // namespace trsyl
