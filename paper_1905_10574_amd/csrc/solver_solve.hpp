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

namespace trsyl {

constexpr int kLd = 17;          // leading dimension of the 16x16 LDS buffers
constexpr int kMaxParts = kMaxLeaves > kWaves ? kMaxLeaves : kWaves;

struct LeafLds {
    double R[16 * kLd];
    double Al[16 * kLd];
    double Bl[16 * kLd];
    int rI[16], cJ[16], rst[17], cst[17];
};

struct SolveLds {
    LeafLds leaf[kWaves];
    double part[kMaxParts][16 * kLd];   // split-K partial sums of the leaf GEMMs
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
// Unguarded small solves of the speculative path: Gaussian elimination with complete pivoting
// (the method of Sec. 2.1) without ProtectUpdate / ProtectDivision; the caller's magnitude
// checks certify that no guard would have fired.  Return false if a pivot is below smin.
// ---------------------------------------------------------------------------------------------
// 2 unknowns: K [x0 x1]^T = [v0 v1]^T, K = [[k00, k01], [k10, k11]].
__device__ __forceinline__ bool solve2_cp(double k00, double k01, double k10, double k11,
                                          double &v0, double &v1, double smin)
{
    const double a00 = fabs(k00), a01 = fabs(k01), a10 = fabs(k10), a11 = fabs(k11);
    const bool rsw = fmax(a10, a11) > fmax(a00, a01);        // pivot in row 1
    double p0 = rsw ? k10 : k00, p1 = rsw ? k11 : k01;       // pivot row
    double q0 = rsw ? k00 : k10, q1 = rsw ? k01 : k11;       // other row
    double w0 = rsw ? v1 : v0, w1 = rsw ? v0 : v1;
    const bool csw = fabs(p1) > fabs(p0);                    // pivot in column 1
    if (csw) {
        double t = p0; p0 = p1; p1 = t;
        t = q0; q0 = q1; q1 = t;
    }
    if (fabs(p0) < smin) return false;
    const double l = q0 / p0;
    const double u11 = fma(-l, p1, q1);
    if (fabs(u11) < smin) return false;
    w1 = fma(-l, w0, w1);
    const double x1 = w1 / u11;
    const double x0 = fma(-p1, x1, w0) / p0;
    v0 = csw ? x1 : x0;
    v1 = csw ? x0 : x1;
    return true;
}

// 4 unknowns (2x2 A-block with 2x2 B-block): K = I (x) A11 + B11^T (x) I on vec(Z).
__device__ __noinline__ bool solve4_cp(const double a[4], const double b[4], double z[4], double smin)
{
    double K[4][4], v[4];
    int perm[4] = {0, 1, 2, 3};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = e & 1, q = e >> 1;
        v[e] = z[e];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int pp = u & 1, qq = u >> 1;
            double x = 0.0;
            if (qq == q) x += a[pp * 2 + p];     // A(p, pp)
            if (pp == p) x += b[q * 2 + qq];     // B(qq, q)
            K[e][u] = x;
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int pi = t, pj = t;
        double best = -1.0;
#pragma unroll
        for (int i = t; i < 4; ++i)
#pragma unroll
            for (int j = t; j < 4; ++j)
                if (fabs(K[i][j]) > best) { best = fabs(K[i][j]); pi = i; pj = j; }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double x = K[t][j];
            double y = x;
#pragma unroll
            for (int i = t + 1; i < 4; ++i) if (i == pi) { y = K[i][j]; K[i][j] = x; }
            K[t][j] = y;
        }
        {
            const double x = v[t];
            double y = x;
#pragma unroll
            for (int i = t + 1; i < 4; ++i) if (i == pi) { y = v[i]; v[i] = x; }
            v[t] = y;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double x = K[i][t];
            double y = x;
#pragma unroll
            for (int j = t + 1; j < 4; ++j) if (j == pj) { y = K[i][j]; K[i][j] = x; }
            K[i][t] = y;
        }
        {
            const int x = perm[t];
            int y = x;
#pragma unroll
            for (int j = t + 1; j < 4; ++j) if (j == pj) { y = perm[j]; perm[j] = x; }
            perm[t] = y;
        }
        if (fabs(K[t][t]) < smin) return false;
#pragma unroll
        for (int i = t + 1; i < 4; ++i) {
            const double l = K[i][t] / K[t][t];
#pragma unroll
            for (int j = t + 1; j < 4; ++j) K[i][j] = fma(-l, K[t][j], K[i][j]);
            v[i] = fma(-l, v[t], v[i]);
        }
    }
#pragma unroll
    for (int i = 3; i >= 0; --i) {
#pragma unroll
        for (int j = i + 1; j < 4; ++j) v[i] = fma(-K[i][j], v[j], v[i]);
        v[i] = v[i] / K[i][i];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int x = 0; x < 4; ++x) if (perm[t] == x) z[x] = v[t];
    return true;
}

// ---------------------------------------------------------------------------------------------
// Leaf solve (one wave): A_l Y + Y B_l = R on a leaf of nr x nc <= 16 x 16 held in L.R (ld 17),
// with A_l, B_l in L.Al, L.Bl.  Block anti-diagonals s = 0, 1, ...: the blocks on diagonal s are
// solved (a 1x1 block in its own lane; a block with 2 or 4 unknowns by the lane that owns its
// top-left entry, from values published to LDS), then every pending entry subtracts the
// contributions of the block just solved in its block column (below it) and in its block row
// (left of it).  Lane (c = lane & 15, q = lane >> 4) owns rows q, q+4, q+8, q+12 of column c.
// Returns 1 if the certificate held.
// ---------------------------------------------------------------------------------------------
__device__ int leaf_solve(LeafLds &L, int nr, int nc, double smin, double Tc)
{
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, q = lane >> 4;
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
    const bool cvalid = c < nc;
    const int Jc = cvalid ? L.cJ[c] : 0;
    const int cb0 = cvalid ? L.cst[Jc] : 0;
    const int csz = cvalid ? L.cst[Jc + 1] - cb0 : 0;
    const double bcc = cvalid ? L.Bl[c * kLd + c] : 0.0;
    double acc[4], dinv[4];
    int Ir[4], fin[4];
    bool single[4], owner[4], valid[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = q + 4 * i;
        valid[i] = cvalid && r < nr;
        Ir[i] = valid[i] ? L.rI[r] : 0;
        const int rb0 = valid[i] ? L.rst[Ir[i]] : 0;
        const int rsz = valid[i] ? L.rst[Ir[i] + 1] - rb0 : 0;
        fin[i] = valid[i] ? (na - 1 - Ir[i]) + Jc : -1;
        single[i] = rsz == 1 && csz == 1;
        owner[i] = valid[i] && r == rb0 && c == cb0;
        acc[i] = valid[i] ? L.R[c * kLd + r] : 0.0;
        const double dd = valid[i] ? L.Al[r * kLd + r] + bcc : 1.0;
        if (valid[i] && single[i] && fabs(dd) < smin) ok = 0;
        dinv[i] = dd;
    }
    const int steps = na + nb - 1;
    for (int s = 0; s < steps; ++s) {
        // finalise the blocks on anti-diagonal s: 1x1 blocks in place, larger ones published
        bool multi = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (fin[i] != s) continue;
            const int r = q + 4 * i;
            if (single[i]) {
                const double y = acc[i] / dinv[i];
                if (!(fabs(y) <= Tc)) ok = 0;
                L.R[c * kLd + r] = y;
            } else {
                L.R[c * kLd + r] = acc[i];
                multi = true;
            }
        }
        if (__ballot(multi)) {
            wave_sync_lds();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (fin[i] != s || single[i] || !owner[i]) continue;
                const int ra = q + 4 * i, rsz = L.rst[Ir[i] + 1] - ra;
                double a[4], b[4], z[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int p = t & 1, pp = t >> 1;   // column-major 2x2 position (p, pp)
                    a[t] = (p < rsz && pp < rsz) ? L.Al[(ra + pp) * kLd + ra + p] : 0.0;
                    b[t] = (p < csz && pp < csz) ? L.Bl[(c + pp) * kLd + c + p] : 0.0;
                    z[t] = (p < rsz && pp < csz) ? L.R[(c + pp) * kLd + ra + p] : 0.0;
                }
                bool good;
                if (rsz == 2 && csz == 2) {
                    good = solve4_cp(a, b, z, smin);
                } else if (rsz == 2) {   // (A11 + b I) z = r over the two rows
                    good = solve2_cp(a[0] + b[0], a[2], a[1], a[3] + b[0], z[0], z[1], smin);
                } else {                 // z (a I + B11) = r over the two columns
                    good = solve2_cp(a[0] + b[0], b[1], b[2], a[0] + b[3], z[0], z[2], smin);
                }
                if (!good) ok = 0;
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
        const int Is = na - 1 - (s - Jc);                // block solved in my block column
        const bool colsrc = cvalid && Is >= 0 && Is < na;
        const int rs0 = colsrc ? L.rst[Is] : 0, rs1 = colsrc ? L.rst[Is + 1] : 0;
        const double y0 = colsrc ? L.R[c * kLd + rs0] : 0.0;
        const double y1 = (colsrc && rs1 - rs0 == 2) ? L.R[c * kLd + rs0 + 1] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (!valid[i] || fin[i] <= s) continue;
            const int r = q + 4 * i;
            double v = acc[i];
            if (colsrc && Is > Ir[i]) {
                v = fma(-L.Al[rs0 * kLd + r], y0, v);
                if (rs1 - rs0 == 2) v = fma(-L.Al[(rs0 + 1) * kLd + r], y1, v);
            }
            const int Js = s - (na - 1 - Ir[i]);         // block solved in my block row
            if (Js >= 0 && Js < Jc) {
                const int cs0 = L.cst[Js], cs1 = L.cst[Js + 1];
                v = fma(-L.R[cs0 * kLd + r], L.Bl[c * kLd + cs0], v);
                if (cs1 - cs0 == 2) v = fma(-L.R[(cs0 + 1) * kLd + r], L.Bl[c * kLd + cs0 + 1], v);
            }
            if (!(fabs(v) <= Tc)) ok = 0;
            acc[i] = v;
        }
    }
    wave_sync_lds();
    return ok;
}

// ---------------------------------------------------------------------------------------------
// One wave accumulates acc += Aop(0:nr, k) Bop(k, 0:ncl) over k in [k0, k1) with the next
// 16-k chunk's operands loaded while the current chunk's MFMAs run.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void leaf_gemm(d4 &acc, const double *Aop, int64_t lda, int nr,
                                          const double *Bop, int64_t ldb, int ncl, int k0, int k1)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    if (k0 >= k1) return;
    double af[4], bf[4];
    auto load = [&](int kc, double (&a)[4], double (&b)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kc + 4 * q + j;
            a[j] = (r < nr && k < k1) ? Aop[(int64_t)k * lda + r] : 0.0;
            b[j] = (r < ncl && k < k1) ? Bop[(int64_t)r * ldb + k] : 0.0;
        }
    };
    load(k0, af, bf);
    for (int kc = k0; kc < k1; kc += 16) {
        double an[4], bn[4];
        if (kc + 16 < k1) load(kc + 16, an, bn);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = mfma16(bf[j], af[j], acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) { af[j] = an[j]; bf[j] = bn[j]; }
    }
}

// ---------------------------------------------------------------------------------------------
// Speculative tile solve.  Returns 1 if certified (tile holds Y with beta = 1).
// ---------------------------------------------------------------------------------------------
__device__ int tile_solve_fast(const Plan &P, const double *Ad, const double *Bd, double *Y,
                               int mr_, int nc_, double smin, double Tc, SolveLds &L)
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
        const int nleaf = jhi - jlo + 1;
        const int parts = nleaf >= kWaves ? 1 : kWaves / nleaf;
        // phase A: partial right-hand-side GEMMs, work item = leaf * parts + part
        for (int item = w; item < nleaf * parts; item += kWaves) {
            const int J = jlo + item / parts, part = item % parts;
            const int I = nla - 1 - (d - J);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
            const int kb = L.la[I + 1];
            const int K1 = mr - kb, K2 = lc0;               // rows below, columns left
            const int nch = (K1 + 15) / 16 + (K2 + 15) / 16;
            const int c0 = (int)(((int64_t)part * nch) / parts), c1 = (int)(((int64_t)(part + 1) * nch) / parts);
            const int n1 = (K1 + 15) / 16;                  // chunks of the first term
            d4 acc = zero4();
            // first term: A(I, below) Y(below, J), chunks [c0, min(c1, n1))
            if (c0 < n1)
                leaf_gemm(acc, Ad + (int64_t)kb * P.lda + lr0, P.lda, nr, Y + (int64_t)lc0 * P.ldc + kb,
                          P.ldc, ncl, 16 * c0, c1 < n1 ? 16 * c1 : K1);
            // second term: Y(I, left) B(left, J), chunks [max(c0, n1), c1) shifted by n1
            if (c1 > n1) {
                const int s0 = (c0 > n1 ? c0 : n1) - n1, s1 = c1 - n1;
                leaf_gemm(acc, Y + lr0, P.ldc, nr, Bd + (int64_t)lc0 * P.ldb, P.ldb, ncl, 16 * s0,
                          16 * s1 < K2 ? 16 * s1 : K2);
            }
            double *pp = L.part[item];
#pragma unroll
            for (int i = 0; i < 4; ++i) pp[((lane >> 4) + 4 * i) * kLd + (lane & 15)] = acc[i];
        }
        __syncthreads();
        // phase B: wave J - jlo (mod kWaves) reduces its leaf's parts in order and solves it
        for (int li = w; li < nleaf; li += kWaves) {
            const int J = jlo + li;
            const int I = nla - 1 - (d - J);
            const int lr0 = L.la[I], nr = L.la[I + 1] - lr0;
            const int lc0 = L.lb[J], ncl = L.lb[J + 1] - lc0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mm = lane & 15, nn = (lane >> 4) + 4 * i;
                double v = 0.0;
                if (mm < nr && nn < ncl) {
                    double g = 0.0;
                    for (int p = 0; p < parts; ++p) g += L.part[li * parts + p][nn * kLd + mm];
                    v = Y[(int64_t)(lc0 + nn) * P.ldc + lr0 + mm] - g;
                    if (!(fabs(v) <= Tc)) ok = 0;
                }
                LL.R[nn * kLd + mm] = v;
            }
            for (int t = lane; t < 256; t += 64) {
                const int rr = t & 15, cc = t >> 4;
                LL.Al[cc * kLd + rr] = (rr < nr && cc < nr && rr <= cc + 1)
                                           ? Ad[(int64_t)(lr0 + cc) * P.lda + lr0 + rr] : 0.0;
                LL.Bl[cc * kLd + rr] = (rr < ncl && cc < ncl && rr <= cc + 1)
                                           ? Bd[(int64_t)(lc0 + cc) * P.ldb + lc0 + rr] : 0.0;
            }
            wave_sync_lds();
            if (!leaf_solve(LL, nr, ncl, smin, Tc)) ok = 0;
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
        const double Tc = kOmega / (64.0 + 8.0 * (dA + dB1 + dB));
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
            // the unguarded small solves assume unscaled Kronecker entries: max|A|,|B| < 2^1016
            if (!big && *P.gmax < 0x1p1016) done = uniform(tile_solve_fast(P, Ad, Bd, Y, mr, nc, smin, Tc, L));
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
