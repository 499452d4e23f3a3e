// Leaf solve of the speculative tile solve: A_l Y + Y B_l = R on a leaf of at most 16 x 16
// (a diagonal block pair of the tile, Sec. 2.1's RobustSyl without scaling, certified by the
// caller), one wave per leaf.
//
// Lane (c, q) = c + 16 q holds column c and rows q, q + 4, q + 8, q + 12 of the leaf.  The solve
// walks the block anti-diagonals s = 0, 1, ...: the blocks on diagonal s become final, then every
// entry subtracts the contributions of the block solved at step s in its block column (rows
// below it) and in its block row (columns left of it).  Which block that is at step s is looked
// up in four small offset tables built once per leaf.  Updates are not masked: once an entry is
// final, the sources the tables give it lie in its own block or beyond, where A and B hold exact
// zeros outside the block, so its register keeps only the (tiny) residual of its block.
//
// Every division of the step loop is taken out of it: 1x1 blocks keep the reciprocal of
// a_rr + b_cc, and the 2- and 4-unknown block systems (Sec. 2.1) are factored once per leaf by
// Gaussian elimination with complete pivoting, one block per lane, and the factors applied to
// the unit vectors, which stores each block's inverse in LDS.  Every lane keeps, in registers,
// the row of that inverse belonging to the next entry it finalises, loaded at least two steps
// ahead; at a step that solves a multi-entry block, each lane of the block gathers the block's
// right-hand sides by cross-lane permutes and takes its unknown as one short dot product, so a
// step needs the permutes and one LDS round trip (publish the solved values, read the sources).
// A block beyond the stored slots is factored and solved at its step instead.
#pragma once
#include "device_common.hpp"
#include "plan.hpp"

namespace trsyl {

constexpr int kLd = 17;              // leading dimension of the 17 x 17 leaf buffers
constexpr int kSlab = kLd * 8;       // bytes per column of a leaf buffer
constexpr int kF2Slots = 64;         // stored factorisations of 2-unknown blocks per leaf
constexpr int kF4Slots = 16;         // stored factorisations of 4-unknown blocks per leaf
constexpr uint32_t kNoSlot = 255u;
constexpr int kTab = 80;             // source-table words: 16 before, 16 blocks, 48 after
constexpr int kTabIdle = 32;         // table index of step 0 for an entry outside the leaf

struct LeafLds {
    double R[17 * kLd];    // Y(r, k) at [k * 17 + r]: the right-hand side, then the solution
    double Al[17 * kLd];   // A_l(r, k) at [k * 17 + r]
    double Bl[17 * kLd];   // B_l(r, k) at [k * 17 + r]
    // Row 16 and column 16 of R, Al, Bl hold zeros.  Source tables, kTab words each: word 16 + k
    // describes the k-th source block, every other word points at the zero row / column 16.
    // A word packs the byte offsets of the block's first and second row (column); a 1x1 block's
    // second one is the zero row (column).
    uint32_t tcA[kTab];      // k-th block row from the bottom, offsets into Al columns (r * kSlab)
    uint32_t tcY[kTab];      //   the same rows as offsets inside a column of R (r * 8)
    uint32_t trY[kTab];      // k-th block column from the left, offsets into R columns (c * kSlab)
    uint32_t trB[kTab];      //   the same columns as offsets inside a column of Bl (c * 8)
    double f2[kF2Slots][4];      // inverses of 2-unknown blocks, row k at [2k], [2k + 1]
    double f4[kF4Slots][16];     // inverses of 4-unknown blocks in position order, row t at [4t ..]
    uint8_t slot[16 * 16];       // inverse slot of the block with top-left entry (r, c)
};

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double lds_at(const char *base, uint32_t off)
{
    return *(const double *)(base + off);
}

// ---------------------------------------------------------------------------------------------
// Small systems of the speculative path: Gaussian elimination with complete pivoting (Sec. 2.1)
// without ProtectUpdate / ProtectDivision; the caller's magnitude checks certify that no guard
// would have fired.  Factorisations return false if a pivot is below smin.
// ---------------------------------------------------------------------------------------------
// 2 unknowns, K = [[k00, k01], [k10, k11]]: pivot choices, multiplier and pivot reciprocals.
struct Factor2 {
    double l, p1, rp0, ru11;
    int sw;                    // bit 0: rows swapped, bit 1: columns swapped
};
__device__ __forceinline__ bool factor2_cp(double k00, double k01, double k10, double k11, double smin,
                                           Factor2 &f)
{
    const bool rsw = fmax(fabs(k10), fabs(k11)) > fmax(fabs(k00), fabs(k01));
    double p0 = rsw ? k10 : k00, p1 = rsw ? k11 : k01;
    double q0 = rsw ? k00 : k10, q1 = rsw ? k01 : k11;
    const bool csw = fabs(p1) > fabs(p0);
    if (csw) {
        double t = p0; p0 = p1; p1 = t;
        t = q0; q0 = q1; q1 = t;
    }
    f.sw = (rsw ? 1 : 0) | (csw ? 2 : 0);
    f.p1 = p1;
    if (fabs(p0) < smin) { f.l = 0.0; f.rp0 = 0.0; f.ru11 = 0.0; return false; }
    f.l = q0 / p0;
    const double u11 = fma(-f.l, p1, q1);
    f.rp0 = 1.0 / p0;
    if (fabs(u11) < smin) { f.ru11 = 0.0; return false; }
    f.ru11 = 1.0 / u11;
    return true;
}
__device__ __forceinline__ void apply2(const Factor2 &f, double &v0, double &v1)
{
    double w0 = (f.sw & 1) ? v1 : v0, w1 = (f.sw & 1) ? v0 : v1;
    w1 = fma(-f.l, w0, w1);
    const double x1 = w1 * f.ru11;
    const double x0 = fma(-f.p1, x1, w0) * f.rp0;
    v0 = (f.sw & 2) ? x1 : x0;
    v1 = (f.sw & 2) ? x0 : x1;
}

// The 4-unknown system of a 2x2 A-block with a 2x2 B-block: K = I (x) A11 + B11^T (x) I on the
// entries in position order t = p + 2 pp (entry (p, pp) of the block).  a, b: the blocks in
// column-major order.
__device__ __forceinline__ void kron4(const double (&a)[4], const double (&b)[4], double (&K)[4][4])
{
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = e & 1, q = e >> 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int pp = u & 1, qq = u >> 1;
            double x = 0.0;
            if (qq == q) x += a[pp * 2 + p];     // A(p, pp)
            if (pp == p) x += b[q * 2 + qq];     // B(qq, q)
            K[e][u] = x;
        }
    }
}

// P K Q = L U by elimination with complete pivoting, row swaps carried through the recorded
// multipliers.  f[0..5]: l10 l20 l30 l21 l31 l32; f[6..11]: u01 u02 u03 u12 u13 u23;
// f[12..15]: 1 / u_tt.  perm bits 2t: the position of row t, bits 8 + 2t: of column t.
__device__ __forceinline__ bool factor4_cp(const double (&a)[4], const double (&b)[4], double smin,
                                           double (&f)[16], uint32_t &perm)
{
    double K[4][4], Lm[4][4];
    int pr[4] = {0, 1, 2, 3}, pc[4] = {0, 1, 2, 3};
    kron4(a, b, K);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int u = 0; u < 4; ++u) Lm[e][u] = 0.0;
    bool good = true;
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
            const double x = K[t][j], xl = Lm[t][j];
            double y = x, yl = xl;
#pragma unroll
            for (int i = t + 1; i < 4; ++i)
                if (i == pi) { y = K[i][j]; K[i][j] = x; yl = Lm[i][j]; Lm[i][j] = xl; }
            K[t][j] = y;
            Lm[t][j] = yl;
        }
        {
            const int x = pr[t];
            int y = x;
#pragma unroll
            for (int i = t + 1; i < 4; ++i) if (i == pi) { y = pr[i]; pr[i] = x; }
            pr[t] = y;
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
            const int x = pc[t];
            int y = x;
#pragma unroll
            for (int j = t + 1; j < 4; ++j) if (j == pj) { y = pc[j]; pc[j] = x; }
            pc[t] = y;
        }
        if (fabs(K[t][t]) < smin) good = false;
        const double piv = good ? K[t][t] : 1.0;
#pragma unroll
        for (int i = t + 1; i < 4; ++i) {
            const double l = K[i][t] / piv;
            Lm[i][t] = l;
#pragma unroll
            for (int j = t + 1; j < 4; ++j) K[i][j] = fma(-l, K[t][j], K[i][j]);
        }
        f[12 + t] = 1.0 / piv;
    }
    f[0] = Lm[1][0]; f[1] = Lm[2][0]; f[2] = Lm[3][0]; f[3] = Lm[2][1]; f[4] = Lm[3][1]; f[5] = Lm[3][2];
    f[6] = K[0][1]; f[7] = K[0][2]; f[8] = K[0][3]; f[9] = K[1][2]; f[10] = K[1][3]; f[11] = K[2][3];
    perm = (uint32_t)(pr[0] | (pr[1] << 2) | (pr[2] << 4) | (pr[3] << 6) |
                      (pc[0] << 8) | (pc[1] << 10) | (pc[2] << 12) | (pc[3] << 14));
    return good;
}
// v: the right-hand side in row order; returns the unknowns in column order.
__device__ __forceinline__ void apply4(const double *f, double (&v)[4])
{
    v[1] = fma(-f[0], v[0], v[1]);
    v[2] = fma(-f[1], v[0], v[2]);
    v[3] = fma(-f[2], v[0], v[3]);
    v[2] = fma(-f[3], v[1], v[2]);
    v[3] = fma(-f[4], v[1], v[3]);
    v[3] = fma(-f[5], v[2], v[3]);
    v[3] = v[3] * f[15];
    v[2] = fma(-f[11], v[3], v[2]) * f[14];
    v[1] = fma(-f[9], v[2], v[1]);
    v[1] = fma(-f[10], v[3], v[1]) * f[13];
    v[0] = fma(-f[6], v[1], v[0]);
    v[0] = fma(-f[7], v[2], v[0]);
    v[0] = fma(-f[8], v[3], v[0]) * f[12];
}

// ---------------------------------------------------------------------------------------------
// Block structure of a leaf as bit masks (bit i: row / column i), from the subdiagonals.
// ---------------------------------------------------------------------------------------------
struct LeafMasks {
    uint32_t rmask, cmask, m2, n2;   // first rows / columns of blocks, of 2x2 blocks
    int na, nb;
};
__device__ __forceinline__ LeafMasks leaf_masks(const LeafLds &L, int nr, int nc)
{
    const int lane = threadIdx.x & 63;
    const bool rstart = (lane < nr) && (lane == 0 || L.Al[(lane - 1) * kLd + lane] == 0.0);
    const bool cstart = (lane < nc) && (lane == 0 || L.Bl[(lane - 1) * kLd + lane] == 0.0);
    LeafMasks M;
    M.rmask = (uint32_t)__ballot(rstart);
    M.cmask = (uint32_t)__ballot(cstart);
    M.m2 = M.rmask & ~(M.rmask >> 1) & ((1u << (nr - 1)) - 1u);
    M.n2 = M.cmask & ~(M.cmask >> 1) & ((1u << (nc - 1)) - 1u);
    M.na = __popc(M.rmask);
    M.nb = __popc(M.cmask);
    return M;
}
// Steps that solve a block with 2 or 4 unknowns: block (Ib, Jb) is final at step
// (na - 1 - Ib) + Jb, so a 2x2 block row Ib marks steps na - 1 - Ib + [0, nb) and a 2x2 block
// column Jb marks steps Jb + [0, na).
__device__ __forceinline__ uint32_t multi_steps(const LeafMasks &M)
{
    uint32_t ms = 0u;
    for (uint32_t x = M.m2; x; x &= x - 1u) {
        const int r = __ffs((int)x) - 1;
        const int Ib = __popc(M.rmask & ((1u << r) - 1u));
        ms |= ((1u << M.nb) - 1u) << (M.na - 1 - Ib);
    }
    for (uint32_t x = M.n2; x; x &= x - 1u) {
        const int c = __ffs((int)x) - 1;
        const int Jb = __popc(M.cmask & ((1u << c) - 1u));
        ms |= ((1u << M.na) - 1u) << Jb;
    }
    return ms;
}
__device__ __forceinline__ int kth_bit(uint32_t m, int k)   // index of the k-th set bit (k < 16)
{
    for (int t = 0; t < k && t < 16; ++t) m &= m - 1u;
    return __ffs((int)m) - 1;
}

// ---------------------------------------------------------------------------------------------
// Per-leaf set-up by its wave: the source tables and the factorisations of every 2- and
// 4-unknown block (one block per lane; blocks beyond the slots are factored at their step).
// Returns 0 in a lane whose factorisation met a pivot below smin.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int leaf_setup(LeafLds &L, const LeafMasks &M, double smin)
{
    const int lane = threadIdx.x & 63;
    constexpr uint32_t zA = (16u * kSlab) | ((16u * kSlab) << 16), zY = (16u * 8u) | ((16u * 8u) << 16);
    for (int t = lane; t < kTab; t += 64) {
        L.tcA[t] = zA;
        L.tcY[t] = zY;
        L.trY[t] = zA;
        L.trB[t] = zY;
    }
    ((uint32_t *)L.slot)[lane] = 0xFFFFFFFFu;
    wave_sync_lds();
    if (lane < 16) {
        const uint32_t below = (1u << lane) - 1u;
        if ((M.rmask >> lane) & 1u) {
            const int k = M.na - 1 - __popc(M.rmask & below);
            const uint32_t r1 = ((M.m2 >> lane) & 1u) ? lane + 1 : 16;
            L.tcA[16 + k] = (uint32_t)(lane * kSlab) | ((r1 * kSlab) << 16);
            L.tcY[16 + k] = (uint32_t)(lane * 8) | ((r1 * 8) << 16);
        }
        if ((M.cmask >> lane) & 1u) {
            const int k = __popc(M.cmask & below);
            const uint32_t c1 = ((M.n2 >> lane) & 1u) ? lane + 1 : 16;
            L.trY[16 + k] = (uint32_t)(lane * kSlab) | ((c1 * kSlab) << 16);
            L.trB[16 + k] = (uint32_t)(lane * 8) | ((c1 * 8) << 16);
        }
    }
    int ok = 1;
    const uint32_t m1 = M.rmask & ~M.m2, n1 = M.cmask & ~M.n2;
    const int A2 = __popc(M.m2), A1 = __popc(m1), B2 = __popc(M.n2), B1 = __popc(n1);
    // 2-unknown blocks: a 2x2 A-block with a 1x1 B-block (rows), then 1x1 with 2x2 (columns)
    if (lane < A2 * B1 + A1 * B2) {
        const bool rows = lane < A2 * B1;
        const int j = rows ? lane : lane - A2 * B1;
        const int nbj = rows ? B1 : B2;              // >= 1 here
        const int ra = kth_bit(rows ? M.m2 : m1, j / nbj);
        const int cb = kth_bit(rows ? n1 : M.n2, j % nbj);
        const double arr = L.Al[ra * kLd + ra], bcc = L.Bl[cb * kLd + cb];
        Factor2 F;
        bool good;
        if (rows)   // (A11 + b I) z = r over the two rows
            good = factor2_cp(arr + bcc, L.Al[(ra + 1) * kLd + ra], L.Al[ra * kLd + ra + 1],
                              L.Al[(ra + 1) * kLd + ra + 1] + bcc, smin, F);
        else        // z (a I + B11) = r over the two columns
            good = factor2_cp(arr + bcc, L.Bl[cb * kLd + cb + 1], L.Bl[(cb + 1) * kLd + cb],
                              arr + L.Bl[(cb + 1) * kLd + cb + 1], smin, F);
        if (!good) ok = 0;
        // the inverse's columns: the factors applied to the unit vectors
        double x00 = 1.0, x10 = 0.0, x01 = 0.0, x11 = 1.0;
        apply2(F, x00, x10);
        apply2(F, x01, x11);
        L.f2[lane][0] = x00;
        L.f2[lane][1] = x01;
        L.f2[lane][2] = x10;
        L.f2[lane][3] = x11;
        L.slot[ra * 16 + cb] = (uint8_t)lane;
    }
    if (lane < A2 * B2 && lane < kF4Slots) {
        const int ra = kth_bit(M.m2, lane / B2), cb = kth_bit(M.n2, lane % B2);
        double a[4], b[4], f[16];
        uint32_t pm;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int p = t & 1, pp = t >> 1;
            a[t] = L.Al[(ra + pp) * kLd + ra + p];
            b[t] = L.Bl[(cb + pp) * kLd + cb + p];
        }
        if (!factor4_cp(a, b, smin, f, pm)) ok = 0;
        // column j of the inverse: the right-hand side e_j in the factorisation's row order,
        // the unknowns come back in its column order
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) v[t] = ((pm >> (2 * t)) & 3u) == (uint32_t)j ? 1.0 : 0.0;
            apply4(f, v);
#pragma unroll
            for (int t = 0; t < 4; ++t) L.f4[lane][4 * ((pm >> (8 + 2 * t)) & 3u) + j] = v[t];
        }
        L.slot[ra * 16 + cb] = (uint8_t)lane;
    }
    wave_sync_lds();
    return ok;
}

// ---------------------------------------------------------------------------------------------
// The step loop.  Returns 0 in a lane where a pivot fell below smin or a value it produced
// exceeded Tc (the first non-finite value is an infinity, which the running maximum keeps).
// With vmax_out, the lane's largest magnitude is stored there instead and only the pivots
// decide the return value.  MULTI = false is the loop of a leaf made of 1x1 blocks only.
// ---------------------------------------------------------------------------------------------
template <bool MULTI>
__device__ __forceinline__ int leaf_solve_t(LeafLds &L, int nr, int nc, double smin, double Tc,
                                            const LeafMasks &M, double *vmax_out)
{
    constexpr int E = 4;
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, q = lane >> 4;
    const uint32_t rmask = M.rmask, cmask = M.cmask, m2 = M.m2, n2 = M.n2;
    const int na = M.na, steps = M.na + M.nb - 1;
    const uint32_t msteps = multi_steps(M);
    const bool cvalid = c < nc;
    const uint32_t cle = cmask & ((2u << c) - 1u);
    const int Jc = __popc(cle) - 1;                  // my block column
    const int cb0 = cle ? 31 - __clz(cle) : 0;       // its first column
    const int csz = 1 + ((n2 >> cb0) & 1);
    const double bcc = L.Bl[c * kLd + c];
    const int ctab = cvalid ? 16 - Jc : kTabIdle;    // table index of step 0

    int ok = 1;
    double vmax = 0.0;
    double acc[E], rdd[E];
    int fin[E], rtab[E];
    uint32_t info[E];                                // kind | pos << 2 | slot << 4 | block lane << 12
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int r = q + 4 * i;
        const bool valid = cvalid && r < nr;
        const uint32_t rle = rmask & ((2u << r) - 1u);
        const int Ir = __popc(rle) - 1;
        const int rb0 = rle ? 31 - __clz(rle) : 0;
        const int rsz = 1 + ((m2 >> rb0) & 1);
        const int rowst = na - 1 - Ir;               // first step with a row source
        fin[i] = valid ? rowst + Jc : -1;            // step at which the entry is final
        rtab[i] = valid ? 16 - rowst : kTabIdle;
        acc[i] = L.R[c * kLd + r];
        const uint32_t kind = (rsz == 2 ? 1u : 0u) + (csz == 2 ? 2u : 0u);
        const uint32_t pos = (uint32_t)((r - rb0) + 2 * (c - cb0));
        const uint32_t sl = (valid && kind) ? L.slot[rb0 * 16 + cb0] : kNoSlot;
        const uint32_t bl = (uint32_t)((cb0 + 16 * (rb0 & 3)) & 63);
        info[i] = kind | (pos << 2) | (sl << 4) | (bl << 12);
        rdd[i] = 1.0;
        if (valid && kind == 0) {
            const double dd = L.Al[r * kLd + r] + bcc;
            if (fabs(dd) < smin) ok = 0;
            rdd[i] = 1.0 / dd;
        }
    }
    // cn: the row of the block inverse of the entry this lane finalises next, over the block's
    // positions p + 2 pp (a 1x1 block: its reciprocal in cn[0]); a block without a stored inverse
    // leaves zeros and is solved from its factorisation at its step
    double cn[4] = {0.0, 0.0, 0.0, 0.0};
    auto fetch = [&](uint32_t inf, double rd) __attribute__((always_inline)) {
        const uint32_t kind = inf & 3u, pos = (inf >> 2) & 3u, sl = (inf >> 4) & 255u;
        if (kind == 0u) {
            cn[0] = rd; cn[1] = 0.0; cn[2] = 0.0; cn[3] = 0.0;
        } else if (sl == kNoSlot) {
            cn[0] = 0.0; cn[1] = 0.0; cn[2] = 0.0; cn[3] = 0.0;
        } else if (kind == 3u) {
#pragma unroll
            for (int t = 0; t < 4; ++t) cn[t] = L.f4[sl][4 * pos + t];
        } else {
            const uint32_t k = kind == 1u ? pos : pos >> 1;
            const double x0 = L.f2[sl][2 * k], x1 = L.f2[sl][2 * k + 1];
            cn[0] = x0;
            cn[1] = kind == 1u ? x1 : 0.0;
            cn[2] = kind == 1u ? 0.0 : x1;
            cn[3] = 0.0;
        }
    };
    if constexpr (MULTI) {
        // entries finalise from the last valid one (largest row) upwards
        uint32_t finf = 0u;
        double frd = 1.0;
        bool any = false;
#pragma unroll
        for (int i = 0; i < E; ++i)
            if (fin[i] >= 0) { finf = info[i]; frd = rdd[i]; any = true; }
        if (any) fetch(finf, frd);
    }
    const char *Rb = (const char *)L.R, *Ab = (const char *)L.Al, *Bb = (const char *)L.Bl;
    const char *Rc = Rb + c * kSlab, *Bc = Bb + c * kSlab;
    // Software pipeline: the source tables of step s + 2 and the coefficients of step s + 1 are
    // read while step s's updates run (neither depends on the values being solved).
    struct Tabs { uint32_t ta, ty, tb[E], tz[E]; };
    struct Coef { double a0[E], a1[E], b0[E], b1[E]; };
    auto tables = [&](int s, Tabs &T) {
        T.ta = L.tcA[ctab + s];
        T.ty = L.tcY[ctab + s];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            T.tb[i] = L.trB[rtab[i] + s];
            T.tz[i] = L.trY[rtab[i] + s];
        }
    };
    auto coefs = [&](const Tabs &T, Coef &C) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            C.a0[i] = lds_at(Ab, (T.ta & 0xffffu) + 8 * (q + 4 * i));
            C.a1[i] = lds_at(Ab, (T.ta >> 16) + 8 * (q + 4 * i));
            C.b0[i] = lds_at(Bc, T.tb[i] & 0xffffu);
            C.b1[i] = lds_at(Bc, T.tb[i] >> 16);
        }
    };
    // one step: finalise the entries of step s, publish them, read the values the updates need,
    // start the loads of the next operands (into the table set just consumed and the free
    // coefficient set), then apply the updates.  Two steps per loop trip swap the roles of the
    // register sets, so no operand is copied between trips.
    auto step = [&](int s, Tabs &Tc_, const Tabs &Tn, const Coef &Cc, Coef &Cn) __attribute__((always_inline)) {
        // the entry this lane finalises at step s, if any (at most one: its rows lie in distinct
        // block rows)
        double accf = 0.0, rdf = 1.0;
        int rf = -1, fi = -1;
        uint32_t inf = 0u;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            if (fin[i] == s) {
                accf = acc[i]; rf = q + 4 * i; fi = i;
                if constexpr (MULTI) inf = info[i];
                else rdf = rdd[i];
            }
        }
        double yf;
        if (MULTI && ((msteps >> s) & 1u)) {
            const uint32_t kind = inf & 3u, pos = (inf >> 2) & 3u, sl = (inf >> 4) & 255u;
            const int bl = (int)(inf >> 12);
            // the block's right-hand sides in position order p + 2 pp (entry (rb0 + p, cb0 + pp)
            // sits in lane cb0 + pp + 16 ((rb0 + p) & 3)); positions outside the block read as 0
            double g[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) g[t] = __shfl(accf, (bl + 16 * (t & 1) + (t >> 1)) & 63, 64);
            const double g1 = (kind & 1u) ? g[1] : 0.0, g2 = (kind & 2u) ? g[2] : 0.0;
            const double g3 = kind == 3u ? g[3] : 0.0;
            yf = fma(cn[3], g3, fma(cn[2], g2, fma(cn[1], g1, cn[0] * g[0])));
            if (rf >= 0 && kind != 0u && sl == kNoSlot) {
                // no stored inverse: factor the block here
                const int ra = rf - (int)(pos & 1u), cb = c - (int)(pos >> 1);
                if (kind != 3u) {
                    const double arr = L.Al[ra * kLd + ra], bb = L.Bl[cb * kLd + cb];
                    Factor2 F;
                    bool good;
                    if (kind == 1u)
                        good = factor2_cp(arr + bb, L.Al[(ra + 1) * kLd + ra], L.Al[ra * kLd + ra + 1],
                                          L.Al[(ra + 1) * kLd + ra + 1] + bb, smin, F);
                    else
                        good = factor2_cp(arr + bb, L.Bl[cb * kLd + cb + 1], L.Bl[(cb + 1) * kLd + cb],
                                          arr + L.Bl[(cb + 1) * kLd + cb + 1], smin, F);
                    if (!good) ok = 0;
                    double v0 = g[0], v1 = kind == 1u ? g[1] : g[2];
                    apply2(F, v0, v1);
                    yf = pos == 0u ? v0 : v1;
                } else {
                    double a[4], b[4], f[16], w[4];
                    uint32_t pm2;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int p = t & 1, pp = t >> 1;
                        a[t] = L.Al[(ra + pp) * kLd + ra + p];
                        b[t] = L.Bl[(cb + pp) * kLd + cb + p];
                    }
                    if (!factor4_cp(a, b, smin, f, pm2)) ok = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const uint32_t e = (pm2 >> (2 * t)) & 3u;
                        w[t] = e == 0u ? g[0] : e == 1u ? g[1] : e == 2u ? g[2] : g[3];
                    }
                    apply4(f, w);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (((pm2 >> (8 + 2 * t)) & 3u) == pos) yf = w[t];
                }
            }
        } else {
            yf = accf * (MULTI ? cn[0] : rdf);       // only 1x1 blocks finalise at this step
        }
        if (rf >= 0) {
            vmax = fmax(vmax, fabs(yf));
            L.R[c * kLd + rf] = yf;
        }
        wave_sync_lds();
        // values of the blocks solved at step s, then the next step's operands
        const double y0 = lds_at(Rc, Tc_.ty & 0xffffu), y1 = lds_at(Rc, Tc_.ty >> 16);
        double z0[E], z1[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            z0[i] = lds_at(Rb, (Tc_.tz[i] & 0xffffu) + 8 * (q + 4 * i));
            z1[i] = lds_at(Rb, (Tc_.tz[i] >> 16) + 8 * (q + 4 * i));
        }
        if constexpr (MULTI) {
            // the inverse row of the entry above the one just finalised (used two or more steps on)
            uint32_t ninf = 0u;
            double nrd = 1.0;
#pragma unroll
            for (int i = 1; i < E; ++i)
                if (fi == i) { ninf = info[i - 1]; nrd = rdd[i - 1]; }
            if (fi > 0) fetch(ninf, nrd);
        }
        coefs(Tn, Cn);
        tables(s + 2, Tc_);
        __builtin_amdgcn_sched_barrier(0);
        // contributions of the blocks solved at step s
#pragma unroll
        for (int i = 0; i < E; ++i) {
            double v = acc[i];
            v = fma(-Cc.a0[i], y0, v);
            v = fma(-Cc.a1[i], y1, v);
            v = fma(-z0[i], Cc.b0[i], v);
            v = fma(-z1[i], Cc.b1[i], v);
            acc[i] = v;
            vmax = fmax(vmax, fabs(v));
        }
    };
    Tabs TA, TB;
    Coef CA, CB;
    tables(0, TA);
    tables(1, TB);
    coefs(TA, CA);
    for (int s = 0; s < steps; s += 2) {
        step(s, TA, TB, CA, CB);
        if (s + 1 < steps) step(s + 1, TB, TA, CB, CA);
    }
    wave_sync_lds();
    if (vmax_out) *vmax_out = vmax;
    else if (!(vmax <= Tc)) ok = 0;
    return ok;
}
__device__ __forceinline__ int leaf_solve(LeafLds &L, int nr, int nc, double smin, double Tc,
                                          const LeafMasks &M, double *vmax_out = nullptr)
{
    if (M.m2 | M.n2) return leaf_solve_t<true>(L, nr, nc, smin, Tc, M, vmax_out);
    return leaf_solve_t<false>(L, nr, nc, smin, Tc, M, vmax_out);
}

}  // namespace trsyl
