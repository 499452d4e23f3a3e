// Leaf solve of the speculative tile solve: A_l Y + Y B_l = R on a leaf of at most 16 x 16
// (a diagonal block pair of the tile, Sec. 2.1's RobustSyl without scaling, certified by the
// caller), one wave per leaf.
//
// Layout.  The leaf's rows are grouped into at most 8 row pairs: each 2x2 block of A_l is a pair,
// and the 1x1 blocks are paired in order of appearance (an odd one out is paired with nothing).
// The columns are grouped into column pairs the same way from B_l.  Lane rho + 8 kappa holds the
// four entries (row pair rho) x (column pair kappa), so every 1x1, 2x1, 1x2 or 2x2 block of
// unknowns lies inside one lane.  The inverse of every block system the lane owns (Sec. 2.1's
// 1, 2 and 4-unknown systems, factored by Gaussian elimination with complete pivoting and
// applied to the unit vectors) forms a 4 x 4 block-diagonal matrix W held in the lane's
// registers, so a block's unknowns are W times its right-hand sides, with no cross-lane traffic.
//
// Sweep.  Step s makes the blocks on block anti-diagonal s final.  Every step each lane writes
// W times its four right-hand sides to the leaf buffer (an entry becomes correct at its own step
// and is only read from then on), then reads the two source blocks of each entry (the block
// solved at step s in its block column, the block solved at step s in its block row) and
// subtracts their contributions.  For the duration of the sweep the diagonal blocks of A_l and
// B_l are set to zero: an entry's only sources after its own step lie in its own block or beyond,
// so its right-hand side, and with it the value written for it, stays fixed from then on.
// Source positions come from two small offset tables per leaf; a 1x1 source block's second row
// (column) is the leaf buffer's zero row (column) 16, which no lane writes (patch entries outside
// the leaf write to a per-lane sink).
#pragma once
#include "device_common.hpp"
#include "plan.hpp"

namespace trsyl {

constexpr int kLd = 17;              // leading dimension of the 17 x 17 leaf buffers
constexpr int kSlab = kLd * 8;       // bytes per column of a leaf buffer
constexpr int kTab = 80;             // source-table entries: 16 before, 16 blocks, 48 after
constexpr int kTabIdle = 32;         // table index of step 0 for an entry outside the leaf

struct LeafLds {
    double R[17 * kLd];    // Y(r, k) at [k * 17 + r]: the right-hand side, then the solution
    double Al[17 * kLd];   // A_l(r, k) at [k * 17 + r]
    double Bl[17 * kLd + 1];   // B_l(r, k) at [k * 17 + r]; one zero after the last column
    // Row 16 and column 16 of R, Al, Bl hold zeros.
    double sink[64];    // per lane: where the values of patch entries outside the leaf go
};

// Block structure of one leaf of A_kk (its rows) or of B_ll (its columns), built once per tile.
struct LeafShape {
    uint32_t mask, two;   // bit i: a block starts at i; a 2x2 block starts at i
    int n, nb;            // size, number of blocks
    // Source table, kTab entries: entry 16 + k describes the k-th source block, every other entry
    // points at the zero row / column.  Rows: k-th block row from the bottom, first row r0,
    // second r1 (16 for 1x1): x = r0 * kSlab (a column of Al), y = r0 * 8 | r1 * 8 << 16 (rows of
    // R).  Columns: k-th block column from the left, first column c0, second c1: x = c0 * 8 (rows
    // of a column of Bl), y = c0 * kSlab | c1 * kSlab << 16.
    uint2 tab[kTab];
    uint8_t pair[2][8];   // pairs: first and second member (16: none)
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
__device__ __forceinline__ bool factor4_cp(double (&K)[4][4], double smin, double (&f)[16], uint32_t &perm)
{
    double Lm[4][4];
    int pr[4] = {0, 1, 2, 3}, pc[4] = {0, 1, 2, 3};
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
        const double rpiv = 1.0 / piv;
#pragma unroll
        for (int i = t + 1; i < 4; ++i) {
            const double l = K[i][t] * rpiv;
            Lm[i][t] = l;
#pragma unroll
            for (int j = t + 1; j < 4; ++j) K[i][j] = fma(-l, K[t][j], K[i][j]);
        }
        f[12 + t] = rpiv;
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
// Shape of a leaf of size n whose diagonal block starts at (o, o) of T (ld), by one wave: a
// block starts at i unless T(o + i, o + i - 1) != 0.  Rows and columns are paired in the order
// the pairs open: at a 2x2 block, and at every other 1x1 block.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void leaf_shape_wave(const double *T, int64_t ld, int o, int n, bool cols, LeafShape &S)
{
    const int lane = lane_here();
    const bool start = lane < n && (lane == 0 || ldg(T + (int64_t)(o + lane - 1) * ld + o + lane) == 0.0);
    const uint32_t mask = (uint32_t)__ballot(start);
    const uint32_t two = mask & ~(mask >> 1) & ((1u << (n - 1)) - 1u);
    const int nb = __popc(mask);
    constexpr uint32_t zA = 16u * kSlab, zY = (16u * 8u) | ((16u * 8u) << 16);
    constexpr uint32_t zB = 16u * 8u, zZ = (16u * kSlab) | ((16u * kSlab) << 16);
    for (int t = lane; t < kTab; t += 64) S.tab[t] = cols ? make_uint2(zB, zZ) : make_uint2(zA, zY);
    if (lane < 16) (&S.pair[0][0])[lane] = 16;
    if (lane == 0) {
        S.mask = mask;
        S.two = two;
        S.n = n;
        S.nb = nb;
    }
    wave_sync_lds();
    if (lane < 16 && ((mask >> lane) & 1u)) {
        const int r = lane;
        const uint32_t one = mask & ~two, below = (1u << r) - 1u;
        const int n2b = __popc(two & below), k1 = __popc(one & below);
        const bool is2 = (two >> r) & 1u;
        const uint32_t r1 = is2 ? (uint32_t)r + 1u : 16u;
        if (!cols)
            S.tab[16 + nb - 1 - __popc(mask & below)] =
                make_uint2((uint32_t)r * kSlab, ((uint32_t)r * 8u) | ((r1 * 8u) << 16));
        else
            S.tab[16 + __popc(mask & below)] =
                make_uint2((uint32_t)r * 8u, ((uint32_t)r * kSlab) | ((r1 * kSlab) << 16));
        if (is2) {
            const int pi = n2b + ((k1 + 1) >> 1);
            S.pair[0][pi] = (uint8_t)r;
            S.pair[1][pi] = (uint8_t)(r + 1);
        } else if (!(k1 & 1)) {
            S.pair[0][n2b + (k1 >> 1)] = (uint8_t)r;
        } else {
            const int rp = 31 - __clz(one & below);    // the 1x1 block that opened this pair
            S.pair[1][__popc(two & ((1u << rp) - 1u)) + ((k1 - 1) >> 1)] = (uint8_t)r;
        }
    }
    wave_sync_lds();
}

// ---------------------------------------------------------------------------------------------
// The lane's patch: rows r[x] and columns c[y] of its four entries t = x + 2 y (16: none), and
// W, the inverse of every block system inside the patch (zero elsewhere), its rows in the order
// perm gives (the rows come out in the factorisation's column order, which the sweep undoes by
// where it writes each value).  ok = 0 when a pivot of those systems fell below smin.
// ---------------------------------------------------------------------------------------------
struct LeafPatch {
    int r[2], c[2];
    double w[4][4];
    uint32_t perm;   // row t of W gives the unknown of entry (perm >> 2 t) & 3
    int ok;
};

// Every lane factors one 4 x 4 system, K = I (x) A_p + B_p^T (x) I over its patch, where A_p
// (B_p) is the 2x2 block of its row (column) pair when the pair is a 2x2 block and the pair's
// diagonal otherwise: K then falls apart into the patch's 1-, 2- and 4-unknown systems of
// Sec. 2.1, which elimination with complete pivoting factors independently (the coupling
// between them is exactly zero).  An entry outside the leaf gets a row and column of its own with
// pivot 2 smin.  A leaf without 2x2 blocks takes the reciprocals of the 1x1 systems directly.
__device__ __forceinline__ LeafPatch leaf_setup(LeafLds &L, const LeafShape &RS, const LeafShape &CS, double smin)
{
    const int lane = lane_here();
    if (lane == 0) L.Bl[17 * kLd] = 0.0;
    LeafPatch P;
    const int rho = lane & 7, kap = lane >> 3;
    P.r[0] = RS.pair[0][rho];
    P.r[1] = RS.pair[1][rho];
    P.c[0] = CS.pair[0][kap];
    P.c[1] = CS.pair[1][kap];
    const int ra = P.r[0], rb = P.r[1], ca = P.c[0], cb = P.c[1];
    // the patch's diagonal blocks (row / column 16 of the buffers hold zeros)
    const double a00 = L.Al[ra * kLd + ra], a11 = L.Al[rb * kLd + rb];
    const double b00 = L.Bl[ca * kLd + ca], b11 = L.Bl[cb * kLd + cb];
    bool pad[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) pad[t] = P.r[t & 1] >= 16 || P.c[t >> 1] >= 16;
    int ok = 1;
    P.perm = 0xE4u;                                     // rows in entry order
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) P.w[i][j] = 0.0;
    if (uniform((RS.two | CS.two) ? 1 : 0) == 0) {
        const double d[4] = {a00 + b00, a11 + b00, a00 + b11, a11 + b11};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (!pad[t] && !(fabs(d[t]) >= smin)) ok = 0;
            P.w[t][t] = pad[t] ? 0.0 : 1.0 / d[t];
        }
    } else {
        const bool R2 = ra < 16 && ((RS.two >> ra) & 1u);
        const bool C2 = ca < 16 && ((CS.two >> ca) & 1u);
        const double a10 = R2 ? L.Al[ra * kLd + rb] : 0.0, a01 = R2 ? L.Al[rb * kLd + ra] : 0.0;
        const double b10 = C2 ? L.Bl[ca * kLd + cb] : 0.0, b01 = C2 ? L.Bl[cb * kLd + ca] : 0.0;
        const double a[4] = {a00, a10, a01, a11}, b[4] = {b00, b10, b01, b11};
        double K[4][4];
        kron4(a, b, K);
        const double pv = 2.0 * smin;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (pad[i] || pad[j]) K[i][j] = i == j ? pv : 0.0;
        double f[16];
        uint32_t pm;
        if (!factor4_cp(K, smin, f, pm)) ok = 0;
        // column j of the inverse: e_j in the factorisation's row order; the unknowns come back
        // in its column order, kept as the row order of W
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) v[t] = ((pm >> (2 * t)) & 3u) == (uint32_t)j ? 1.0 : 0.0;
            apply4(f, v);
#pragma unroll
            for (int t = 0; t < 4; ++t) P.w[t][j] = v[t];
        }
        P.perm = (pm >> 8) & 0xFFu;
    }
    P.ok = ok;
    return P;
}

// ---------------------------------------------------------------------------------------------
// The sweep.  MODE 1: W is a general 4 x 4 (rows in perm order), MODE 0: W is diagonal.
// Returns 0 when a value it produced (a right-hand side after an update, or a value written)
// exceeded Tc or was not finite; with vmax_out the largest magnitude (infinity for a non-finite
// value) is stored there instead and 1 is returned.
// ---------------------------------------------------------------------------------------------
template <int MODE>
__device__ __forceinline__ int leaf_solve_t(LeafLds &L, const LeafPatch &P, const LeafShape &RS, const LeafShape &CS,
                                            int nr, int nc,
                                            double Tc, double *vmax_out)
{
    const int lane = lane_here();
    const int steps = RS.nb + CS.nb - 1;
    // set the diagonal blocks of A_l (lanes 0..15, row r) and B_l (lanes 16..31, column c) to
    // zero for the sweep; the lane keeps the values it cleared
    double *dz = lane < 16 ? L.Al : L.Bl;
    const uint32_t dtwo = lane < 16 ? RS.two : CS.two;
    const int di = lane & 15;
    int zo0 = -1, zo1 = -1;
    double zv0 = 0.0, zv1 = 0.0;
    if (lane < 32 && di < (lane < 16 ? nr : nc)) {
        zo0 = di * kLd + di;
        int pt = -1;                                   // the other row (column) of a 2x2 block
        if ((dtwo >> di) & 1u) pt = di + 1;
        else if (di > 0 && ((dtwo >> (di - 1)) & 1u)) pt = di - 1;
        if (pt >= 0) zo1 = lane < 16 ? pt * kLd + di : di * kLd + pt;
    }
    if (zo0 >= 0) { zv0 = dz[zo0]; dz[zo0] = 0.0; }
    if (zo1 >= 0) { zv1 = dz[zo1]; dz[zo1] = 0.0; }
    // tables, offsets and right-hand sides of the patch
    int rtab[2], ctab[2];
    uint32_t rof[2], cof[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const int r = P.r[x];
        rof[x] = (uint32_t)r * 8u;
        rtab[x] = kTabIdle;
        if (r < 16) rtab[x] = 16 - (RS.nb - 1 - (__popc(RS.mask & ((2u << r) - 1u)) - 1));
    }
#pragma unroll
    for (int y = 0; y < 2; ++y) {
        const int c = P.c[y];
        cof[y] = (uint32_t)c * kSlab;
        ctab[y] = kTabIdle;
        if (c < 16) ctab[y] = 16 - (__popc(CS.mask & ((2u << c) - 1u)) - 1);
    }
    wave_sync_lds();
    const char *Rb = (const char *)L.R, *Ab = (const char *)L.Al, *Bb = (const char *)L.Bl;
    char *Rw = (char *)L.R;
    double acc[4];
    uint32_t wof[4];     // where row t of W x (right-hand sides) goes: its entry's place in R,
                         // or the lane's sink for an entry outside the leaf
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc[t] = lds_at(Rb, cof[t >> 1] + rof[t & 1]);
        const uint32_t u = (P.perm >> (2 * t)) & 3u;
        const bool real = P.r[u & 1] < 16 && P.c[u >> 1] < 16;
        wof[t] = real ? cof[u >> 1] + rof[u & 1] : (uint32_t)((const char *)&L.sink[lane] - Rb);
    }
    double vmax = 0.0;
    // software pipeline: the tables of step s + 2 and the coefficients of step s + 1 are read
    // while step s's updates run
    struct Tabs { uint2 col[2], row[2]; };
    struct Coef { double a0[4], a1[4], b0[4], b1[4]; };
    auto tables = [&](int s, Tabs &T) {
#pragma unroll
        for (int y = 0; y < 2; ++y) T.col[y] = RS.tab[ctab[y] + s];
#pragma unroll
        for (int x = 0; x < 2; ++x) T.row[x] = CS.tab[rtab[x] + s];
    };
    auto coefs = [&](const Tabs &T, Coef &C) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int x = t & 1, y = t >> 1;
            const char *pa = Ab + T.col[y].x + rof[x];            // A(r_x, r0), A(r_x, r0 + 1)
            C.a0[t] = lds_at(pa, 0);
            C.a1[t] = lds_at(pa, kSlab);
            const char *pb = Bb + cof[y] + T.row[x].x;            // B(c0, c_y), B(c0 + 1, c_y)
            C.b0[t] = lds_at(pb, 0);
            C.b1[t] = lds_at(pb, 8);
        }
    };
    double ynan = 0.0;   // stays 0 unless a value written was not finite
    auto step = [&](int s, Tabs &Tc_, const Tabs &Tn, const Coef &Cc, Coef &Cn) __attribute__((always_inline)) {
        // W times the right-hand sides: final for the blocks of step s and every earlier one
        double yv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double v;
            if constexpr (MODE == 1) {
                v = P.w[t][0] * acc[0];
                v = fma(P.w[t][1], acc[1], v);
                v = fma(P.w[t][2], acc[2], v);
                v = fma(P.w[t][3], acc[3], v);
            } else {
                v = P.w[t][t] * acc[t];
            }
            yv[t] = v;
            *(double *)(Rw + wof[t]) = v;
        }
        wave_sync_lds();
        // values of the blocks solved at step s, then the next step's operands
        double y0[2], y1[2], z0[2], z1[2];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            y0[y] = lds_at(Rb, cof[y] + (Tc_.col[y].y & 0xffffu));
            y1[y] = lds_at(Rb, cof[y] + (Tc_.col[y].y >> 16));
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            z0[x] = lds_at(Rb, (Tc_.row[x].y & 0xffffu) + rof[x]);
            z1[x] = lds_at(Rb, (Tc_.row[x].y >> 16) + rof[x]);
        }
        coefs(Tn, Cn);
        tables(s + 2, Tc_);
        __builtin_amdgcn_sched_barrier(0);
        // every value written is checked: its magnitude, and whether it is finite (a NaN, from
        // two overflowing products of opposite sign, is invisible to the maximum; 0 times a
        // non-finite value is NaN, times a finite one 0)
#pragma unroll
        for (int t = 0; t < 4; ++t) vmax = fmax(vmax, fabs(yv[t]));
        ynan = fma((yv[0] + yv[1]) + (yv[2] + yv[3]), 0.0, ynan);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int x = t & 1, y = t >> 1;
            double v = acc[t];
            v = fma(-Cc.a0[t], y0[y], v);
            v = fma(-Cc.a1[t], y1[y], v);
            v = fma(-z0[x], Cc.b0[t], v);
            v = fma(-z1[x], Cc.b1[t], v);
            acc[t] = v;
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
    if (ynan != 0.0) vmax = __builtin_inf();
    wave_sync_lds();
    if (zo0 >= 0) dz[zo0] = zv0;
    if (zo1 >= 0) dz[zo1] = zv1;
    wave_sync_lds();
    if (vmax_out) {
        *vmax_out = vmax;
        return 1;
    }
    return vmax <= Tc ? 1 : 0;
}
__device__ __forceinline__ int leaf_solve(LeafLds &L, const LeafPatch &P, const LeafShape &RS, const LeafShape &CS,
                                          int nr, int nc, double Tc, double *vmax_out = nullptr)
{
    // with any 2x2 block, W comes from 4 x 4 factorisations whose pivoting may order its rows
    // freely: the full product; without, W is diagonal
    if (uniform((RS.two | CS.two) ? 1 : 0)) return leaf_solve_t<1>(L, P, RS, CS, nr, nc, Tc, vmax_out);
    return leaf_solve_t<0>(L, P, RS, CS, nr, nc, Tc, vmax_out);
}

}  // namespace trsyl
