/*
 * Plain FP64 CPU oracle for the robust triangular Sylvester solve
 *
 *     A Y + Y B = alpha C,      A (m x m), B (n x n) upper quasi-triangular,
 *
 * following Schwarz & Kjelgaard Mikkelsen, "Robust Task-Parallel Solution of the Triangular
 * Sylvester Equation" (arXiv 1905.10574), Sec. 2.
 *
 * TEST INFRASTRUCTURE.  This is a checker, not part of the product: only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no code, header or
 * constant generator with the GPU library.
 *
 * Conventions
 *   - Column-major storage with leading dimensions.  Only entries on or above the first
 *     subdiagonal of A and B are read.
 *   - Scale factors are powers of two carried as non-negative integer exponents:
 *     alpha = 2^-e.  (The paper's scalars in (0,1] underflow for strongly growing problems;
 *     an exponent never does.)
 *   - Overflow threshold OMEGA = 2^1022 (the paper only says "Omega > 0"; two factors of two
 *     below the largest double leave room for sums of two Omega-bounded numbers).
 *   - Matrix norms ||.||_inf are maximum absolute row sums, as in ProtectUpdate's contract.
 *
 * Parity pins for every routine live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <float.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMEGA 0x1p1022
#define EL(M, ld, i, j) ((M)[(size_t)(j) * (size_t)(ld) + (size_t)(i)])

enum { ORC_OK = 0, ORC_PERTURBED = 1, ORC_BAD_STRUCTURE = 2, ORC_BAD_INPUT = 3, ORC_NOMEM = 5 };

/* ------------------------------------------------------------------------------------------
 * Robust scalar primitives (Sec. 2.1).  The paper gives only their contracts; these are
 * power-of-two versions written from those contracts, so every scaling is exact.
 * ---------------------------------------------------------------------------------------- */

/* ProtectUpdate(c, a, y), Sec. 2.1: for 0 <= c, a, y <= OMEGA return s >= 0 such that
 * zeta = 2^-s satisfies zeta * (c + a*y) <= OMEGA.  s is the smallest such integer except when
 * the bound c + a*y had to be rounded and lies within a relative 2^-51 below a threshold: a
 * rounded bound is pushed up by that guard so the contract itself always holds.  a*y is never
 * formed unscaled, so nothing overflows. */
int orc_protect_update(double c, double a, double y)
{
    int ec = 0, ea = 0, ey = 0;
    double fc = frexp(c, &ec), fa = frexp(a, &ea), fy = frexp(y, &ey);
    double prod = fa * fy;                          /* in [0.25, 1) or 0 */
    double prod_err = fma(fa, fy, -prod);           /* exact rounding error of the product */
    int eprod = ea + ey;
    int K;
    if (prod == 0.0) K = ec;
    else if (fc == 0.0) K = eprod;
    else K = ec > eprod ? ec : eprod;
    double xc = ldexp(fc, ec - K), xp = ldexp(prod, eprod - K);
    double g = xc + xp;                             /* (c + a*y) * 2^-K, in (0, 2] */
    if (g == 0.0) return 0;
    double bv = g - xc, av = g - bv;                /* TwoSum: exact error of the addition */
    double sum_err = (xc - av) + (xp - bv);
    int exact = prod_err == 0.0 && sum_err == 0.0 && ldexp(xc, K - ec) == fc
                && ldexp(xp, K - eprod) == prod;
    if (!exact) g *= 1.0 + 0x1p-51;
    int eg = 0;
    double fg = frexp(g, &eg);
    long E = (long)eg + K;                          /* c + a*y <= fg * 2^E */
    long s = (fg == 0.5) ? E - 1023 : E - 1022;
    return s > 0 ? (int)s : 0;
}

/* ProtectDivision(b, t), Sec. 2.1: for |b| <= OMEGA and t != 0 return the smallest s >= 0 with
 * 2^-s |b| <= |t| OMEGA, so that (2^-s b) / t cannot exceed OMEGA. */
int orc_protect_division(double b, double t)
{
    double ab = fabs(b), at = fabs(t);
    if (ab == 0.0 || at >= 1.0) return 0;
    int eb = 0, et = 0;
    double fb = frexp(ab, &eb), ft = frexp(at, &et);
    long s = (long)eb - et - 1022 + (fb > ft ? 1 : 0);
    return s > 0 ? (int)s : 0;
}

/* ------------------------------------------------------------------------------------------
 * Structure: diagonal blocks (Sec. 1, eq. (4)) and tiles (Sec. 2.2).
 * ---------------------------------------------------------------------------------------- */

/* Block starts of an upper quasi-triangular matrix: a nonzero first-subdiagonal entry
 * T(i+1, i) opens a 2x2 block at i.  start must hold n+1 entries; start[nb] = n.  Returns the
 * number of blocks, or -1 if two consecutive subdiagonal entries are nonzero. */
int64_t orc_block_starts(int64_t n, const double *T, int64_t ldt, int64_t *start)
{
    int64_t nb = 0, i = 0;
    while (i < n) {
        start[nb++] = i;
        if (i + 1 < n && EL(T, ldt, i + 1, i) != 0.0) {
            if (i + 2 < n && EL(T, ldt, i + 2, i + 1) != 0.0) return -1;
            i += 2;
        } else {
            i += 1;
        }
    }
    start[nb] = n;
    return nb;
}

/* Tile boundaries for tile size t (Sec. 2.2: diagonal tiles are square and 2x2 blocks are not
 * split).  A nominal boundary b = t, 2t, ... that falls inside a 2x2 block (T(b, b-1) != 0)
 * moves down to b+1.  off must hold n/t + 2 entries; off[count] = n.  Returns the tile count. */
int64_t orc_tile_offsets(int64_t n, const double *T, int64_t ldt, int64_t t, int64_t *off)
{
    int64_t cnt = 0;
    off[cnt++] = 0;
    if (t < 1) t = 1;
    for (int64_t b = t; b < n; b += t) {
        int64_t bb = (EL(T, ldt, b, b - 1) != 0.0) ? b + 1 : b;
        if (bb >= n) break;
        if (bb > off[cnt - 1]) off[cnt++] = bb;
    }
    off[cnt] = n;
    return cnt;
}

/* ---------------------------------------------------------------------------------------- */

static double inf_norm(int64_t r, int64_t c, const double *M, int64_t ld)
{
    double best = 0.0;
    for (int64_t i = 0; i < r; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < c; ++j) s += fabs(EL(M, ld, i, j));
        if (s > best) best = s;
    }
    return best;
}

/* ||T||_inf of a square diagonal tile of a quasi-triangular matrix: only the entries on or above
 * the first subdiagonal belong to the matrix. */
static double quasi_inf_norm(int64_t r, const double *M, int64_t ld)
{
    double best = 0.0;
    for (int64_t i = 0; i < r; ++i) {
        double s = 0.0;
        for (int64_t j = (i > 0 ? i - 1 : 0); j < r; ++j) s += fabs(EL(M, ld, i, j));
        if (s > best) best = s;
    }
    return best;
}

static void scale_block(int64_t r, int64_t c, double *M, int64_t ld, long s)
{
    if (s == 0) return;
    for (int64_t j = 0; j < c; ++j)
        for (int64_t i = 0; i < r; ++i) EL(M, ld, i, j) = ldexp(EL(M, ld, i, j), (int)(-s));
}

/* Smallest s >= 0 with 2^-s ||M||_inf <= OMEGA, for entries each at most OMEGA (the row sums are
 * formed from 2^-16 |m_ij|, which cannot overflow for up to 2^16 columns). */
static long tile_excess_shift(int64_t r, int64_t c, const double *M, int64_t ld)
{
    double g = 0.0;
    for (int64_t i = 0; i < r; ++i) {
        double t = 0.0;
        for (int64_t j = 0; j < c; ++j) t += ldexp(fabs(EL(M, ld, i, j)), -16);
        if (t > g) g = t;
    }
    long s = 0;
    while (ldexp(g, (int)(16 - s)) > OMEGA) ++s;
    return s;
}

/* ------------------------------------------------------------------------------------------
 * Small Sylvester solve (Sec. 2.1): A11 Z + Z B11 = beta R with A11 r x r, B11 c x c,
 * r, c in {1, 2}, written as the Kronecker system K vec(Z) = beta vec(R),
 * K = I_c (x) A11 + B11^T (x) I_r (Bartels & Stewart), and solved by Gaussian elimination with
 * complete pivoting.  Every right-hand-side update is guarded by ProtectUpdate and every
 * division by ProtectDivision; each guard's factor rescales the whole vector and is folded
 * into beta = 2^-(*s_beta).  Pivots smaller than smin are replaced by +-smin (*perturbed = 1).
 * On return ||Z||_inf <= OMEGA.  R (ld ldr) is overwritten with Z.
 * ---------------------------------------------------------------------------------------- */
void orc_small_solve(int r, int c, const double *A11, int64_t lda, const double *B11, int64_t ldb,
                     double *R, int64_t ldr, double smin, int *s_beta, int *perturbed)
{
    int nn = r * c;
    double K[4][4], v[4];
    int perm[4] = {0, 1, 2, 3};
    long stot = 0;

    for (int q = 0; q < c; ++q)
        for (int p = 0; p < r; ++p) {
            int row = q * r + p;                   /* equation for Z(p, q) */
            v[row] = EL(R, ldr, p, q);
            for (int qq = 0; qq < c; ++qq)
                for (int pp = 0; pp < r; ++pp) {
                    int col = qq * r + pp;         /* unknown Z(pp, qq) */
                    double x = 0.0;
                    if (qq == q) x += EL(A11, lda, p, pp);
                    if (pp == p) x += EL(B11, ldb, qq, q);
                    K[row][col] = x;
                }
        }

    /* Keep elimination growth (at most 2 per step, three steps) below OMEGA. */
    double kmax = 0.0;
    for (int i = 0; i < nn; ++i)
        for (int j = 0; j < nn; ++j)
            if (fabs(K[i][j]) > kmax) kmax = fabs(K[i][j]);
    if (kmax > OMEGA / 8) {
        int ek = 0;
        frexp(kmax, &ek);
        int sig = ek - 1019;                       /* kmax * 2^-sig < 2^1019 = OMEGA/8 */
        for (int i = 0; i < nn; ++i) {
            v[i] = ldexp(v[i], -sig);
            for (int j = 0; j < nn; ++j) K[i][j] = ldexp(K[i][j], -sig);
        }
    }

    for (int t = 0; t < nn; ++t) {
        int pi = t, pj = t;
        double best = -1.0;
        for (int i = t; i < nn; ++i)
            for (int j = t; j < nn; ++j)
                if (fabs(K[i][j]) > best) { best = fabs(K[i][j]); pi = i; pj = j; }
        if (pi != t) {
            for (int j = 0; j < nn; ++j) { double x = K[t][j]; K[t][j] = K[pi][j]; K[pi][j] = x; }
            double x = v[t]; v[t] = v[pi]; v[pi] = x;
        }
        if (pj != t) {
            for (int i = 0; i < nn; ++i) { double x = K[i][t]; K[i][t] = K[i][pj]; K[i][pj] = x; }
            int x = perm[t]; perm[t] = perm[pj]; perm[pj] = x;
        }
        if (fabs(K[t][t]) < smin) {
            K[t][t] = (K[t][t] < 0.0) ? -smin : smin;
            *perturbed = 1;
        }
        for (int i = t + 1; i < nn; ++i) {
            double l = K[i][t] / K[t][t];
            for (int j = t + 1; j < nn; ++j) K[i][j] -= l * K[t][j];
            K[i][t] = 0.0;
            int s = orc_protect_update(fabs(v[i]), fabs(l), fabs(v[t]));
            if (s) { for (int q = 0; q < nn; ++q) v[q] = ldexp(v[q], -s); stot += s; }
            v[i] -= l * v[t];
        }
    }
    for (int i = nn - 1; i >= 0; --i) {
        for (int j = i + 1; j < nn; ++j) {
            int s = orc_protect_update(fabs(v[i]), fabs(K[i][j]), fabs(v[j]));
            if (s) { for (int q = 0; q < nn; ++q) v[q] = ldexp(v[q], -s); stot += s; }
            v[i] -= K[i][j] * v[j];
        }
        int s = orc_protect_division(v[i], K[i][i]);
        if (s) { for (int q = 0; q < nn; ++q) v[q] = ldexp(v[q], -s); stot += s; }
        v[i] /= K[i][i];
    }
    double z[4];
    for (int t = 0; t < nn; ++t) z[perm[t]] = v[t];
    /* each |z| <= OMEGA; a row of two may sum to 2*OMEGA: one halving restores ||Z||_inf <= OMEGA */
    double rowmax = 0.0;
    for (int p = 0; p < r; ++p) {
        double s = 0.0;
        for (int q = 0; q < c; ++q) s += fabs(z[q * r + p]);
        if (s > rowmax) rowmax = s;
    }
    if (rowmax > OMEGA) {
        for (int q = 0; q < nn; ++q) z[q] = ldexp(z[q], -1);
        stot += 1;
    }
    for (int q = 0; q < c; ++q)
        for (int p = 0; p < r; ++p) EL(R, ldr, p, q) = z[q * r + p];
    *s_beta = (int)stot;
}

/* ------------------------------------------------------------------------------------------
 * Algorithm 1 (NonRobustSyl): block backward substitution with no scaling at all.  Used only
 * as the control that must overflow on growth inputs.  Y (in: C) is overwritten.
 * ---------------------------------------------------------------------------------------- */
int orc_nonrobust_syl(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                      int64_t ldb, double *Y, int64_t ldy)
{
    int64_t *as = malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *bs = malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!as || !bs) { free(as); free(bs); return ORC_NOMEM; }
    int64_t p = orc_block_starts(m, A, lda, as), q = orc_block_starts(n, B, ldb, bs);
    if (p < 0 || q < 0) { free(as); free(bs); return ORC_BAD_STRUCTURE; }
    for (int64_t l = 0; l < q; ++l) {
        int64_t c0 = bs[l], c = bs[l + 1] - bs[l];
        for (int64_t k = p - 1; k >= 0; --k) {
            int64_t r0 = as[k], r = as[k + 1] - as[k];
            /* plain Kronecker solve by Cramer's rule / elimination without any guard */
            double K[4][4], v[4];
            int nn = (int)(r * c);
            for (int qq = 0; qq < c; ++qq)
                for (int pp = 0; pp < r; ++pp) {
                    int row = qq * (int)r + pp;
                    v[row] = EL(Y, ldy, r0 + pp, c0 + qq);
                    for (int q2 = 0; q2 < c; ++q2)
                        for (int p2 = 0; p2 < r; ++p2) {
                            double x = 0.0;
                            if (q2 == qq) x += EL(A, lda, r0 + pp, r0 + p2);
                            if (p2 == pp) x += EL(B, ldb, c0 + q2, c0 + qq);
                            K[row][q2 * (int)r + p2] = x;
                        }
                }
            for (int t = 0; t < nn; ++t)             /* partial pivoting, no guards */
            {
                int pi = t;
                for (int i = t + 1; i < nn; ++i) if (fabs(K[i][t]) > fabs(K[pi][t])) pi = i;
                for (int j = 0; j < nn; ++j) { double x = K[t][j]; K[t][j] = K[pi][j]; K[pi][j] = x; }
                double x = v[t]; v[t] = v[pi]; v[pi] = x;
                for (int i = t + 1; i < nn; ++i) {
                    double l = K[i][t] / K[t][t];
                    for (int j = t; j < nn; ++j) K[i][j] -= l * K[t][j];
                    v[i] -= l * v[t];
                }
            }
            for (int i = nn - 1; i >= 0; --i) {
                for (int j = i + 1; j < nn; ++j) v[i] -= K[i][j] * v[j];
                v[i] /= K[i][i];
            }
            for (int qq = 0; qq < c; ++qq)
                for (int pp = 0; pp < r; ++pp) EL(Y, ldy, r0 + pp, c0 + qq) = v[qq * (int)r + pp];
            /* Y(0:r0, block l) -= A(0:r0, block k) * Y_kl */
            for (int64_t jj = 0; jj < c; ++jj)
                for (int64_t kk = 0; kk < r; ++kk) {
                    double y = EL(Y, ldy, r0 + kk, c0 + jj);
                    for (int64_t i = 0; i < r0; ++i) EL(Y, ldy, i, c0 + jj) -= EL(A, lda, i, r0 + kk) * y;
                }
            /* Y(block k, c0+c:n) -= Y_kl * B(block l, c0+c:n) */
            for (int64_t j = c0 + c; j < n; ++j)
                for (int64_t kk = 0; kk < c; ++kk) {
                    double b = EL(B, ldb, c0 + kk, j);
                    for (int64_t i = 0; i < r; ++i) EL(Y, ldy, r0 + i, j) -= EL(Y, ldy, r0 + i, c0 + kk) * b;
                }
        }
    }
    free(as);
    free(bs);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------
 * Algorithm 2 (RobustSyl) on an arbitrary quasi-triangular pair, Sec. 2.1.  Block columns of
 * Y left to right, block rows bottom to top.  At each block: small robust solve (beta), then
 * the column update guarded by gamma_1 and the row update guarded by gamma_2; every factor
 * rescales the whole of Y and is accumulated into alpha = 2^-e.  Y-norms are recomputed exactly
 * where used; the A/B panel norms are precomputed.  Y (in: C, ld ldy) is overwritten.
 * ---------------------------------------------------------------------------------------- */
int orc_robust_syl(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                   int64_t ldb, double *Y, int64_t ldy, double smin, int64_t *e_out,
                   int *perturbed)
{
    *e_out = 0;
    if (m == 0 || n == 0) return ORC_OK;
    int64_t *as = malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *bs = malloc(sizeof(int64_t) * (size_t)(n + 1));
    double *anorm = malloc(sizeof(double) * (size_t)(m + 1));
    double *bnorm = malloc(sizeof(double) * (size_t)(n + 1));
    if (!as || !bs || !anorm || !bnorm) { free(as); free(bs); free(anorm); free(bnorm); return ORC_NOMEM; }
    int64_t p = orc_block_starts(m, A, lda, as), q = orc_block_starts(n, B, ldb, bs);
    if (p < 0 || q < 0) { free(as); free(bs); free(anorm); free(bnorm); return ORC_BAD_STRUCTURE; }

    /* anorm[k] = || A(0:as[k], block k) ||_inf ;  bnorm[l] = max_{j>l} || B(block l, block j) ||_inf */
    for (int64_t k = 0; k < p; ++k)
        anorm[k] = inf_norm(as[k], as[k + 1] - as[k], &EL(A, lda, 0, as[k]), lda);
    for (int64_t l = 0; l < q; ++l) {
        double best = 0.0;
        for (int64_t j = l + 1; j < q; ++j) {
            double x = inf_norm(bs[l + 1] - bs[l], bs[j + 1] - bs[j], &EL(B, ldb, bs[l], bs[j]), ldb);
            if (x > best) best = x;
        }
        bnorm[l] = best;
    }

    long e = 0;
    for (int64_t l = 0; l < q; ++l) {
        int64_t c0 = bs[l], c = bs[l + 1] - bs[l];
        for (int64_t k = p - 1; k >= 0; --k) {
            int64_t r0 = as[k], r = as[k + 1] - as[k];
            double Z[4];
            for (int64_t jj = 0; jj < c; ++jj)
                for (int64_t ii = 0; ii < r; ++ii) Z[jj * 2 + ii] = EL(Y, ldy, r0 + ii, c0 + jj);
            int sb = 0;
            orc_small_solve((int)r, (int)c, &EL(A, lda, r0, r0), lda, &EL(B, ldb, c0, c0), ldb, Z, 2,
                            smin, &sb, perturbed);
            if (sb) { scale_block(m, n, Y, ldy, sb); e += sb; }           /* Y <- beta Y */
            for (int64_t jj = 0; jj < c; ++jj)
                for (int64_t ii = 0; ii < r; ++ii) EL(Y, ldy, r0 + ii, c0 + jj) = Z[jj * 2 + ii];
            double znorm = inf_norm(r, c, Z, 2);

            if (r0 > 0) {                                                  /* column update */
                double ynorm = inf_norm(r0, c, &EL(Y, ldy, 0, c0), ldy);
                int s1 = orc_protect_update(ynorm, anorm[k], znorm);
                if (s1) {
                    scale_block(m, n, Y, ldy, s1); e += s1;
                    znorm = inf_norm(r, c, &EL(Y, ldy, r0, c0), ldy);
                }
                for (int64_t jj = 0; jj < c; ++jj)
                    for (int64_t kk = 0; kk < r; ++kk) {
                        double y = EL(Y, ldy, r0 + kk, c0 + jj);
                        for (int64_t i = 0; i < r0; ++i)
                            EL(Y, ldy, i, c0 + jj) -= EL(A, lda, i, r0 + kk) * y;
                    }
            }
            if (l + 1 < q) {                                               /* row update */
                double ynorm = 0.0;
                for (int64_t j = l + 1; j < q; ++j) {
                    double x = inf_norm(r, bs[j + 1] - bs[j], &EL(Y, ldy, r0, bs[j]), ldy);
                    if (x > ynorm) ynorm = x;
                }
                int s2 = orc_protect_update(ynorm, znorm, bnorm[l]);
                if (s2) { scale_block(m, n, Y, ldy, s2); e += s2; }
                for (int64_t j = c0 + c; j < n; ++j)
                    for (int64_t kk = 0; kk < c; ++kk) {
                        double b = EL(B, ldb, c0 + kk, j);
                        for (int64_t i = 0; i < r; ++i)
                            EL(Y, ldy, r0 + i, j) -= EL(Y, ldy, r0 + i, c0 + kk) * b;
                    }
            }
        }
    }
    *e_out = e;
    free(as); free(bs); free(anorm); free(bnorm);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------
 * Input checks shared by the drivers: finite entries, |entries| <= OMEGA, valid structure.
 * smin = max(2^-52 * max|A, B|, DBL_MIN) is the pivot floor of the small solves.
 * ---------------------------------------------------------------------------------------- */
static int check_quasi(int64_t n, const double *T, int64_t ld, double *maxabs)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t iend = (j + 2 < n) ? j + 2 : n;
        for (int64_t i = 0; i < iend; ++i) {
            double x = EL(T, ld, i, j);
            if (!(fabs(x) <= OMEGA)) return ORC_BAD_INPUT;
            if (fabs(x) > *maxabs) *maxabs = fabs(x);
        }
    }
    return ORC_OK;
}

double orc_smin(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb)
{
    double mx = 0.0;
    check_quasi(m, A, lda, &mx);
    check_quasi(n, B, ldb, &mx);
    double s = 0x1p-52 * mx;
    return s > DBL_MIN ? s : DBL_MIN;
}

/* ------------------------------------------------------------------------------------------
 * Algorithm 3 (RobustUpdate), Sec. 2.2, for the two shapes Algorithm 4 uses; one operand is
 * always an unscaled tile of A or B (scale 1).  With the target <gamma, C> = <2^-eC, C> and the
 * solved tile <2^-eY, Y>:
 *     eta  = min(gamma, alpha_Y)                    -> emax = max(eC, eY)
 *     zeta = ProtectUpdate((eta/gamma)||C||, ||T||, (eta/alpha_Y)||Y||)     (T = A_ik or B_lj)
 *     delta = eta * zeta                            -> new exponent emax + s
 *     D = (delta/gamma) C - T ((delta/alpha_Y) Y)   (column update)
 *     D = (delta/gamma) C - ((delta/alpha_Y) Y) T   (row update)
 * The printed update applies delta to both factors of the product; since delta^-1 D must equal
 * gamma^-1 C - alpha^-1 A beta^-1 B, delta enters the product once (here through Y).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int64_t m, n, pt, qt;
    const double *A, *B;
    int64_t lda, ldb, ldc;
    double *C;
    const int64_t *ro, *co;
    long *et;          /* pt x qt exponents, et[k * qt + l] */
    double *ynorm;     /* pt x qt tracked ||Y_kl||_inf */
    double *anorm;     /* pt x pt: ||A_ik||_inf */
    double *bnorm;     /* qt x qt: ||B_lj||_inf */
} tiled_t;

#define TILE(P, M, ld, i0, j0) (&EL((M), (ld), (i0), (j0)))

static void update_col(tiled_t *T, int64_t i, int64_t l, int64_t k, double *tmp)
{
    /* target (i, l) -= A_ik * Y_kl */
    int64_t ri = T->ro[i + 1] - T->ro[i], rk = T->ro[k + 1] - T->ro[k], cl = T->co[l + 1] - T->co[l];
    long eC = T->et[i * T->qt + l], eY = T->et[k * T->qt + l];
    long emax = eC > eY ? eC : eY;
    double cn = ldexp(T->ynorm[i * T->qt + l], (int)(eC - emax));
    double yn = ldexp(T->ynorm[k * T->qt + l], (int)(eY - emax));
    int s = orc_protect_update(cn, T->anorm[i * T->pt + k], yn);
    long enew = emax + s;
    double *Ct = TILE(T, T->C, T->ldc, T->ro[i], T->co[l]);
    const double *Yt = TILE(T, T->C, T->ldc, T->ro[k], T->co[l]);
    const double *At = &EL(T->A, T->lda, T->ro[i], T->ro[k]);
    scale_block(ri, cl, Ct, T->ldc, enew - eC);
    for (int64_t j = 0; j < cl; ++j)
        for (int64_t x = 0; x < rk; ++x) tmp[j * rk + x] = ldexp(EL(Yt, T->ldc, x, j), (int)(eY - enew));
    for (int64_t j = 0; j < cl; ++j)
        for (int64_t x = 0; x < rk; ++x) {
            double y = tmp[j * rk + x];
            for (int64_t r = 0; r < ri; ++r) EL(Ct, T->ldc, r, j) -= EL(At, T->lda, r, x) * y;
        }
    T->et[i * T->qt + l] = enew;
    T->ynorm[i * T->qt + l] = inf_norm(ri, cl, Ct, T->ldc);
}

static void update_row(tiled_t *T, int64_t k, int64_t j, int64_t l, double *tmp)
{
    /* target (k, j) -= Y_kl * B_lj */
    int64_t rk = T->ro[k + 1] - T->ro[k], cl = T->co[l + 1] - T->co[l], cj = T->co[j + 1] - T->co[j];
    long eC = T->et[k * T->qt + j], eY = T->et[k * T->qt + l];
    long emax = eC > eY ? eC : eY;
    double cn = ldexp(T->ynorm[k * T->qt + j], (int)(eC - emax));
    double yn = ldexp(T->ynorm[k * T->qt + l], (int)(eY - emax));
    int s = orc_protect_update(cn, yn, T->bnorm[l * T->qt + j]);
    long enew = emax + s;
    double *Ct = TILE(T, T->C, T->ldc, T->ro[k], T->co[j]);
    const double *Yt = TILE(T, T->C, T->ldc, T->ro[k], T->co[l]);
    const double *Bt = &EL(T->B, T->ldb, T->co[l], T->co[j]);
    scale_block(rk, cj, Ct, T->ldc, enew - eC);
    for (int64_t x = 0; x < cl; ++x)
        for (int64_t r = 0; r < rk; ++r) tmp[x * rk + r] = ldexp(EL(Yt, T->ldc, r, x), (int)(eY - enew));
    for (int64_t jj = 0; jj < cj; ++jj)
        for (int64_t x = 0; x < cl; ++x) {
            double b = EL(Bt, T->ldb, x, jj);
            for (int64_t r = 0; r < rk; ++r) EL(Ct, T->ldc, r, jj) -= tmp[x * rk + r] * b;
        }
    T->et[k * T->qt + j] = enew;
    T->ynorm[k * T->qt + j] = inf_norm(rk, cj, Ct, T->ldc);
}

/* ------------------------------------------------------------------------------------------
 * Algorithm 4 (tiled robust solver), Sec. 2.2, with plain loops.  Tiles of size tA x tB (2x2
 * blocks never split); every tile of Y carries its own exponent.  Tile rows bottom to top,
 * tile columns left to right: RobustSyl on the tile (its beta multiplies the tile's existing
 * scale), then RobustUpdate of every tile above in the same tile column and every tile right
 * in the same tile row.  Finally alpha = min alpha_kl and each tile is rescaled to alpha.
 * The updates issued by one solved tile write disjoint tiles, so they may run in parallel
 * (nthreads > 1) without changing any result.  C (ld ldc) is overwritten with Y; e: alpha=2^-e.
 * Returns 0, 1 (a pivot was perturbed), 2 (bad structure), 3 (non-finite or > OMEGA input, or a
 * tile of A, B or C whose infinity norm exceeds OMEGA).
 * ---------------------------------------------------------------------------------------- */
int orc_drsylv(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
               double *C, int64_t ldc, int64_t tA, int64_t tB, int nthreads, int64_t *e_out)
{
    *e_out = 0;
    if (m == 0 || n == 0) return ORC_OK;
    double mx = 0.0;
    if (check_quasi(m, A, lda, &mx) || check_quasi(n, B, ldb, &mx)) return ORC_BAD_INPUT;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            if (!(fabs(EL(C, ldc, i, j)) <= OMEGA)) return ORC_BAD_INPUT;
    double smin = 0x1p-52 * mx;
    if (smin < DBL_MIN) smin = DBL_MIN;

    int64_t *as = malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *bs = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *ro = malloc(sizeof(int64_t) * (size_t)(m / (tA > 0 ? tA : 1) + 2));
    int64_t *co = malloc(sizeof(int64_t) * (size_t)(n / (tB > 0 ? tB : 1) + 2));
    if (!as || !bs || !ro || !co) { free(as); free(bs); free(ro); free(co); return ORC_NOMEM; }
    if (orc_block_starts(m, A, lda, as) < 0 || orc_block_starts(n, B, ldb, bs) < 0) {
        free(as); free(bs); free(ro); free(co);
        return ORC_BAD_STRUCTURE;
    }
    free(as); free(bs);
    tiled_t T;
    T.m = m; T.n = n; T.A = A; T.B = B; T.C = C; T.lda = lda; T.ldb = ldb; T.ldc = ldc;
    T.pt = orc_tile_offsets(m, A, lda, tA, ro);
    T.qt = orc_tile_offsets(n, B, ldb, tB, co);
    T.ro = ro; T.co = co;
    int64_t pt = T.pt, qt = T.qt;
    T.et = calloc((size_t)(pt * qt), sizeof(long));
    T.ynorm = calloc((size_t)(pt * qt), sizeof(double));
    T.anorm = calloc((size_t)(pt * pt), sizeof(double));
    T.bnorm = calloc((size_t)(qt * qt), sizeof(double));
    if (!T.et || !T.ynorm || !T.anorm || !T.bnorm) {
        free(ro); free(co); free(T.et); free(T.ynorm); free(T.anorm); free(T.bnorm);
        return ORC_NOMEM;
    }
    /* Bound: ||A_ik||_inf (i < k), ||B_lj||_inf (l < j), and the initial ||C_kl||_inf */
    for (int64_t k = 0; k < pt; ++k)
        for (int64_t i = 0; i < k; ++i)
            T.anorm[i * pt + k] = inf_norm(ro[i + 1] - ro[i], ro[k + 1] - ro[k], &EL(A, lda, ro[i], ro[k]), lda);
    for (int64_t j = 0; j < qt; ++j)
        for (int64_t l = 0; l < j; ++l)
            T.bnorm[l * qt + j] = inf_norm(co[l + 1] - co[l], co[j + 1] - co[j], &EL(B, ldb, co[l], co[j]), ldb);
    for (int64_t k = 0; k < pt; ++k)
        for (int64_t l = 0; l < qt; ++l)
            T.ynorm[k * qt + l] = inf_norm(ro[k + 1] - ro[k], co[l + 1] - co[l], &EL(C, ldc, ro[k], co[l]), ldc);
    /* The data requirement of Algorithm 4: every tile of A, B and C in this partition has
     * infinity norm at most OMEGA.  Entries at most OMEGA do not imply it (a row sum runs over a
     * tile's width of them), so the tile norms are checked as well. */
    {
        int bad = 0;
        for (int64_t k = 0; k < pt; ++k) {
            for (int64_t i = 0; i < k; ++i) bad |= !(T.anorm[i * pt + k] <= OMEGA);
            bad |= !(quasi_inf_norm(ro[k + 1] - ro[k], &EL(A, lda, ro[k], ro[k]), lda) <= OMEGA);
        }
        for (int64_t j = 0; j < qt; ++j) {
            for (int64_t l = 0; l < j; ++l) bad |= !(T.bnorm[l * qt + j] <= OMEGA);
            bad |= !(quasi_inf_norm(co[j + 1] - co[j], &EL(B, ldb, co[j], co[j]), ldb) <= OMEGA);
        }
        for (int64_t t = 0; t < pt * qt; ++t) bad |= !(T.ynorm[t] <= OMEGA);
        if (bad) {
            free(ro); free(co); free(T.et); free(T.ynorm); free(T.anorm); free(T.bnorm);
            return ORC_BAD_INPUT;
        }
    }

    int64_t tmax = 0;
    for (int64_t k = 0; k < pt; ++k) if (ro[k + 1] - ro[k] > tmax) tmax = ro[k + 1] - ro[k];
    int64_t cmax = 0;
    for (int64_t l = 0; l < qt; ++l) if (co[l + 1] - co[l] > cmax) cmax = co[l + 1] - co[l];
    int nth = nthreads > 0 ? nthreads : 1;
#ifndef _OPENMP
    nth = 1;
#endif
    double *tmp = malloc(sizeof(double) * (size_t)(tmax * cmax) * (size_t)nth);
    if (!tmp) {
        free(ro); free(co); free(T.et); free(T.ynorm); free(T.anorm); free(T.bnorm);
        return ORC_NOMEM;
    }
    int perturbed = 0;
    for (int64_t k = pt - 1; k >= 0; --k) {
        for (int64_t l = 0; l < qt; ++l) {
            int64_t e_syl = 0;
            orc_robust_syl(ro[k + 1] - ro[k], co[l + 1] - co[l], &EL(A, lda, ro[k], ro[k]), lda,
                           &EL(B, ldb, co[l], co[l]), ldb, &EL(C, ldc, ro[k], co[l]), ldc, smin,
                           &e_syl, &perturbed);
            T.et[k * qt + l] += e_syl;
            /* Algorithm 2 bounds its 1x1 / 2x2 blocks by OMEGA, Algorithm 4 needs the tile's
             * ||Y_kl||_inf <= OMEGA (its postcondition and Algorithm 3's precondition): a tile
             * whose row sums exceed OMEGA is scaled by the smallest power of two that fixes it,
             * folded into its scale (reading S23) */
            {
                const long sx = tile_excess_shift(ro[k + 1] - ro[k], co[l + 1] - co[l], &EL(C, ldc, ro[k], co[l]), ldc);
                if (sx) {
                    scale_block(ro[k + 1] - ro[k], co[l + 1] - co[l], &EL(C, ldc, ro[k], co[l]), ldc, sx);
                    T.et[k * qt + l] += sx;
                }
            }
            T.ynorm[k * qt + l] = inf_norm(ro[k + 1] - ro[k], co[l + 1] - co[l], &EL(C, ldc, ro[k], co[l]), ldc);
            int64_t nupd = k + (qt - 1 - l);
#pragma omp parallel for num_threads(nth) schedule(dynamic, 1) if (nth > 1 && nupd > 1)
            for (int64_t u = 0; u < nupd; ++u) {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                double *mytmp = tmp + (size_t)tid * (size_t)(tmax * cmax);
                if (u < k) update_col(&T, k - 1 - u, l, k, mytmp);
                else update_row(&T, k, l + 1 + (u - k), l, mytmp);
            }
        }
    }
    long e = 0;
    for (int64_t t = 0; t < pt * qt; ++t) if (T.et[t] > e) e = T.et[t];
    for (int64_t k = 0; k < pt; ++k)
        for (int64_t l = 0; l < qt; ++l)
            scale_block(ro[k + 1] - ro[k], co[l + 1] - co[l], &EL(C, ldc, ro[k], co[l]), ldc, e - T.et[k * qt + l]);
    *e_out = e;
    free(tmp); free(ro); free(co); free(T.et); free(T.ynorm); free(T.anorm); free(T.bnorm);
    return perturbed ? ORC_PERTURBED : ORC_OK;
}

/* Whole-problem RobustSyl driver with the same input checks and smin as orc_drsylv. */
int orc_robust_syl_driver(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                          int64_t ldb, double *C, int64_t ldc, int64_t *e_out)
{
    *e_out = 0;
    if (m == 0 || n == 0) return ORC_OK;
    double mx = 0.0;
    if (check_quasi(m, A, lda, &mx) || check_quasi(n, B, ldb, &mx)) return ORC_BAD_INPUT;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            if (!(fabs(EL(C, ldc, i, j)) <= OMEGA)) return ORC_BAD_INPUT;
    double smin = 0x1p-52 * mx;
    if (smin < DBL_MIN) smin = DBL_MIN;
    int perturbed = 0;
    int rc = orc_robust_syl(m, n, A, lda, B, ldb, C, ldc, smin, e_out, &perturbed);
    if (rc) return rc;
    return perturbed ? ORC_PERTURBED : ORC_OK;
}

/* ------------------------------------------------------------------------------------------
 * Adjoint problem A^T G + G B^T = alpha W.  With the order-reversing permutations P (m x m) and
 * Q (n x n), P A^T P and Q B^T Q are again upper quasi-triangular, and G = P Gh Q where
 * (P A^T P) Gh + Gh (Q B^T Q) = alpha (P W Q).  The oracle forms the flipped problem
 * explicitly and calls Algorithm 4.  W (ld ldw) is overwritten with G (scaled by alpha).
 * ---------------------------------------------------------------------------------------- */
int orc_adjoint(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                double *W, int64_t ldw, int64_t tA, int64_t tB, int nthreads, int64_t *e_out)
{
    *e_out = 0;
    if (m == 0 || n == 0) return ORC_OK;
    double *Af = calloc((size_t)(m * m), sizeof(double));
    double *Bf = calloc((size_t)(n * n), sizeof(double));
    double *Wf = malloc(sizeof(double) * (size_t)(m * n));
    if (!Af || !Bf || !Wf) { free(Af); free(Bf); free(Wf); return ORC_NOMEM; }
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i)
            if (i <= j + 1) EL(Af, m, i, j) = EL(A, lda, m - 1 - j, m - 1 - i);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            if (i <= j + 1) EL(Bf, n, i, j) = EL(B, ldb, n - 1 - j, n - 1 - i);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) EL(Wf, m, i, j) = EL(W, ldw, m - 1 - i, n - 1 - j);
    int rc = orc_drsylv(m, n, Af, m, Bf, n, Wf, m, tA, tB, nthreads, e_out);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) EL(W, ldw, i, j) = EL(Wf, m, m - 1 - i, n - 1 - j);
    free(Af); free(Bf); free(Wf);
    return rc;
}

/* ------------------------------------------------------------------------------------------
 * Relative residual, eq. (9):  ||R||_F / ((||A||_F + ||B||_F) ||Y||_F + ||alpha C||_F),
 * R = alpha C - (A Y + Y B), alpha = 2^-e.  The quotient is unchanged when Y and alpha are
 * multiplied by the same power of two, so Y is brought to max|Y| <= 1 first; sums are kept in
 * long double.  Only the quasi-triangular part of A and B is read.
 * ---------------------------------------------------------------------------------------- */
static int ynorm_shift(int64_t m, int64_t n, const double *Y, int64_t ldy)
{
    double ymax = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) if (fabs(EL(Y, ldy, i, j)) > ymax) ymax = fabs(EL(Y, ldy, i, j));
    int ey = 0;
    if (ymax > 0.0) frexp(ymax, &ey);
    return ey;                                    /* ymax * 2^-ey < 1 */
}

double orc_relres(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                  const double *Y, int64_t ldy, int64_t e, const double *C, int64_t ldc)
{
    if (m == 0 || n == 0) return 0.0;
    int sy = ynorm_shift(m, n, Y, ldy);
    long double alpha = ldexpl(1.0L, (int)(-(e + sy)));
    long double rr = 0.0L, yy = 0.0L, aa = 0.0L, bb = 0.0L, cc = 0.0L;
    long double *col = malloc(sizeof(long double) * (size_t)m);
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) col[i] = alpha * (long double)EL(C, ldc, i, j);
        for (int64_t k = 0; k < m; ++k) {                   /* (A Y)(:, j) */
            long double y = ldexpl((long double)EL(Y, ldy, k, j), -sy);
            int64_t iend = (k + 2 < m) ? k + 2 : m;
            for (int64_t i = 0; i < iend; ++i) col[i] -= (long double)EL(A, lda, i, k) * y;
        }
        int64_t kend = (j + 2 < n) ? j + 2 : n;
        for (int64_t k = 0; k < kend; ++k) {                 /* (Y B)(:, j) */
            long double b = (long double)EL(B, ldb, k, j);
            if (b == 0.0L) continue;
            for (int64_t i = 0; i < m; ++i) col[i] -= ldexpl((long double)EL(Y, ldy, i, k), -sy) * b;
        }
        for (int64_t i = 0; i < m; ++i) {
            rr += col[i] * col[i];
            long double y = ldexpl((long double)EL(Y, ldy, i, j), -sy);
            yy += y * y;
            long double c = alpha * (long double)EL(C, ldc, i, j);
            cc += c * c;
        }
    }
    for (int64_t j = 0; j < m; ++j) {
        int64_t iend = (j + 2 < m) ? j + 2 : m;
        for (int64_t i = 0; i < iend; ++i) aa += (long double)EL(A, lda, i, j) * EL(A, lda, i, j);
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t iend = (j + 2 < n) ? j + 2 : n;
        for (int64_t i = 0; i < iend; ++i) bb += (long double)EL(B, ldb, i, j) * EL(B, ldb, i, j);
    }
    free(col);
    long double den = (sqrtl(aa) + sqrtl(bb)) * sqrtl(yy) + sqrtl(cc);
    if (den == 0.0L) return 0.0;
    return (double)(sqrtl(rr) / den);
}

/* Eq. (9) restricted to a set of rows: returns sum over the listed rows of |R_ij|^2 and of
 * |Y_ij|^2 and |alpha C_ij|^2 (after the same power-of-two normalisation by 2^-shift, which the
 * caller passes so that several row sets share one scale).  Used for sampled checks of large
 * solves, where the full residual is too costly for the CPU. */
void orc_residual_rows(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                       int64_t ldb, const double *Y, int64_t ldy, int64_t e, const double *C,
                       int64_t ldc, int shift, int64_t nrows, const int64_t *rows, double *out3)
{
    long double alpha = ldexpl(1.0L, (int)(-(e + shift)));
    long double rr = 0.0L, yy = 0.0L, cc = 0.0L;
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows[t];
        int64_t kstart = i > 0 ? i - 1 : 0;
        for (int64_t j = 0; j < n; ++j) {
            long double r = alpha * (long double)EL(C, ldc, i, j);
            for (int64_t k = kstart; k < m; ++k)
                r -= (long double)EL(A, lda, i, k) * ldexpl((long double)EL(Y, ldy, k, j), -shift);
            int64_t kend = (j + 2 < n) ? j + 2 : n;
            for (int64_t k = 0; k < kend; ++k)
                r -= ldexpl((long double)EL(Y, ldy, i, k), -shift) * (long double)EL(B, ldb, k, j);
            rr += r * r;
            long double y = ldexpl((long double)EL(Y, ldy, i, j), -shift);
            yy += y * y;
            long double c = alpha * (long double)EL(C, ldc, i, j);
            cc += c * c;
        }
    }
    out3[0] = (double)rr;
    out3[1] = (double)yy;
    out3[2] = (double)cc;
}
