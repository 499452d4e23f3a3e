// Kernels behind the entry points other than the forward solve:
//
//  * order-reversal transposes that map the adjoint equation A^T G + G B^T = alpha W onto the
//    forward solver (P A^T P and Q B^T Q are upper quasi-triangular when A and B are, with the
//    1x1 / 2x2 block structure reversed; P, Q reverse the index order);
//  * a general FP64 MFMA GEMM  Out = cs * Cin + as * Aop Bop  with strided operands, optional
//    quasi-triangular operand structure (entries outside it are never read), an optional
//    quasi-triangular output pattern, and power-of-two scales taken from exponents in device
//    memory -- used for the gradient products dA = -G Y^T, dB = -Y^T G and for the residual of
//    eq. (9);
//  * scale-safe Frobenius norms (max first, then a sum of squares of power-of-two-scaled entries,
//    reduced in a fixed order).
#include "device_common.hpp"
#include "extras.hpp"

namespace trsyl {

constexpr int kGT = 128;      // output tile of the GEMM
constexpr int kGK = 16;       // k per LDS stage
constexpr int kGS = kGT + 2;  // padded LDS row

// ---------------------------------------------------------------------------------------------
// D(p, q) = sign * T(p, q), or sign * T(n-1-q, n-1-p) with flip (the order-reversed transpose
// P T^T P, again upper quasi-triangular), on and above the first subdiagonal; zero below.
// ---------------------------------------------------------------------------------------------
__global__ void k_quasi_copy(const double *T, int64_t ldt, int n, int flip, double sign, double *D)
{
    const int64_t tot = (int64_t)n * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(t % n), q = (int)(t / n);
        double v = 0.0;
        if (p <= q + 1) {
            const double x = flip ? ldg(T + (int64_t)(n - 1 - p) * ldt + (n - 1 - q))
                                  : ldg(T + (int64_t)q * ldt + p);
            v = sign * x;
        }
        stg(D + (int64_t)q * n + p, v);
    }
}

// In place: W(i, j) <-> W(m-1-i, n-1-j) (rows and cols), W(m-1-i, j) (rows only) or
// W(i, n-1-j) (cols only); each pair is swapped by one thread.
__global__ void k_flip_axes(double *W, int64_t ldw, int m, int n, int rows, int cols)
{
    const int mh = m / 2, nh = n / 2;
    const int64_t pairs = rows && cols ? (int64_t)m * n / 2 : rows ? (int64_t)mh * n : (int64_t)m * nh;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < pairs;
         e += (int64_t)gridDim.x * blockDim.x) {
        int i, j, i2, j2;
        if (rows && cols) { i = (int)(e % m); j = (int)(e / m); i2 = m - 1 - i; j2 = n - 1 - j; }
        else if (rows) { i = (int)(e % mh); j = (int)(e / mh); i2 = m - 1 - i; j2 = j; }
        else { i = (int)(e % m); j = (int)(e / m); i2 = i; j2 = n - 1 - j; }
        double *p = W + (int64_t)j * ldw + i;
        double *q = W + (int64_t)j2 * ldw + i2;
        const double a = ldg(p), b = ldg(q);
        stg(p, b);
        stg(q, a);
    }
}

// ---------------------------------------------------------------------------------------------
// Power-of-two shift that brings a Frobenius norm 2^s sqrt(t) (launch_norm) to OMEGA = 2^1022 or
// below: *negshift = -shift, *total += shift.
// ---------------------------------------------------------------------------------------------
__global__ void k_norm_shift(const int32_t *s, const double *t, int64_t *negshift, int64_t *total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t shift = 0;
    if (*s != 0x7FFFFFFF && *t > 0.0) {
        const int64_t h = (int64_t)*s + ilogb(sqrt(*t)) + 1;     // 2^h > the norm
        shift = h > 1022 ? h - 1022 : 0;
    }
    *negshift = -shift;
    *total += shift;
}

// *e += *add; *scale = 2^-e (0 once e > 1074); scale may be null.
__global__ void k_add_exponent(int64_t *e, double *scale, const int64_t *add)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t v = *e + *add;
    *e = v;
    if (scale) *scale = v > 1074 ? 0.0 : ldexp(1.0, (int)-v);
}

// ---------------------------------------------------------------------------------------------
// GEMM.  One workgroup of 512 threads computes a 128 x 128 output tile: wave w = 4 wr + wc owns
// the 4 x 2 blocks of 16 x 16 at rows 16 (4 wr) .., columns 16 (2 wc) .., accumulated with
// v_mfma_f64_16x16x4 from double-buffered LDS stages of 16 k.  Operand values outside the
// matrices or outside a quasi-triangular operand's structure are staged as zeros (and never
// loaded).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double exp_scale(double sign, int e0, int e1, int e2, const int64_t *p1,
                                            const int64_t *p2)
{
    int64_t e = e0;
    if (e1) e += (int64_t)e1 * *p1;
    if (e2) e += (int64_t)e2 * *p2;
    if (e > 2100) e = 2100;
    if (e < -2100) e = -2100;
    return ldexp(sign, (int)e);
}

struct GemmLds {
    double As[2][kGK][kGS];
    double Bs[2][kGK][kGS];
};

__global__ void __launch_bounds__(512) k_gemm(GemmDesc g)
{
    __shared__ GemmLds L;
    if (g.skip && __builtin_amdgcn_readfirstlane(*(volatile const int32_t *)g.skip) != 0) return;
    const int m0 = kGT * blockIdx.x, n0 = kGT * blockIdx.y;
    const int w = uniform((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const int wr = w >> 2, wc = w & 3;
    const double as = exp_scale(g.asign, g.ae0, g.ae1, g.ae2, g.ep1, g.ep2);
    const double cs = g.Cin ? exp_scale(g.csign, g.ce0, g.ce1, g.ce2, g.ep1, g.ep2) : 0.0;
    const double sa = g.sa1 ? exp_scale(1.0, 0, g.sa1, 0, g.ep1, g.ep2) : 1.0;
    const double sb = g.sb1 ? exp_scale(1.0, 0, g.sb1, 0, g.ep1, g.ep2) : 1.0;
    const int Mp = g.M - m0 < kGT ? g.M - m0 : kGT, Np = g.N - n0 < kGT ? g.N - n0 : kGT;

    // k range that can contribute to this tile
    int klo = 0, khi = g.K;
    if (g.triA && m0 - 1 > klo) klo = m0 - 1;
    if (g.triB && n0 + kGT + 1 < khi) khi = n0 + kGT + 1;
    const bool below = g.mask && m0 > n0 + kGT;        // tile entirely below the output pattern

    d4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a) { acc[a][0] = zero4(); acc[a][1] = zero4(); }

    if (!below && klo < khi) {
        double ra[4], rb[4];
        auto load = [&](int kc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = threadIdx.x + 512 * i;       // 2048 = 16 x 128 elements each
                {
                    const int m = e & 127, k = kc + (e >> 7);
                    const int gm = m0 + m;
                    bool ok = m < Mp && k < khi;
                    if (g.triA) ok = ok && k >= gm - 1;
                    const double v = ldg(g.A + (int64_t)(ok ? gm : m0) * g.sAm + (int64_t)(ok ? k : klo) * g.sAk);
                    ra[i] = ok ? v * sa : 0.0;
                }
                {
                    const int k = kc + (e & 15), n = e >> 4;
                    const int gn = n0 + n;
                    bool ok = n < Np && k < khi;
                    if (g.triB) ok = ok && k <= gn + 1;
                    const double v = ldg(g.B + (int64_t)(ok ? k : klo) * g.sBk + (int64_t)(ok ? gn : n0) * g.sBn);
                    rb[i] = ok ? v * sb : 0.0;
                }
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = threadIdx.x + 512 * i;
                L.As[buf][e >> 7][e & 127] = ra[i];
                L.Bs[buf][e & 15][e >> 4] = rb[i];
            }
        };
        const int nkc = (khi - klo + kGK - 1) / kGK;
        load(klo);
        store(0);
        __syncthreads();
        for (int c = 0; c < nkc; ++c) {
            const int buf = c & 1;
            const bool more = c + 1 < nkc;
            if (more) load(klo + kGK * (c + 1));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 4 * q + j;
                double av[4], bv[2];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = L.As[buf][k][16 * (4 * wr + a) + r];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = L.Bs[buf][k][16 * (2 * wc + b) + r];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
            }
            if (more) store(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue (result lane layout: row 16 a + r, columns 16 b + q + 4 i)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = m0 + 16 * (4 * wr + a) + r;
        if (i >= g.M) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = n0 + 16 * (2 * wc + b) + q + 4 * t;
                if (j >= g.N) continue;
                double v = as * acc[a][b][t];
                if (g.Cin) v += cs * ldg(g.Cin + (int64_t)j * g.ldcin + i);
                if (g.mask) {
                    bool keep = i <= j;
                    if (i == j + 1) keep = ldg(g.pat + (int64_t)j * g.ldpat + i) != 0.0;
                    if (!keep) v = 0.0;
                }
                stg(g.Out + (int64_t)j * g.ldo + i, v);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Norms.  part[b] of block b: the block's partial over a grid-stride range.  Pattern 1 restricts
// to the quasi-triangular pattern of a square matrix (on or above the first subdiagonal).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}
__device__ __forceinline__ double block_max(double v, double *red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmax(s, red[i]);
    return s;
}

// pass 0: partial max |x|;  pass 1: partial sum of (x 2^-s)^2 with 2^s the power of two at or
// above the max (s read from *sexp).
__global__ void k_norm_part(const double *X, int64_t ld, int rows, int cols, int pattern, int pass,
                            const int32_t *sexp, double *part, const int32_t *skip)
{
    __shared__ double red[16];
    if (skip && __builtin_amdgcn_readfirstlane(*(volatile const int32_t *)skip) != 0) return;
    const int64_t tot = (int64_t)rows * cols;
    const int s = pass ? *sexp : 0;
    double v = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % rows), j = (int)(t / rows);
        if (pattern && i > j + 1) continue;
        const double x = ldg(X + (int64_t)j * ld + i);
        if (pass == 0) v = fmax(v, fabs(x));
        else { const double y = ldexp(x, -s); v = fma(y, y, v); }
    }
    const double r = pass == 0 ? block_max(v, red) : block_sum(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// Reduces nparts partials in order.  pass 0: *sexp = the exponent s with 2^s >= max (0 for a
// zero matrix) and a non-finite max is flagged by s = INT32_MAX.  pass 1: out[0] = sum, so the
// norm is 2^s sqrt(out[0]).
__global__ void k_norm_final(const double *part, int nparts, int pass, int32_t *sexp, double *out,
                             const int32_t *skip)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (skip && *skip) return;
    if (pass == 0) {
        double m = 0.0;
        bool bad = false;
        for (int i = 0; i < nparts; ++i) {
            if (!(part[i] <= 1.7976931348623157e308)) bad = true;
            m = fmax(m, part[i]);
        }
        int s = 0;
        if (bad) s = 0x7FFFFFFF;
        else if (m > 0.0) {
            s = ilogb(m) + 1;                      // 2^s > m
        }
        *sexp = s;
    } else {
        double t = 0.0;
        for (int i = 0; i < nparts; ++i) t += part[i];
        out[0] = t;
    }
}

// ---------------------------------------------------------------------------------------------
// Residual quotient of eq. (9) from the norm pairs (2^s sqrt(t)) of R, A, B, Y and C, with R and
// the Y, C scales described in trsyl_residual: Y is used as Ys = 2^-sy Y and alpha C as
// 2^-(e + sy) C.
// ---------------------------------------------------------------------------------------------
__device__ double residual_quotient(const int32_t *s5, const double *t5, const int64_t *e)
{
    for (int i = 0; i < 5; ++i)
        if (s5[i] == 0x7FFFFFFF || !(t5[i] <= 1.7976931348623157e308)) return __builtin_nan("");
    // norms as (mantissa, exponent): R, A, B, Ys, aC
    const int sy = s5[3];
    double v[5];
    int64_t x[5];
    for (int i = 0; i < 5; ++i) { v[i] = sqrt(t5[i]); x[i] = s5[i]; }
    x[3] -= sy;                    // Ys = 2^-sy Y
    x[4] -= (*e + sy);             // 2^-(e + sy) C
    // denominator D = (A + B) Ys + aC, in a common exponent
    const int64_t xab = x[1] > x[2] ? x[1] : x[2];
    const double ab = ldexp(v[1], (int)(x[1] - xab > -3000 ? x[1] - xab : -3000)) +
                      ldexp(v[2], (int)(x[2] - xab > -3000 ? x[2] - xab : -3000));
    const int64_t xp = xab + x[3];
    const double p = ab * v[3];
    const int64_t xd = xp > x[4] ? xp : x[4];
    const double d = ldexp(p, (int)(xp - xd > -3000 ? xp - xd : -3000)) +
                     ldexp(v[4], (int)(x[4] - xd > -3000 ? x[4] - xd : -3000));
    if (d == 0.0) return v[0] == 0.0 ? 0.0 : __builtin_inf();
    int64_t xq = x[0] - xd;
    if (xq > 3000) xq = 3000;
    if (xq < -3000) xq = -3000;
    return ldexp(v[0] / d, (int)xq);
}

__global__ void k_residual_final(const int32_t *s5, const double *t5, const int64_t *e, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *out = residual_quotient(s5, t5, e);
}

__global__ void k_refine_check(const int32_t *s5, const double *t5, const int64_t *e, double tol, int32_t *skip)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (*skip) return;
    const double q = residual_quotient(s5, t5, e);
    if (q <= tol) *skip = 1;
}

// dC = 2^(eG - eY) G
__global__ void k_scale_copy(const double *G, int64_t ldg_, int m, int n, const int64_t *eG,
                             const int64_t *eY, double *dC, int64_t lddc)
{
    const double sc = exp_scale(1.0, 0, 1, -1, eG, eY);
    const int64_t tot = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % m), j = (int)(t / m);
        stg(dC + (int64_t)j * lddc + i, sc * ldg(G + (int64_t)j * ldg_ + i));
    }
}

// -sy with 2^sy >= max|Y| as an int64 (the norm pass-0 exponent of Y)
__global__ void k_neg_exp(const int32_t *s, int64_t *out, const int32_t *skip)
{
    if (skip && *skip) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = -(int64_t)(*s == 0x7FFFFFFF ? 0 : *s);
}

// ---------------------------------------------------------------------------------------------
// Refinement step of the precision form: with 2^sy > max|Y| (sy = -*negsy), 2^sD > max|D| and
//   x = max(0, max(sy - eD, sy + sD) + 1 - (1022 - 9)),
// Y <- 2^-(eD + x) Y + 2^(sy - x) D,  e <- e + eD + x,  status <- max(status, correction status),
// scale <- 2^-e.  Since A Y + Y B = 2^-e C - 2^sy R' and A D + D B = 2^-eD R', the new pair
// satisfies A Y + Y B = 2^-(e + eD + x) C; x keeps every entry below 2^(1022-9), so tiles of up to
// 512 columns keep their infinity norms below OMEGA.
// ---------------------------------------------------------------------------------------------
__global__ void k_refine_update(double *Y, int64_t ldy, const double *D, int64_t ldd, int m, int n,
                                const int64_t *eD, const int64_t *negsy, const int32_t *sD, int64_t *e,
                                int32_t *info, const int32_t *infoD, double *scale, const int32_t *skip,
                                uint32_t *sweeps)
{
    if (skip && __builtin_amdgcn_readfirstlane(*(volatile const int32_t *)skip) != 0) return;
    const int64_t sy = -*negsy;
    const int64_t sd = *sD == 0x7FFFFFFF ? 0 : *sD;
    int64_t top = sy - *eD;
    if (sy + sd > top) top = sy + sd;
    int64_t x = top + 1 - (1022 - 9);
    if (x < 0) x = 0;
    int64_t ay = *eD + x, ad = x - sy;
    if (ay > 2100) ay = 2100;
    if (ad > 2100) ad = 2100;
    if (ad < -2100) ad = -2100;
    const int64_t tot = (int64_t)m * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % m), j = (int)(t / m);
        double *p = Y + (int64_t)j * ldy + i;
        stg(p, ldexp(ldg(p), -(int)ay) + ldexp(ldg(D + (int64_t)j * ldd + i), -(int)ad));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t en = *e + *eD + x;
        *e = en;
        if (*infoD > *info) *info = *infoD;
        if (scale) *scale = en > 1074 ? 0.0 : ldexp(1.0, -(int)en);
        if (sweeps) *sweeps += 1u;
    }
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
static int grid_for(int64_t work, int per = 256)
{
    int64_t g = (work + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

hipError_t launch_quasi_copy(const double *T, int64_t ldt, int n, bool flip, double sign, double *D,
                             hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_quasi_copy, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, T, ldt, n,
                       flip ? 1 : 0, sign, D);
    return hipGetLastError();
}

hipError_t launch_flip_transpose(const double *A, int64_t lda, int n, double *Ah, hipStream_t s)
{
    return launch_quasi_copy(A, lda, n, true, 1.0, Ah, s);
}

hipError_t launch_flip_axes(double *W, int64_t ldw, int m, int n, bool rows, bool cols, hipStream_t s)
{
    if (m <= 0 || n <= 0 || (!rows && !cols)) return hipSuccess;
    hipLaunchKernelGGL(k_flip_axes, dim3(grid_for((int64_t)m * n / 2 + 1)), dim3(256), 0, s, W, ldw, m,
                       n, rows ? 1 : 0, cols ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_flip(double *W, int64_t ldw, int m, int n, hipStream_t s)
{
    return launch_flip_axes(W, ldw, m, n, true, true, s);
}

hipError_t launch_norm_shift(const int32_t *s, const double *t, int64_t *negshift, int64_t *total,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_norm_shift, dim3(1), dim3(64), 0, st, s, t, negshift, total);
    return hipGetLastError();
}

hipError_t launch_add_exponent(int64_t *e, double *scale, const int64_t *add, hipStream_t st)
{
    hipLaunchKernelGGL(k_add_exponent, dim3(1), dim3(64), 0, st, e, scale, add);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmDesc &g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.M + kGT - 1) / kGT, (g.N + kGT - 1) / kGT);
    hipLaunchKernelGGL(k_gemm, grid, dim3(512), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_scale_copy(const double *G, int64_t ldg_, int m, int n, const int64_t *eG,
                             const int64_t *eY, double *dC, int64_t lddc, hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for((int64_t)m * n)), dim3(256), 0, s, G, ldg_, m, n, eG,
                       eY, dC, lddc);
    return hipGetLastError();
}

// 2^s sqrt(*t) = ||X||_F (pattern 1: quasi-triangular part).  part: kNormParts doubles.
hipError_t launch_norm(const double *X, int64_t ld, int rows, int cols, int pattern, double *part,
                       int32_t *s, double *t, hipStream_t st, const int32_t *skip)
{
    const int nb = kNormParts;
    hipLaunchKernelGGL(k_norm_part, dim3(nb), dim3(512), 0, st, X, ld, rows, cols, pattern, 0, s, part, skip);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, part, nb, 0, s, t, skip);
    hipLaunchKernelGGL(k_norm_part, dim3(nb), dim3(512), 0, st, X, ld, rows, cols, pattern, 1, s, part, skip);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, part, nb, 1, s, t, skip);
    return hipGetLastError();
}

hipError_t launch_neg_exp(const int32_t *s, int64_t *out, hipStream_t st, const int32_t *skip)
{
    hipLaunchKernelGGL(k_neg_exp, dim3(1), dim3(64), 0, st, s, out, skip);
    return hipGetLastError();
}

hipError_t launch_refine_check(const int32_t *s5, const double *t5, const int64_t *e, double tol, int32_t *skip,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_refine_check, dim3(1), dim3(64), 0, st, s5, t5, e, tol, skip);
    return hipGetLastError();
}

hipError_t launch_residual_final(const int32_t *s5, const double *t5, const int64_t *e, double *out,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(64), 0, st, s5, t5, e, out);
    return hipGetLastError();
}

hipError_t launch_refine_update(double *Y, int64_t ldy, const double *D, int64_t ldd, int m, int n,
                                const int64_t *eD, const int64_t *negsy, const int32_t *sD, int64_t *e,
                                int32_t *info, const int32_t *infoD, double *scale, hipStream_t st,
                                const int32_t *skip, uint32_t *sweeps)
{
    hipLaunchKernelGGL(k_refine_update, dim3(grid_for((int64_t)m * n)), dim3(256), 0, st, Y, ldy, D, ldd,
                       m, n, eD, negsy, sD, e, info, infoD, scale, skip, sweeps);
    return hipGetLastError();
}

// 2^s > max |X| (s = 0 for a zero matrix, INT32_MAX if non-finite).  part: kNormParts doubles.
hipError_t launch_absmax_exp(const double *X, int64_t ld, int rows, int cols, double *part, int32_t *s,
                             hipStream_t st, const int32_t *skip)
{
    hipLaunchKernelGGL(k_norm_part, dim3(kNormParts), dim3(512), 0, st, X, ld, rows, cols, 0, 0, s, part, skip);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, part, kNormParts, 0, s, (double *)nullptr, skip);
    return hipGetLastError();
}

}  // namespace trsyl
