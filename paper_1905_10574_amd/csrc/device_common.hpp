// Device-side building blocks shared by the solver kernels (gfx950 / CDNA4).
//
//  * Robust scalar primitives ProtectUpdate / ProtectDivision (Sec. 2.1), power-of-two versions
//    written from their contracts, with exponents carried as integers.
//  * The robust small Sylvester solve for 1x1 / 2x2 diagonal blocks (Sec. 2.1): Gaussian
//    elimination with complete pivoting on the <= 4x4 Kronecker system.
//  * Wave-level FP64 MFMA helpers (v_mfma_f64_16x16x4_f64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trsyl {

constexpr double kOmega = 0x1p1022;   // overflow threshold: two factors of two below DBL_MAX
constexpr int kWave = 64;

enum Status : int32_t {
    kOk = 0,
    kPerturbed = 1,
    kBadStructure = 2,
    kBadInput = 3,
    kWatchdog = 4,
};

__device__ __forceinline__ double col(const double *M, int64_t ld, int64_t i, int64_t j)
{
    return M[j * ld + i];
}

// A value every thread of the workgroup holds (typically read back from LDS after a barrier),
// made visibly uniform to the compiler.  Any branch or loop bound that encloses a workgroup
// barrier must be decided by such a value: otherwise the compiler lays the region out as
// divergent control flow, and waves can reach the barriers a different number of times.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// The lane index, opaque to the compiler: what is derived from it is computed where it is used
// instead of being hoisted out of the enclosing loops, where it would hold registers (and spill)
// for the whole loop.
__device__ __forceinline__ int lane_here()
{
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}

// --------------------------------------------------------------------------------------------
// ProtectUpdate(c, a, y) (Sec. 2.1): for 0 <= c, a, y <= OMEGA, an s >= 0 with
//     2^-s (c + a y) <= OMEGA.
// a*y is evaluated as (ma*my) 2^(ea+ey) with mantissas in [1,2); the scaled sum is pushed up by
// 2^-50 to cover its roundings, so the contract holds exactly and s exceeds the minimum by at
// most one, and only when c + a*y lies within that margin of a power-of-two threshold.
// --------------------------------------------------------------------------------------------
__device__ __forceinline__ int protect_update(double c, double a, double y)
{
    if (a == 0.0 || y == 0.0) return 0;            // c <= OMEGA by precondition
    const int ea = ilogb(a), ey = ilogb(y);
    const double mprod = ldexp(a, -ea) * ldexp(y, -ey);   // [1, 4)
    int E = ea + ey;
    if (c != 0.0) {
        const int ec = ilogb(c);
        if (ec > E) E = ec;
    }
    double g = ldexp(c, -E) + ldexp(mprod, ea + ey - E);  // (c + a y) 2^-E, in [1, 6)
    g *= 1.0 + 0x1p-50;
    int cl = ilogb(g);                              // g in [2^cl, 2^(cl+1))
    if (g != ldexp(1.0, cl)) cl += 1;               // ceil(log2 g)
    const int s = cl + E - 1022;
    return s > 0 ? s : 0;
}

// ProtectDivision(b, t) (Sec. 2.1): the smallest s >= 0 with 2^-s |b| <= |t| OMEGA, for
// |b| <= OMEGA and t != 0, so that (2^-s b) / t cannot exceed OMEGA.
__device__ __forceinline__ int protect_division(double b, double t)
{
    const double ab = fabs(b), at = fabs(t);
    if (ab == 0.0 || at >= 1.0) return 0;
    const int eb = ilogb(ab), et = ilogb(at);
    const double mb = ldexp(ab, -eb), mt = ldexp(at, -et);   // [1, 2)
    const int s = eb - et - 1022 + (mb > mt ? 1 : 0);
    return s > 0 ? s : 0;
}

// --------------------------------------------------------------------------------------------
// Robust small Sylvester solve  A11 Z + Z B11 = beta R,  A11 r x r, B11 c x c, r, c in {1, 2}
// (Sec. 2.1).  vec(Z) solves K vec(Z) = beta vec(R) with K = I_c (x) A11 + B11^T (x) I_r.  The
// system is embedded in a 4x4 one (unused unknowns decoupled by identity rows, zero right-hand
// side), then eliminated with complete pivoting; every right-hand-side update is guarded by
// ProtectUpdate and every division by ProtectDivision, each guard rescaling the whole vector.
// a[4] = A11 column-major (a11, a21, a12, a22), b[4] likewise, z[4] = R column-major on entry
// (z11, z21, z12, z22), Z on exit.  Returns the total exponent s (beta = 2^-s); sets *pert when
// a pivot was raised to smin.  On exit ||Z||_inf <= OMEGA.
// --------------------------------------------------------------------------------------------
__device__ inline int small_solve(int r, int c, const double a[4], const double b[4], double z[4],
                                  double smin, int *pert)
{
    if (r == 1 && c == 1) {
        double d = a[0] + b[0];
        if (fabs(d) < smin) { d = (d < 0.0) ? -smin : smin; *pert = 1; }
        const int s = protect_division(z[0], d);
        z[0] = ldexp(z[0], -s) / d;
        return s;
    }
    // unknown u <-> Z(p, q) with u = q*r + p; equation e <-> entry (p, q) likewise.  All
    // register arrays are indexed with compile-time indices (runtime r, c enter through selects).
    double K[4][4], v[4];
    int perm[4] = {0, 1, 2, 3};
    const int nn = r * c;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = (r == 2) ? (e & 1) : 0, q = (r == 2) ? (e >> 1) : e;
        const bool live = e < nn;
        double zv = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) zv = (t == q * 2 + p) ? z[t] : zv;
        v[e] = live ? zv : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int pp = (r == 2) ? (u & 1) : 0, qq = (r == 2) ? (u >> 1) : u;
            double x = 0.0;
            if (live && u < nn) {
                double av = 0.0, bv = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    av = (t == pp * 2 + p) ? a[t] : av;     // A(p, pp)
                    bv = (t == q * 2 + qq) ? b[t] : bv;     // B(qq, q)
                }
                if (qq == q) x += av;
                if (pp == p) x += bv;
            } else if (!live && u == e) {
                x = 1.0;
            }
            K[e][u] = x;
        }
    }
    double kmax = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) kmax = fmax(kmax, fabs(K[i][j]));
    if (kmax > 0x1p1019) {                          // growth <= 2^3 keeps entries <= OMEGA
        const int sh = ilogb(kmax) + 1 - 1019;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = ldexp(v[i], -sh);
#pragma unroll
            for (int j = 0; j < 4; ++j) K[i][j] = ldexp(K[i][j], -sh);
        }
    }
    int stot = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int pi = t, pj = t;
        double best = -1.0;
#pragma unroll
        for (int i = t; i < 4; ++i)
#pragma unroll
            for (int j = t; j < 4; ++j)
                if (fabs(K[i][j]) > best) { best = fabs(K[i][j]); pi = i; pj = j; }
        // row swap t <-> pi, column swap t <-> pj (unknown order tracked in perm)
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
        if (fabs(K[t][t]) < smin) { K[t][t] = (K[t][t] < 0.0) ? -smin : smin; *pert = 1; }
#pragma unroll
        for (int i = t + 1; i < 4; ++i) {
            const double l = K[i][t] / K[t][t];    // |l| <= 1 by complete pivoting
#pragma unroll
            for (int j = t + 1; j < 4; ++j) K[i][j] = fma(-l, K[t][j], K[i][j]);
            K[i][t] = 0.0;
            const int s = protect_update(fabs(v[i]), fabs(l), fabs(v[t]));
            if (s) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = ldexp(v[q], -s);
                stot += s;
            }
            v[i] = fma(-l, v[t], v[i]);
        }
    }
#pragma unroll
    for (int i = 3; i >= 0; --i) {
#pragma unroll
        for (int j = i + 1; j < 4; ++j) {
            const int s = protect_update(fabs(v[i]), fabs(K[i][j]), fabs(v[j]));
            if (s) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = ldexp(v[q], -s);
                stot += s;
            }
            v[i] = fma(-K[i][j], v[j], v[i]);
        }
        const int s = protect_division(v[i], K[i][i]);
        if (s) {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = ldexp(v[q], -s);
            stot += s;
        }
        v[i] = v[i] / K[i][i];
    }
    double u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int x = 0; x < 4; ++x) if (perm[t] == x) u[x] = v[t];
    }
    // back to (p, q) positions; a row of two entries <= OMEGA each may sum to 2 OMEGA
    double zo[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int p = t & 1, q = t >> 1;
        double x = 0.0;
        if (p < r && q < c) {
#pragma unroll
            for (int uu = 0; uu < 4; ++uu) x = (uu == q * r + p) ? u[uu] : x;
        }
        zo[t] = x;
    }
    const double rowmax = fmax(fabs(zo[0]) + fabs(zo[2]), fabs(zo[1]) + fabs(zo[3]));
    const int extra = (rowmax > kOmega) ? 1 : 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) z[t] = ldexp(zo[t], -extra);
    return stot + extra;
}

// --------------------------------------------------------------------------------------------
// Non-negative doubles order like their bit patterns: atomic max through uint64.
// --------------------------------------------------------------------------------------------
__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v)
{
    atomicMax(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ __forceinline__ void set_status(int32_t *status, int32_t code)
{
    // larger codes win (2, 3, 4 are errors; 1 is a warning)
    atomicMax(status, code);
}

// --------------------------------------------------------------------------------------------
// FP64 MFMA 16x16x4 (gfx950).  Operand / result layout per lane l (measured):
//   a operand: A'(row = l & 15, k = l >> 4); b operand: B'(k = l >> 4, col = l & 15);
//   result element i: D'(row = (l >> 4) + 4 i, col = l & 15).
// The solver computes D^T: A' = Bop^T, B' = Aop^T, so result element i of lane l is
//   D(m = l & 15, n = (l >> 4) + 4 i)
// and the fast (lane) index runs down the column of the column-major output.
// Within a chunk of 16 k values, MFMA step j uses k = 4 (l >> 4) + j for the lane's quad, so
// each lane reads 4 consecutive k of a column of Bop.
// --------------------------------------------------------------------------------------------
// Global-memory access helpers.  The solver's pointers come from the plan, so the compiler
// cannot infer their address space and would emit flat accesses (which also count against the
// LDS counter and force full waits); ldg / stg cast to the global address space.
//
// Data that workgroups of one launch hand to each other (tiles of Y, per-tile norms and
// exponents) goes through DevView: raw buffer loads and stores whose cache policy asks for device
// scope (sc1).  Such loads bypass the XCD-private caches' possibly stale copies and such stores
// write through, so a producer's stores are visible to any consumer once they have completed
// (s_waitcnt) and the consumer has observed the producer's counter.  No cache-wide invalidation or
// write-back is needed, so read-only operands (A, B) stay cached.  These are plain (non-atomic)
// memory operations, so the compiler keeps many in flight; relaxed atomic loads would each be
// preceded by a full wait.  A view covers `bytes` bytes from a wave-uniform base (offsets are
// 32-bit); accesses past the end read zero and are dropped, by the buffer range check.
#ifndef TRSYL_AS_GLOBAL
#define TRSYL_AS_GLOBAL __attribute__((address_space(1)))
#endif
typedef TRSYL_AS_GLOBAL double gdouble;

__device__ __forceinline__ double ldg(const double *p) { return *(const gdouble *)p; }
__device__ __forceinline__ void stg(double *p, double v) { *(gdouble *)p = v; }

constexpr int kPolicyDevice = 16;        // cache policy bits: sc1 (device scope)
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer descriptor word 3 for gfx9-family parts

struct DevView {
    __amdgpu_buffer_rsrc_t r;
};
// The descriptor must live in scalar registers; its fields are read with readfirstlane so that
// the compiler sees them as uniform (a view's base and size are the same in every lane).
__device__ __forceinline__ DevView dev_view(const void *base, uint64_t bytes)
{
    const uint64_t b = (uint64_t)(uintptr_t)base;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    void *ub = (void *)(uintptr_t)(((uint64_t)hi << 32) | lo);
    const uint32_t nb = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)(bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes));
    return DevView{__builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)nb, kRsrcWord3)};
}
// View of a column-major rows x cols block with leading dimension ld.
__device__ __forceinline__ DevView dev_view(const double *base, int64_t ld, int rows, int cols)
{
    const int64_t n = rows > 0 && cols > 0 ? (int64_t)(cols - 1) * ld + rows : 1;
    return dev_view((const void *)base, (uint64_t)n * 8u);
}
__device__ __forceinline__ double ld_dev(const DevView &v, int64_t idx)
{
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(v.r, (int)(uint32_t)(idx * 8), 0, kPolicyDevice);
    double d;
    __builtin_memcpy(&d, &x, 8);
    return d;
}
__device__ __forceinline__ void st_dev(const DevView &v, int64_t idx, double d)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    u32x2 x;
    __builtin_memcpy(&x, &d, 8);
    __builtin_amdgcn_raw_buffer_store_b64(x, v.r, (int)(uint32_t)(idx * 8), 0, kPolicyDevice);
}
__device__ __forceinline__ int32_t ld_dev_i32(const DevView &v, int64_t idx)
{
    return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(v.r, (int)(uint32_t)(idx * 4), 0, kPolicyDevice);
}
__device__ __forceinline__ void st_dev_i32(const DevView &v, int64_t idx, int32_t x)
{
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)x, v.r, (int)(uint32_t)(idx * 4), 0, kPolicyDevice);
}

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 zero4() { return (d4){0.0, 0.0, 0.0, 0.0}; }

}  // namespace trsyl
