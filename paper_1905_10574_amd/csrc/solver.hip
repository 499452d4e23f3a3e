// Kernels of the robust tiled triangular Sylvester solver (Algorithm 4, Sec. 2.2) for gfx950.
//
//   k_structure      tile boundaries (2x2 blocks never split) and structure check
//   k_bounds_A/B/C   Bound tasks: ||A_ik||_inf, ||B_lj||_inf, ||C_kl||_inf, input checks
//   k_dag            persistent scheduler: each workgroup takes the next task of a static,
//                    topologically ordered list and waits for its dependencies
//   k_front_*        alternative scheduler: one launch per anti-diagonal front
//   k_finalize       alpha = min alpha_kl (max exponent), status
//   k_consistency    consistency scaling Y_kl <- (alpha / alpha_kl) Y_kl
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "launch.hpp"
#include "plan.hpp"
#include "solver_solve.hpp"
#include "solver_update.hpp"

namespace trsyl {

// ---------------------------------------------------------------------------------------------
// Structure and tiling
// ---------------------------------------------------------------------------------------------
__device__ void structure_body(const Plan &P, int64_t blk, int64_t nblk)
{
    if (plan_skipped(P)) return;
    const int64_t tid = blk * blockDim.x + threadIdx.x;
    const int64_t nthr = nblk * blockDim.x;
    for (int64_t i = tid; i + 2 < P.m; i += nthr)
        if (P.A[i * P.lda + i + 1] != 0.0 && P.A[(i + 1) * P.lda + i + 2] != 0.0)
            set_status(P.status, kBadStructure);
    for (int64_t i = tid; i + 2 < P.n; i += nthr)
        if (P.B[i * P.ldb + i + 1] != 0.0 && P.B[(i + 1) * P.ldb + i + 2] != 0.0)
            set_status(P.status, kBadStructure);
    for (int64_t k = tid; k <= P.pt; k += nthr) {
        int64_t v;
        if (k == 0) v = 0;
        else if (k == P.pt) v = P.m;
        else {
            const int64_t b = k * P.tm;
            v = (P.A[(b - 1) * P.lda + b] != 0.0) ? b + 1 : b;
            if (v > P.m) v = P.m;
        }
        P.rowoff[k] = (int32_t)v;
    }
    for (int64_t k = tid; k <= P.qt; k += nthr) {
        int64_t v;
        if (k == 0) v = 0;
        else if (k == P.qt) v = P.n;
        else {
            const int64_t b = k * P.tn;
            v = (P.B[(b - 1) * P.ldb + b] != 0.0) ? b + 1 : b;
            if (v > P.n) v = P.n;
        }
        P.coloff[k] = (int32_t)v;
    }
}
__global__ void k_structure(Plan P) { structure_body(P, blockIdx.x, gridDim.x); }

// ||T_ik||_inf for a tile pair of the quasi-triangular matrix T (A or B); the diagonal tile also
// feeds the global max |entry| and, for B, the 1-norm.  Entries below the first subdiagonal are
// never read.  Non-finite or > OMEGA entries raise status 3, and so does a tile norm above OMEGA
// (Algorithm 4 requires every tile of A, B and C to have infinity norm at most OMEGA; entries at
// most OMEGA do not imply it).
__device__ void bound_tile(const Plan &P, const double *T, int64_t ld, const int32_t *off, int nt,
                           int i, int k, double *out, double *out1)
{
    __shared__ double red[kWaves];
    const int r0 = off[i], r1 = off[i + 1], c0 = off[k], c1 = off[k + 1];
    double best = 0.0, mx = 0.0;
    int bad = 0;
    for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
        double s = 0.0;
        const int cstart = (i == k) ? (r - 1 > c0 ? r - 1 : c0) : c0;
        for (int c = cstart; c < c1; ++c) {
            const double x = T[(int64_t)c * ld + r];
            if (!(fabs(x) <= kOmega)) bad = 1;
            s += fabs(x);
            mx = fmax(mx, fabs(x));
        }
        best = fmax(best, s);
    }
    if (bad) set_status(P.status, kBadInput);
    best = wg_max(best, red);
    if (threadIdx.x == 0 && !(best <= kOmega)) set_status(P.status, kBadInput);
    if (i == k) {
        mx = wg_max(mx, red);
        if (threadIdx.x == 0) atomic_max_nonneg(P.gmax, mx);
        if (out1) {   // 1-norm: max column sum over the quasi-triangular part
            double cb = 0.0;
            for (int c = c0 + threadIdx.x; c < c1; c += kThreads) {
                double s = 0.0;
                const int rend = (c + 2 < r1) ? c + 2 : r1;
                for (int r = r0; r < rend; ++r) s += fabs(T[(int64_t)c * ld + r]);
                cb = fmax(cb, s);
            }
            cb = wg_max(cb, red);
            if (threadIdx.x == 0) out1[k] = cb;
        }
    }
    if (threadIdx.x == 0) out[(size_t)i * nt + k] = best;
}

__device__ void bounds_A_body(const Plan &P, int b)
{
    if (plan_skipped(P)) return;
    const int i = b / P.pt, k = b % P.pt;
    if (i > k) return;
    bound_tile(P, P.A, P.lda, P.rowoff, P.pt, i, k, P.anorm, nullptr);
}
__device__ void bounds_B_body(const Plan &P, int b)
{
    if (plan_skipped(P)) return;
    const int l = b / P.qt, j = b % P.qt;
    if (l > j) return;
    bound_tile(P, P.B, P.ldb, P.coloff, P.qt, l, j, P.bnorm, P.bdiag1);
}
__global__ void __launch_bounds__(kThreads) k_bounds_A(Plan P) { bounds_A_body(P, blockIdx.x); }
__global__ void __launch_bounds__(kThreads) k_bounds_B(Plan P) { bounds_B_body(P, blockIdx.x); }

// ||C_kl||_inf, input checks (entries and the tile norm), and version 0 of every tile's state.
__device__ void bounds_C_body(const Plan &P, int T)
{
    if (plan_skipped(P)) return;
    __shared__ double red[kWaves];
    const int k = T / P.qt, l = T % P.qt;
    const int r0 = P.rowoff[k], r1 = P.rowoff[k + 1], c0 = P.coloff[l], c1 = P.coloff[l + 1];
    double best = 0.0;
    int bad = 0;
    for (int r = r0 + threadIdx.x; r < r1; r += kThreads) {
        double s = 0.0;
        for (int c = c0; c < c1; ++c) {
            const double x = P.C[(int64_t)c * P.ldc + r];
            if (!(fabs(x) <= kOmega)) bad = 1;
            s += fabs(x);
        }
        best = fmax(best, s);
    }
    if (bad) set_status(P.status, kBadInput);
    best = wg_max(best, red);
    if (threadIdx.x == 0) {
        if (!(best <= kOmega)) set_status(P.status, kBadInput);   // Algorithm 4's data requirement
        tile_norm_store(P, T, 0, 0, best);
        for (int s = 1; s < P.slabs; ++s) tile_norm_store(P, T, 0, s, 0.0);
        tile_exp_store(P, T, 0, 0);
        P.ver[T] = 0;
    }
}
__global__ void __launch_bounds__(kThreads) k_bounds_C(Plan P) { bounds_C_body(P, blockIdx.x); }

// ---------------------------------------------------------------------------------------------
// Persistent scheduler
// ---------------------------------------------------------------------------------------------
union TaskLds {
    UpdateLds upd;
    SolveLds sol;
};

__device__ __forceinline__ bool wait_count(const Plan &P, const uint32_t *ctr, uint32_t need,
                                           uint64_t t0)
{
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (wall_clock64() - t0 > P.spin_limit) return false;
        __builtin_amdgcn_s_sleep(20);   // ~0.5 us between polls keeps the counters' channels free
    }
    return true;
}

// Dependency waits of a task, spread over the threads: for a solve, thread 0 waits for every
// update of the tile; for an update, thread 0 waits for the source's solve and the target's
// previous version; for a multi-term update of g terms, thread t < g waits for the solve of term
// t's source and thread 0 also for the target's version u0.  Returns false on a watchdog timeout
// (the status is set).
__device__ __forceinline__ bool task_wait(const Plan &P, uint64_t task, int kind, int T, uint32_t slabs)
{
    const uint64_t t0 = wall_clock64();
    bool ok = true;
    if (kind == kTaskGroupUpdate) {
        const int g = task_S(task), u0 = task_u(task);
        if ((int)threadIdx.x < g) {
            int ks, ls;
            update_source(P.pt, T / P.qt, T % P.qt, u0 + (int)threadIdx.x, &ks, &ls);
            const int S = ks * P.qt + ls;
            ok = wait_count(P, &P.ver[S], (uint32_t)(tile_updates(P, S) + 1) * slabs, t0);
        }
        if (threadIdx.x == 0) ok = ok && wait_count(P, &P.ver[T], (uint32_t)u0 * slabs, t0);
    } else if (threadIdx.x == 0) {
        if (kind == kTaskSolve) {
            ok = wait_count(P, &P.ver[T], (uint32_t)tile_updates(P, T) * slabs, t0);
        } else {
            const int S = task_S(task), u = task_u(task);
            ok = wait_count(P, &P.ver[S], (uint32_t)(tile_updates(P, S) + 1) * slabs, t0) &&
                 wait_count(P, &P.ver[T], (uint32_t)u * slabs, t0);
        }
    }
    // on a timeout the task is skipped, but its counter still moves so that every other
    // workgroup drains as well; the status reports the failure
    if (!ok) set_status(P.status, kWatchdog);
    return ok;
}

// What a finished task adds to its target's counter (completed modifications x slabs).
__device__ __forceinline__ uint32_t task_increment(uint64_t task, int kind, uint32_t slabs)
{
    return kind == kTaskSolve ? slabs : (kind == kTaskGroupUpdate ? (uint32_t)task_S(task) * slabs : 1u);
}

// The persistent loop has one latch and no divergent exits: every value that decides a branch
// around a barrier is read back from LDS and made uniform, thread-0-only blocks are fenced by
// barriers on both sides, and the back-edge follows a barrier.
__global__ void __launch_bounds__(kThreads) k_dag(Plan Pk)
{
    const Plan P = uniform_plan(Pk);
    __shared__ TaskLds L;
    __shared__ uint32_t s_ticket;
    __shared__ int s_ok;
    if (plan_skipped(P) || uniform(*(volatile int32_t *)P.status) >= kBadStructure) return;
    double *scratch = P.scratch + (size_t)blockIdx.x * kMaxTile * kMaxTile;
    const uint32_t slabs = (uint32_t)P.slabs;
    const uint32_t ntasks = (uint32_t)P.ntasks;
    for (;;) {
        if (threadIdx.x == 0) {
            s_ticket = atomicAdd(P.ticket, 1u);
            s_ok = 1;
        }
        __syncthreads();
        const uint32_t t = uniform(s_ticket);
        if (t >= ntasks) break;
        const uint64_t task = P.tasks[t];
        const int kind = uniform(task_kind(task)), T = uniform(task_T(task));
        if (!task_wait(P, task, kind, T, slabs)) s_ok = 0;
        __syncthreads();
        const uint64_t tstart = wall_clock64();
        if (uniform(s_ok)) {
            if (kind == kTaskSolve) run_solve(P, T, scratch, L.sol);
            else {
#ifdef TRSYL_PHASE_STAMPS
                uint64_t *us = P.trace ? P.trace + 4 * (size_t)max_tasks(P) + 80 * (size_t)P.pt * P.qt + 8 * (size_t)t : nullptr;
#else
                uint64_t *us = nullptr;
#endif
                if (kind == kTaskGroupUpdate) run_update_group(P, T, task_u(task), task_S(task), L.upd, us);
                else run_update(P, kind, T, task_S(task), task_u(task), task_slab(task), L.upd, us);
            }
        }
        if (P.trace && threadIdx.x == 0) {
            uint64_t *rec = P.trace + 4 * (size_t)t;
            rec[0] = task;
            rec[1] = tstart;
            rec[2] = wall_clock64();
            rec[3] = blockIdx.x;
        }
        // every device-scope store of the task has completed before the counter moves
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&P.ver[T], task_increment(task, kind, slabs), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Front scheduler: stream order supplies the dependencies.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_front_solve(Plan Pk, int d)
{
    const Plan P = uniform_plan(Pk);
    __shared__ SolveLds L;
    if (plan_skipped(P) || uniform(*(volatile int32_t *)P.status) >= kBadStructure) return;
    const int lmin = d - (P.pt - 1) > 0 ? d - (P.pt - 1) : 0;
    const int l = lmin + blockIdx.x;
    const int k = P.pt - 1 - (d - l);
    if (l >= P.qt || k < 0) return;
    const int T = k * P.qt + l;
    run_solve(P, T, P.scratch + (size_t)blockIdx.x * kMaxTile * kMaxTile, L);
    if (threadIdx.x == 0) P.ver[T] += P.slabs;
}

// blockIdx.x = (source index on the front) * (targets per source) * slabs
__global__ void __launch_bounds__(kThreads) k_front_update(Plan Pk, int d, int kind)
{
    const Plan P = uniform_plan(Pk);
    __shared__ UpdateLds L;
    if (plan_skipped(P) || uniform(*(volatile int32_t *)P.status) >= kBadStructure) return;
    const int lmin = d - (P.pt - 1) > 0 ? d - (P.pt - 1) : 0;
    const int ntgt = (kind == kTaskColUpdate) ? P.pt - 1 : P.qt - 1;
    const int slab = blockIdx.x % P.slabs;
    const int rest = blockIdx.x / P.slabs;
    const int tgt = rest % ntgt;
    const int src = rest / ntgt;
    const int ls = lmin + src;
    const int ks = P.pt - 1 - (d - ls);
    if (ls >= P.qt || ks < 0) return;
    int ti, tl;
    if (kind == kTaskColUpdate) {
        ti = tgt; tl = ls;
        if (ti >= ks) return;
    } else {
        ti = ks; tl = tgt + 1;
        if (tl <= ls) return;
    }
    const int T = ti * P.qt + tl, S = ks * P.qt + ls;
    const int u = update_index(P.pt, ti, tl, ks, ls);
    run_update(P, kind, T, S, u, slab, L, nullptr);
}

// One workgroup per tile T: the updates of T whose sources lie on front d -- the column source
// (k, l) and the row source (i, j) on that front -- as one two-term update when both exist (the
// grouping of the persistent scheduler's task list), else as a single update.
__global__ void __launch_bounds__(kThreads) k_front_group(Plan Pk, int d)
{
    const Plan P = uniform_plan(Pk);
    __shared__ UpdateLds L;
    if (plan_skipped(P) || uniform(*(volatile int32_t *)P.status) >= kBadStructure) return;
    const int T = blockIdx.x, i = T / P.qt, l = T % P.qt;
    const int ks = P.pt - 1 - (d - l), ls = d - (P.pt - 1 - i);
    const bool col = d - l >= 0 && ks > i, row = ls >= 0 && ls < l;
    if (col && row) run_update_group(P, T, update_index(P.pt, i, l, ks, l), 2, L, nullptr);
    else if (col) run_update(P, kTaskColUpdate, T, ks * P.qt + l, update_index(P.pt, i, l, ks, l), 0, L, nullptr);
    else if (row) run_update(P, kTaskRowUpdate, T, i * P.qt + ls, update_index(P.pt, i, l, i, ls), 0, L, nullptr);
}

// ---------------------------------------------------------------------------------------------
// alpha = min alpha_kl, i.e. e = max e_kl; then consistency scaling.
// ---------------------------------------------------------------------------------------------
__device__ void finalize_body(const Plan &P)
{
    if (plan_skipped(P)) return;
    __shared__ int red[kWaves];
    int e = 0;
    for (int T = threadIdx.x; T < P.pt * P.qt; T += kThreads)
        e = max(e, tile_exp_at(P, T, tile_updates(P, T) + 1));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e = max(e, __shfl_xor(e, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int i = 0; i < kWaves; ++i) r = max(r, red[i]);
        const int st = *P.status;
        if (st >= kBadStructure) r = 0;
        *P.e_out = r;
        if (P.scale_out) *P.scale_out = (r > 1074) ? 0.0 : ldexp(1.0, -r);
        *P.info_out = st;
    }
}
__global__ void __launch_bounds__(kThreads) k_finalize(Plan P) { finalize_body(P); }

__device__ void consistency_body(const Plan &P, int per_tile, int b)
{
    if (plan_skipped(P)) return;
    const int T = b / per_tile, part = b % per_tile;
    const int st = *(volatile int32_t *)P.status;
    if (st >= kBadStructure) return;
    const int eT = tile_exp_at(P, T, tile_updates(P, T) + 1);
    const int64_t e = *P.e_out;
    if (eT == e) return;
    const int k = T / P.qt, l = T % P.qt;
    const int r0 = P.rowoff[k], mr = P.rowoff[k + 1] - r0;
    const int c0 = P.coloff[l], nc = P.coloff[l + 1] - c0;
    const int64_t sh = e - eT;
    const int shi = sh > 4000 ? 4000 : (int)sh;     // beyond 2100 everything is zero anyway
    for (int t = part * kThreads + threadIdx.x; t < mr * nc; t += per_tile * kThreads) {
        const int rr = t % mr, cc = t / mr;
        double *p = P.C + (int64_t)(c0 + cc) * P.ldc + r0 + rr;
        *p = ldexp(*p, -shi);
    }
}
__global__ void __launch_bounds__(kThreads) k_consistency(Plan P, int per_tile)
{
    consistency_body(P, per_tile, blockIdx.x);
}

// ---------------------------------------------------------------------------------------------
// Batched solve: many problems, each with its own plan (device array), in one launch per stage.
// A stage's blocks are split among the problems by the offsets off[0..count] (problem p owns
// blocks off[p] .. off[p+1]-1).  The persistent scheduler takes tickets from one merged task list
// in which every problem's tasks keep their own topological order, so the no-deadlock argument of
// the single solve carries over; a problem with a structure or input error has its tasks skipped
// (their counters still move).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int find_problem(const int32_t *off, int count, int b)
{
    int lo = 0, hi = count - 1;                    // largest p with off[p] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return uniform(lo);
}

__global__ void k_structure_b(const Plan *plans, const int32_t *off, int count)
{
    const int p = find_problem(off, count, blockIdx.x);
    const Plan P = uniform_plan(plans[p]);
    structure_body(P, blockIdx.x - uniform(off[p]), uniform(off[p + 1] - off[p]));
}

__global__ void __launch_bounds__(kThreads) k_bounds_b(const Plan *plans, const int32_t *offA,
                                                       const int32_t *offB, const int32_t *offC, int count)
{
    const int b = blockIdx.x;
    const int totA = uniform(offA[count]), totB = uniform(offB[count]);
    if (b < totA) {
        const int p = find_problem(offA, count, b);
        const Plan P = uniform_plan(plans[p]);
        bounds_A_body(P, b - uniform(offA[p]));
    } else if (b < totA + totB) {
        const int p = find_problem(offB, count, b - totA);
        const Plan P = uniform_plan(plans[p]);
        bounds_B_body(P, b - totA - uniform(offB[p]));
    } else {
        const int p = find_problem(offC, count, b - totA - totB);
        const Plan P = uniform_plan(plans[p]);
        bounds_C_body(P, b - totA - totB - uniform(offC[p]));
    }
}

__global__ void __launch_bounds__(kThreads) k_finalize_b(const Plan *plans)
{
    const Plan P = uniform_plan(plans[blockIdx.x]);
    finalize_body(P);
}

__global__ void __launch_bounds__(kThreads) k_consistency_b(const Plan *plans, const int32_t *off, int count)
{
    const int p = find_problem(off, count, blockIdx.x);
    const Plan P = uniform_plan(plans[p]);
    consistency_body(P, consistency_per_tile(P.tm, P.tn), blockIdx.x - uniform(off[p]));
}

__global__ void __launch_bounds__(kThreads) k_dag_b(const Plan *plans, const uint64_t *tasks,
                                                    const uint32_t *tprob, uint32_t ntasks,
                                                    uint32_t *ticket_, double *scratch_base)
{
    __shared__ TaskLds L;
    __shared__ uint32_t s_ticket;
    __shared__ int s_ok;
    uint32_t *ticket = uniptr(ticket_);
    double *scratch = uniptr(scratch_base) + (size_t)blockIdx.x * kMaxTile * kMaxTile;
    const uint32_t nt = uni32((int)ntasks);
    for (;;) {
        if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t t = uniform(s_ticket);
        if (t >= nt) break;
        const uint64_t task = tasks[t];
        const int p = uni32((int)tprob[t]);
        const Plan P = uniform_plan(plans[p]);
        const uint32_t slabs = (uint32_t)P.slabs;
        const int kind = uniform(task_kind(task)), T = uniform(task_T(task));
        if (threadIdx.x == 0)
            s_ok = (plan_skipped(P) || *(volatile int32_t *)P.status >= kBadStructure) ? 0 : 1;
        __syncthreads();
        if (uniform(s_ok) && !task_wait(P, task, kind, T, slabs)) s_ok = 0;
        __syncthreads();
        if (uniform(s_ok)) {
            if (kind == kTaskSolve) run_solve(P, T, scratch, L.sol);
            else if (kind == kTaskGroupUpdate) run_update_group(P, T, task_u(task), task_S(task), L.upd, nullptr);
            else run_update(P, kind, T, task_S(task), task_u(task), task_slab(task), L.upd, nullptr);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&P.ver[T], task_increment(task, kind, slabs), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Diagnostics: device primitives on argument lists.
// ---------------------------------------------------------------------------------------------
__global__ void k_debug_pu(int count, const double *in, int32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = protect_update(in[3 * i], in[3 * i + 1], in[3 * i + 2]);
}
__global__ void k_debug_pd(int count, const double *in, int32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = protect_division(in[2 * i], in[2 * i + 1]);
}

__global__ void k_fill_zero(uint32_t *p, size_t words)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------------
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    size_t g = (words + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(256), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

hipError_t launch_setup(const Plan &P, hipStream_t s)
{
    const int items = (int)((P.m > P.n ? P.m : P.n) + 2);
    int g = (items + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_structure, dim3(g), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_bounds_A, dim3(P.pt * P.pt), dim3(kThreads), 0, s, P);
    hipLaunchKernelGGL(k_bounds_B, dim3(P.qt * P.qt), dim3(kThreads), 0, s, P);
    hipLaunchKernelGGL(k_bounds_C, dim3(P.pt * P.qt), dim3(kThreads), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_dag(const Plan &P, int workers, hipStream_t s)
{
    hipLaunchKernelGGL(k_dag, dim3(workers), dim3(kThreads), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_fronts(const Plan &P, hipStream_t s)
{
    const int nf = P.pt + P.qt - 1;
    for (int d = 0; d < nf; ++d) {
        const int lmin = d - (P.pt - 1) > 0 ? d - (P.pt - 1) : 0;
        const int lmax = d < P.qt - 1 ? d : P.qt - 1;
        const int nsrc = lmax - lmin + 1;
        hipLaunchKernelGGL(k_front_solve, dim3(nsrc), dim3(kThreads), 0, s, P, d);
        if (P.slabs == 1 && (P.flags & (kFlagPairedUpdates | kFlagDeferredUpdates))) {
            if (d < nf - 1)
                hipLaunchKernelGGL(k_front_group, dim3(P.pt * P.qt), dim3(kThreads), 0, s, P, d);
            continue;
        }
        if (P.pt > 1)
            hipLaunchKernelGGL(k_front_update, dim3(nsrc * (P.pt - 1) * P.slabs), dim3(kThreads), 0, s,
                               P, d, (int)kTaskColUpdate);
        if (P.qt > 1)
            hipLaunchKernelGGL(k_front_update, dim3(nsrc * (P.qt - 1) * P.slabs), dim3(kThreads), 0, s,
                               P, d, (int)kTaskRowUpdate);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const Plan &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, P);
    if (P.pt * P.qt == 0) return hipGetLastError();
    const int gx = consistency_per_tile(P.tm, P.tn);
    hipLaunchKernelGGL(k_consistency, dim3(gx * P.pt * P.qt), dim3(kThreads), 0, s, P, gx);
    return hipGetLastError();
}

hipError_t launch_debug_protect(int which, int count, const double *in, int32_t *out, hipStream_t s)
{
    const int g = (count + 255) / 256;
    if (g == 0) return hipSuccess;
    if (which == 0) hipLaunchKernelGGL(k_debug_pu, dim3(g), dim3(256), 0, s, count, in, out);
    else hipLaunchKernelGGL(k_debug_pd, dim3(g), dim3(256), 0, s, count, in, out);
    return hipGetLastError();
}

hipError_t launch_batched(const BatchedLaunch &b, hipStream_t s)
{
    if (b.count <= 0) return hipSuccess;
    if (b.blocks_structure > 0)
        hipLaunchKernelGGL(k_structure_b, dim3(b.blocks_structure), dim3(256), 0, s, b.plans, b.off_structure, b.count);
    if (b.blocks_bounds > 0)
        hipLaunchKernelGGL(k_bounds_b, dim3(b.blocks_bounds), dim3(kThreads), 0, s, b.plans, b.off_A, b.off_B, b.off_C,
                           b.count);
    if (b.ntasks > 0)
        hipLaunchKernelGGL(k_dag_b, dim3(b.workers), dim3(kThreads), 0, s, b.plans, b.tasks, b.tprob,
                           (uint32_t)b.ntasks, b.ticket, b.scratch);
    hipLaunchKernelGGL(k_finalize_b, dim3(b.count), dim3(kThreads), 0, s, b.plans);
    if (b.blocks_consistency > 0)
        hipLaunchKernelGGL(k_consistency_b, dim3(b.blocks_consistency), dim3(kThreads), 0, s, b.plans,
                           b.off_consistency, b.count);
    return hipGetLastError();
}

}  // namespace trsyl
