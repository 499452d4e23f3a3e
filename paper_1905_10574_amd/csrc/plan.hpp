// Device-visible description of one solve: problem pointers, tiling and the per-tile state that
// the kernels share.  Built by the host (capi.cpp) inside the caller's workspace and passed to
// every kernel by value.
#pragma once
#include <stdint.h>

namespace trsyl {

constexpr int kThreads = 512;        // workgroup size of the solver kernels (8 waves)
constexpr int kWaves = kThreads / 64;
constexpr int kMaxTile = 257;        // nominal tile <= 256, +1 when a boundary dodges a 2x2 block
constexpr int kLeaf = 15;            // nominal leaf (sub-tile) size inside a tile solve; <= 16
constexpr int kMaxLeaves = 18;       // ceil(257 / 15)
constexpr int kMaxSlabRB = 5;        // 16-row blocks per update slab (64 rows + ragged edge)
constexpr int kMaxColBlocksPerWave = 3;   // 17 column blocks over 8 waves

// Plan flags
constexpr int kFlagRobustSolve = 1;   // skip the speculative tile solve
constexpr int kFlagF32Updates = 2;    // tile updates on FP32 MFMA (the precision form's solves)
constexpr int kFlagPairedUpdates = 4; // the two updates of a tile whose sources share an
                                      // anti-diagonal front as one two-term task
constexpr int kFlagDeferredUpdates = 8;   // persistent scheduler: each tile takes all its updates
                                          // in one multi-term task (left-looking), at most
                                          // kMaxGroup terms per task
constexpr int kMaxGroup = 128;        // terms of one multi-term update task

// Task encoding for the persistent scheduler (one 64-bit word):
//   bits  0..1   kind (0 = solve, 1 = column update, 2 = row update, 3 = multi-term update)
//   bits  2..7   slab
//   bits  8..27  target tile index T = i * qt + l
//   bits 28..47  source tile index S; for a multi-term update the number of terms g
//   bits 48..63  u: the update's position in the target's fixed update order (multi-term: the
//                first of the g consecutive updates u .. u + g - 1 it applies)
enum TaskKind : int { kTaskSolve = 0, kTaskColUpdate = 1, kTaskRowUpdate = 2, kTaskGroupUpdate = 3 };

__host__ __device__ inline uint64_t make_task(int kind, int slab, int T, int S, int u)
{
    return (uint64_t)kind | ((uint64_t)slab << 2) | ((uint64_t)T << 8) | ((uint64_t)S << 28) |
           ((uint64_t)u << 48);
}
__host__ __device__ inline int task_kind(uint64_t t) { return (int)(t & 3); }
__host__ __device__ inline int task_slab(uint64_t t) { return (int)((t >> 2) & 63); }
__host__ __device__ inline int task_T(uint64_t t) { return (int)((t >> 8) & 0xFFFFF); }
__host__ __device__ inline int task_S(uint64_t t) { return (int)((t >> 28) & 0xFFFFF); }
__host__ __device__ inline int task_u(uint64_t t) { return (int)((t >> 48) & 0xFFFF); }

struct Plan {
    // problem
    int64_t m, n, lda, ldb, ldc;
    const double *A;
    const double *B;
    double *C;
    // tiling (nominal tile counts; a tile may be empty when its start is pushed to the end)
    int pt, qt, tm, tn, slabs;
    int flags;
    // shared state (all inside the caller's workspace)
    int32_t *rowoff;        // [pt + 1]
    int32_t *coloff;        // [qt + 1]
    double *anorm;          // [pt * pt]  ||A_ik||_inf for i < k; [k*pt+k]: ||A_kk||_inf
    double *bnorm;          // [qt * qt]  ||B_lj||_inf for l < j; [l*qt+l]: ||B_ll||_inf
    double *bdiag1;         // [qt]       ||B_ll||_1
    double *tnorm;          // [2][pt*qt][slabs]  per-version ||Y_T||_inf partials (max over slabs)
    int32_t *texp;          // [2][pt*qt]         per-version scale exponents
    uint32_t *ver;          // [pt*qt]            completed modifications x slabs
    double *gmax;           // [1]  max |entry| of A and B (for smin)
    int32_t *status;        // [1]
    uint32_t *ticket;       // [1]
    uint32_t *stats;        // [4]  counters: 0 fallback tile solves, 1 scaled updates
    const uint64_t *tasks;  // [ntasks] (persistent scheduler)
    int ntasks;
    double *scratch;        // [workers][kMaxTile * kMaxTile] tile backups for the fallback
    // outputs
    int64_t *e_out;
    double *scale_out;
    int32_t *info_out;
    uint64_t spin_limit;    // watchdog for dependency waits
    uint64_t *trace;        // optional per-task timing records (4 words per task)
    const int32_t *skip;    // optional: when *skip != 0 every kernel of the solve returns at once
                            // (refinement sweeps after convergence)
};

// A copy of the plan whose every field is read with readfirstlane.  The plan reaches kernels and
// (non-inlined) task functions through memory the compiler cannot prove uniform, so without
// this every branch on a plan field -- and every barrier inside such a branch -- would be laid
// out as divergent control flow.
__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T> __device__ __forceinline__ T *uniptr(T *p) { return (T *)(uintptr_t)uni64((int64_t)(uintptr_t)p); }
__device__ __forceinline__ int uni32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double unid(double v) { return __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, v))); }

__device__ __forceinline__ Plan uniform_plan(const Plan &in)
{
    Plan P;
    P.m = uni64(in.m); P.n = uni64(in.n);
    P.lda = uni64(in.lda); P.ldb = uni64(in.ldb); P.ldc = uni64(in.ldc);
    P.A = uniptr(in.A); P.B = uniptr(in.B); P.C = uniptr(in.C);
    P.pt = uni32(in.pt); P.qt = uni32(in.qt); P.tm = uni32(in.tm); P.tn = uni32(in.tn);
    P.slabs = uni32(in.slabs); P.flags = uni32(in.flags);
    P.rowoff = uniptr(in.rowoff); P.coloff = uniptr(in.coloff);
    P.anorm = uniptr(in.anorm); P.bnorm = uniptr(in.bnorm); P.bdiag1 = uniptr(in.bdiag1);
    P.tnorm = uniptr(in.tnorm); P.texp = uniptr(in.texp); P.ver = uniptr(in.ver);
    P.gmax = uniptr(in.gmax); P.status = uniptr(in.status); P.ticket = uniptr(in.ticket);
    P.stats = uniptr(in.stats); P.tasks = uniptr(in.tasks); P.ntasks = uni32(in.ntasks);
    P.scratch = uniptr(in.scratch);
    P.e_out = uniptr(in.e_out); P.scale_out = uniptr(in.scale_out); P.info_out = uniptr(in.info_out);
    P.spin_limit = (uint64_t)uni64((int64_t)in.spin_limit);
    P.trace = uniptr(in.trace);
    P.skip = uniptr(in.skip);
    return P;
}

// The solve was switched off by its skip flag (read by every kernel of the solve on entry).
__device__ __forceinline__ bool plan_skipped(const Plan &P)
{
    return P.skip && __builtin_amdgcn_readfirstlane(*(volatile const int32_t *)P.skip) != 0;
}

// blocks per tile of the consistency pass
__host__ __device__ inline int consistency_per_tile(int tm, int tn)
{
    const int per = (tm * tn + kThreads - 1) / kThreads;
    return per < 8 ? per : 8;
}

// Tasks of a solve with one task per tile update and slab (the longest task list; the
// optional phase stamps of the stamped build are stored after this many trace records).
__host__ __device__ inline int64_t max_tasks(const Plan &P)
{
    const int64_t upd = (int64_t)P.qt * P.pt * (P.pt - 1) / 2 + (int64_t)P.pt * P.qt * (P.qt - 1) / 2;
    return (int64_t)P.pt * P.qt + upd * P.slabs;
}

__host__ __device__ inline int tile_updates(const Plan &P, int T)
{
    const int i = T / P.qt, l = T % P.qt;
    return (P.pt - 1 - i) + l;
}

// Position of the update of target (i, l) by source S in the target's fixed order: sources are
// taken in order of their anti-diagonal front (pt-1-k)+l; on a tie the column source (below)
// precedes the row source (left).
__host__ __device__ inline int update_index(int pt, int i, int l, int ks, int ls)
{
    if (ls == l) {                                   // column source (ks, l), ks > i
        const int f = (pt - 1 - ks) + l;
        int rows_before = f - (pt - 1 - i);          // row sources j with front < f
        if (rows_before < 0) rows_before = 0;
        if (rows_before > l) rows_before = l;
        return (f - l) + rows_before;
    } else {                                         // row source (i, ls), ls < l
        const int f = (pt - 1 - i) + ls;
        int cols_upto = f - l + 1;                   // column sources with front <= f
        if (cols_upto < 0) cols_upto = 0;
        if (cols_upto > pt - 1 - i) cols_upto = pt - 1 - i;
        return cols_upto + ls;
    }
}

// The source of update u of target (i, l) in the order of update_index(): the column sources
// (k, l), k = pt-1 down to i+1, sit on fronts l .. l + pt-2-i, the row sources (i, j), j = 0 ..
// l-1, on fronts pt-1-i .. pt-2-i+l; the order is by front, the column source first on a tie.
// Returns the source tile's (row, column) block index in (ks, ls).
__host__ __device__ inline void update_source(int pt, int i, int l, int u, int *ks, int *ls)
{
    const int nc = pt - 1 - i, fc = l;          // column sources: count, first front
    const int nr = l, fr = pt - 1 - i;          // row sources
    // sources on fronts before f: clamp(f - fc, 0, nc) + clamp(f - fr, 0, nr); the last front
    // f with fewer than u + 1 sources before it holds source u
    auto before = [&](int f) {
        const int a = f - fc < 0 ? 0 : (f - fc > nc ? nc : f - fc);
        const int b = f - fr < 0 ? 0 : (f - fr > nr ? nr : f - fr);
        return a + b;
    };
    // before() does not decrease: the largest f < pt + l with before(f) <= u, by a search of a
    // fixed number of steps (tile indices fit in 20 bits), so that lanes never diverge in a loop
    int f = 0;
#pragma unroll
    for (int step = 1 << 20; step > 0; step >>= 1) {
        const int mid = f + step;
        if (mid < pt + l && before(mid) <= u) f = mid;
    }
    const bool col_here = f >= fc && f < fc + nc;
    if (col_here && u == before(f)) { *ks = pt - 1 - (f - l); *ls = l; }
    else { *ks = i; *ls = f - (pt - 1 - i); }
}

}  // namespace trsyl
