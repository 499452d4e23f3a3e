// C ABI of the robust triangular Sylvester solver (include/trsyl.h): argument checks,
// workspace layout, the static task order of the persistent scheduler, and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <vector>

#include "../../include/trsyl.h"
#include "extras.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace trsyl;

namespace {

constexpr int kDefaultTile = 128;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Resolved {
    int tm, tn, slabs, precision, scheduler, max_sweeps, workers, flags;
    double refine_tol;
    uint32_t *counters;
};

int device_cus()
{
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    cache[dev] = cus;
    return cus;
}

// Returns 0 or the (negative) index of the offending option argument.
int resolve(const trsyl_opts *o, Resolved *r, int argpos)
{
    trsyl_opts d;
    trsyl_default_opts(&d);
    if (!o) o = &d;
    r->tm = o->tile_m ? o->tile_m : kDefaultTile;
    r->tn = o->tile_n ? o->tile_n : r->tm;
    if (r->tm < 16 || r->tm > 256 || r->tn < 16 || r->tn > 256) return -argpos;
    r->slabs = o->slabs ? o->slabs : 1;
    const int rbmax = (r->tm + 1 + 15) / 16;
    if (r->slabs < 1 || r->slabs > 32 || r->slabs > rbmax) return -argpos;
    r->precision = o->precision;
    if (r->precision != TRSYL_FP64 && r->precision != TRSYL_FP32_REFINE) return -argpos;
    r->scheduler = o->scheduler;
    if (r->scheduler != TRSYL_SCHED_DAG && r->scheduler != TRSYL_SCHED_FRONTS) return -argpos;
    r->max_sweeps = o->max_sweeps ? (o->max_sweeps < 0 ? 0 : o->max_sweeps) : 3;
    r->refine_tol = o->refine_tol > 0 ? o->refine_tol : 1e-13;
    r->workers = o->workers > 0 ? o->workers : 0;
    r->flags = o->flags;
    r->counters = o->counters;
    return 0;
}

// ------------------------------------------------------------------------------------------
// Workspace layout
// ------------------------------------------------------------------------------------------
struct Layout {
    int pt, qt, workers;
    int64_t ntasks;
    size_t rowoff, coloff, anorm, bnorm, bdiag1, tnorm, texp, ver, misc, tasks, scratch, total;
    size_t zero_begin, zero_end;   // region cleared at the start of each call
};

int64_t count_tasks(int pt, int qt, int slabs)
{
    const int64_t upd = (int64_t)qt * pt * (pt - 1) / 2 + (int64_t)pt * qt * (qt - 1) / 2;
    return (int64_t)pt * qt + upd * slabs;
}

Layout make_layout(int64_t m, int64_t n, const Resolved &r)
{
    Layout L{};
    L.pt = (int)((m + r.tm - 1) / r.tm);
    L.qt = (int)((n + r.tn - 1) / r.tn);
    const int front = std::min(L.pt, L.qt);
    L.workers = r.workers ? r.workers : device_cus();
    L.workers = std::max(L.workers, front);
    L.ntasks = (r.scheduler == TRSYL_SCHED_DAG) ? count_tasks(L.pt, L.qt, r.slabs) : 0;
    const size_t nt = (size_t)L.pt * L.qt;
    size_t o = 0;
    L.rowoff = o; o = align_up(o + 4 * (size_t)(L.pt + 1));
    L.coloff = o; o = align_up(o + 4 * (size_t)(L.qt + 1));
    L.anorm = o; o = align_up(o + 8 * (size_t)L.pt * L.pt);
    L.bnorm = o; o = align_up(o + 8 * (size_t)L.qt * L.qt);
    L.bdiag1 = o; o = align_up(o + 8 * (size_t)L.qt);
    L.tnorm = o; o = align_up(o + 8 * 2 * nt * (size_t)r.slabs);
    L.texp = o; o = align_up(o + 4 * 2 * nt);
    L.zero_begin = o;
    L.ver = o; o = align_up(o + 4 * nt);
    L.misc = o; o = align_up(o + 64);
    L.zero_end = o;
    L.tasks = o; o = align_up(o + 8 * (size_t)L.ntasks);
    L.scratch = o; o = align_up(o + 8 * (size_t)L.workers * kMaxTile * kMaxTile);
    L.total = o;
    return L;
}

// ------------------------------------------------------------------------------------------
// Static task order for the persistent scheduler.  A list-scheduling simulation on `workers`
// identical workers (tasks on the earliest anti-diagonal front first, the tile solve before
// updates of its front) yields the start order, which is a topological order of the task
// graph: a solve after all updates of its tile, an update after its source's solve and after
// the target's previous update (each target takes its updates in the fixed order of
// update_index()).  The simulation's durations matter because the kernel follows the order
// blindly: a solve is weighted solve_cost() update units.
// ------------------------------------------------------------------------------------------
// Tile solve time over tile update time.  Measured on MI355X at tile 128: 0.40 ms per solve
// against 42 us per update (ratio 9.5).  Per solve at m = n = 8192 on one box: 8.5 / 9 / 9.5 /
// 10 / 11 gave 71.0 / 70.5 / 69.9 / 69.5 / 70.3 ms (the middle three and 10 twice each, within
// 0.05 ms), so 10 is used.  The solve's length grows with tm + tn (leaf fronts), the update's with tm tn k, so the
// ratio is scaled by (128 / tm) (128 / tn) for other tiles.
#ifndef TRSYL_SOLVE_COST
#define TRSYL_SOLVE_COST 10.0
#endif
double solve_cost(int tm, int tn)
{
    const double c = TRSYL_SOLVE_COST * (128.0 / tm) * (128.0 / tn);
    return c < 1.0 ? 1.0 : (c > 256.0 ? 256.0 : c);
}
struct TaskCache {
    std::vector<uint64_t> tasks;
    uint64_t *pinned = nullptr;
};

int tile_updates_of(int pt, int qt, int T) { return (pt - 1 - T / qt) + T % qt; }

// How the updates of a tile are grouped into tasks: one task per update (and slab), the default;
// the two updates whose sources lie on the same anti-diagonal front as one two-term task (they
// become ready together); or all pending updates of a tile as one multi-term task (left-looking,
// at most kMaxGroup terms per task).  Multi-term tasks need whole-tile update tasks (one slab).
enum UpdatePolicy : int { kPolicySingle = 0, kPolicyFrontPairs = 1, kPolicyDeferred = 2 };
int update_policy(int slabs, int flags)
{
    if (slabs > 1) return kPolicySingle;
    if (flags & kFlagDeferredUpdates) return kPolicyDeferred;
    return (flags & kFlagPairedUpdates) ? kPolicyFrontPairs : kPolicySingle;
}

std::vector<uint64_t> build_tasks(int pt, int qt, int slabs, int workers, double solve_cost, int policy)
{
    if (slabs > 1) policy = kPolicySingle;
    const int nt = pt * qt;
    std::vector<std::vector<int>> src(nt);
    std::vector<int> U(nt);
    for (int T = 0; T < nt; ++T) {
        const int i = T / qt, l = T % qt;
        U[T] = (pt - 1 - i) + l;
        src[T].assign(U[T], -1);
        for (int ks = i + 1; ks < pt; ++ks) src[T][update_index(pt, i, l, ks, l)] = ks * qt + l;
        for (int ls = 0; ls < l; ++ls) src[T][update_index(pt, i, l, i, ls)] = i * qt + ls;
    }
    std::vector<int> next_u(nt, 0), slabs_left(nt, 0);
    std::vector<char> busy(nt, 0), solved(nt, 0);
    // ready queue keyed by (front of the tile written, solve first, sequence)
    typedef std::tuple<int, int, int64_t, uint64_t> Ready;
    std::priority_queue<Ready, std::vector<Ready>, std::greater<Ready>> ready;
    typedef std::tuple<double, int64_t, uint64_t> Event;
    std::priority_queue<Event, std::vector<Event>, std::greater<Event>> events;
    int64_t seq = 0;
    auto front = [&](int T) { return (pt - 1 - T / qt) + T % qt; };
    auto push_solve = [&](int T) { ready.emplace(front(T), 0, seq++, make_task(kTaskSolve, 0, T, 0, 0)); };
    // number of updates the next task of T covers
    auto group_size = [&](int T) {
        const int u = next_u[T], left = U[T] - u;
        if (policy == kPolicyDeferred) return left < kMaxGroup ? left : kMaxGroup;
        if (policy == kPolicyFrontPairs && left >= 2 && front(src[T][u]) == front(src[T][u + 1])) return 2;
        return 1;
    };
    auto try_start = [&](int T) {
        if (busy[T] || next_u[T] >= U[T]) return;
        const int g = group_size(T);
        for (int j = 0; j < g; ++j)
            if (!solved[src[T][next_u[T] + j]]) return;
        busy[T] = 1;
        if (g > 1) {
            slabs_left[T] = 1;
            ready.emplace(front(T), 1, seq++, make_task(kTaskGroupUpdate, 0, T, g, next_u[T]));
            return;
        }
        const int S = src[T][next_u[T]];
        slabs_left[T] = slabs;
        const int kind = (S % qt == T % qt) ? kTaskColUpdate : kTaskRowUpdate;
        for (int s = 0; s < slabs; ++s) ready.emplace(front(T), 1, seq++, make_task(kind, s, T, S, next_u[T]));
    };
    for (int T = 0; T < nt; ++T)
        if (U[T] == 0) push_solve(T);
    std::vector<uint64_t> order;
    order.reserve((size_t)count_tasks(pt, qt, slabs));
    const double ts = solve_cost, tu = 1.0 / slabs;
    int free_w = workers;
    double now = 0.0;
    for (;;) {
        while (free_w > 0 && !ready.empty()) {
            const uint64_t task = std::get<3>(ready.top());
            ready.pop();
            order.push_back(task);
            --free_w;
            // a g-term update: one target read and write and g products (about half of a
            // single update's time is the products)
            const int kd = task_kind(task);
            const double dt = kd == kTaskSolve ? ts : (kd == kTaskGroupUpdate ? 0.5 + 0.5 * task_S(task) : tu);
            events.emplace(now + dt, seq++, task);
        }
        if (events.empty()) break;
        const Event ev = events.top();
        events.pop();
        now = std::get<0>(ev);
        const uint64_t task = std::get<2>(ev);
        ++free_w;
        const int T = task_T(task);
        if (task_kind(task) == kTaskSolve) {
            solved[T] = 1;
            const int k = T / qt, l = T % qt;
            for (int i = 0; i < k; ++i) try_start(i * qt + l);
            for (int j = l + 1; j < qt; ++j) try_start(k * qt + j);
        } else if (--slabs_left[T] == 0) {
            busy[T] = 0;
            next_u[T] += task_kind(task) == kTaskGroupUpdate ? task_S(task) : 1;
            if (next_u[T] == U[T]) push_solve(T);
            else try_start(T);
        }
    }
    return order;
}

// The kernel trusts the list: every tile solved once, every update covered once (in slabs or in
// a group), every index in range, at most count_tasks entries.
bool tasks_valid(const std::vector<uint64_t> &tasks, int pt, int qt, int slabs)
{
    int64_t solves = 0, covered = 0;
    bool ok = (int64_t)tasks.size() <= count_tasks(pt, qt, slabs);
    for (const uint64_t t : tasks) {
        const int kd = task_kind(t);
        if (task_T(t) >= pt * qt || task_slab(t) >= slabs) ok = false;
        if (kd == kTaskSolve) ++solves;
        else if (kd == kTaskGroupUpdate) {
            const int gsz = task_S(t);
            if (gsz < 2 || gsz > kMaxGroup || slabs != 1 ||
                task_u(t) + gsz > tile_updates_of(pt, qt, task_T(t)))
                ok = false;
            covered += (int64_t)gsz * slabs;
        } else {
            if (task_S(t) >= pt * qt) ok = false;
            covered += 1;
        }
    }
    return ok && solves == (int64_t)pt * qt && covered == count_tasks(pt, qt, slabs) - (int64_t)pt * qt;
}

const TaskCache *get_tasks(int pt, int qt, int slabs, int workers, int tm, int tn, int policy)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int, int>, TaskCache *> cache;
    std::lock_guard<std::mutex> g(mu);
    const auto key = std::make_tuple(pt, qt, slabs, workers, tm, tn, policy);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    TaskCache *tc = new TaskCache;
    tc->tasks = build_tasks(pt, qt, slabs, workers, solve_cost(tm, tn), policy);
    if (!tasks_valid(tc->tasks, pt, qt, slabs)) {
        delete tc;
        return nullptr;
    }
    const size_t bytes = tc->tasks.size() * sizeof(uint64_t);
    if (hipHostMalloc((void **)&tc->pinned, bytes ? bytes : 8, hipHostMallocDefault) != hipSuccess) {
        delete tc;
        return nullptr;
    }
    if (bytes) std::memcpy(tc->pinned, tc->tasks.data(), bytes);
    cache[key] = tc;
    return tc;
}

Plan make_plan(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
               double *C, int64_t ldc, const Resolved &r, const Layout &L, char *ws)
{
    Plan P{};
    P.m = m; P.n = n; P.lda = lda; P.ldb = ldb; P.ldc = ldc;
    P.A = A; P.B = B; P.C = C;
    P.pt = L.pt; P.qt = L.qt; P.tm = r.tm; P.tn = r.tn; P.slabs = r.slabs; P.flags = r.flags;
    P.rowoff = (int32_t *)(ws + L.rowoff);
    P.coloff = (int32_t *)(ws + L.coloff);
    P.anorm = (double *)(ws + L.anorm);
    P.bnorm = (double *)(ws + L.bnorm);
    P.bdiag1 = (double *)(ws + L.bdiag1);
    P.tnorm = (double *)(ws + L.tnorm);
    P.texp = (int32_t *)(ws + L.texp);
    P.ver = (uint32_t *)(ws + L.ver);
    char *misc = ws + L.misc;
    P.gmax = (double *)(misc + 0);
    P.status = (int32_t *)(misc + 8);
    P.ticket = (uint32_t *)(misc + 12);
    P.stats = (uint32_t *)(misc + 16);
    P.tasks = (const uint64_t *)(ws + L.tasks);
    P.ntasks = (int)L.ntasks;
    P.scratch = (double *)(ws + L.scratch);
    P.spin_limit = 100ull * 1000 * 1000 * 10;   // 10 s of the 100 MHz wall clock
    return P;
}

bool bad_ptr(const void *p) { return p == nullptr; }

}  // namespace

namespace {

// The tiled robust solve (Algorithm 4) on C in place; extra_flags adds plan flags (FP32 updates
// for the precision form's solves).  Arguments are already checked.
int solve_core(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
               double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
               const Resolved &r0, int extra_flags, char *ws, hipEvent_t *ev, uint64_t *trace,
               hipStream_t stream, const int32_t *skip = nullptr)
{
    Resolved r = r0;
    r.flags |= extra_flags;
    Layout L = make_layout(std::max<int64_t>(m, 1), std::max<int64_t>(n, 1), r);
    Plan P = make_plan(m, n, A, lda, B, ldb, C, ldc, r, L, ws);
    P.e_out = scale_log2;
    P.scale_out = scale;
    P.info_out = info;
    P.trace = trace;
    P.skip = skip;
    if (m == 0 || n == 0) {
        P.pt = P.qt = 0;
        if (launch_fill_zero(ws, kAlign, stream) != hipSuccess) return -100;
        // finalize with no tiles writes e = 0, alpha = 1 and the (zero) status
        P.status = (int32_t *)(ws + 8);
        if (r.counters && launch_fill_zero(r.counters, 16, stream) != hipSuccess) return -100;
        return launch_finalize(P, stream) == hipSuccess ? 0 : -100;
    }
    if (launch_fill_zero(ws + L.zero_begin, L.zero_end - L.zero_begin, stream) != hipSuccess) return -100;
    if (launch_setup(P, stream) != hipSuccess) return -100;
    if (r.scheduler == TRSYL_SCHED_DAG) {
        const TaskCache *tc = get_tasks(L.pt, L.qt, r.slabs, L.workers, r.tm, r.tn, update_policy(r.slabs, r.flags));
        if (!tc) return -100;
        P.ntasks = (int)tc->tasks.size();
        if (hipMemcpyAsync(ws + L.tasks, tc->pinned, tc->tasks.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, stream) != hipSuccess)
            return -100;
        if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return -100;
        if (launch_dag(P, L.workers, stream) != hipSuccess) return -100;
    } else {
        if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return -100;
        if (launch_fronts(P, stream) != hipSuccess) return -100;
    }
    if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return -100;
    if (launch_finalize(P, stream) != hipSuccess) return -100;
    if (r.counters && hipMemcpyAsync(r.counters, P.stats, 4 * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                     stream) != hipSuccess)
        return -100;
    return 0;
}

size_t refine_extra(int64_t m, int64_t n)
{
    const size_t mn = 8 * (size_t)m * n;
    return 2 * align_up(mn) + align_up(8 * (size_t)kNormParts) + kAlign;
}

// Precision form: the tiled solve with FP32-MFMA tile updates (tile solves, bounds and scale
// decisions in FP64), then at most max_sweeps refinement sweeps in FP64.  Sweep: with 2^sy > max|Y|,
//   R' = 2^-(e+sy) C0 - 2^-sy (A Y + Y B)            (FP64 MFMA GEMMs, C0 the original C)
//   if eq. (9) of (Y, e), formed from ||R'||, ||A||, ||B||, ||Ys||, ||C0||, is at most refine_tol:
//       stop (a device flag turns this and every later kernel of the refinement into a no-op)
//   A D + D B = 2^-eD R'                              (the FP32-update solve, robust)
//   Y <- 2^-(eD+x) Y + 2^(sy-x) D,  e <- e + eD + x  (so A Y + Y B = 2^-e C0 again; the extra
//                                                      power of two x keeps Y in range)
// All on the stream; no host synchronisation.  counters[3] receives the number of sweeps that
// updated Y.
int solve_refined(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                  double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
                  const Resolved &r, char *ws, hipEvent_t *ev, hipStream_t stream)
{
    Resolved rc = r;
    rc.precision = TRSYL_FP64;
    Resolved rsweep = rc;          // the correction solves leave the caller's counters alone
    rsweep.counters = nullptr;
    const size_t core = make_layout(m, n, rc).total;
    const size_t mn = 8 * (size_t)m * n;
    double *C0 = (double *)(ws + core);
    double *D = (double *)(ws + core + align_up(mn));
    double *part = (double *)(ws + core + 2 * align_up(mn));
    char *sc = ws + core + 2 * align_up(mn) + align_up(8 * (size_t)kNormParts);
    int64_t *eD = (int64_t *)(sc + 0);
    int64_t *negsy = (int64_t *)(sc + 8);
    int32_t *infoD = (int32_t *)(sc + 16);
    int32_t *sD = (int32_t *)(sc + 20);
    int32_t *skip = (int32_t *)(sc + 24);
    uint32_t *sweeps = (uint32_t *)(sc + 28);
    int32_t *s5 = (int32_t *)(sc + 32);        // norm exponents of R', A, B, Y, C0
    double *t5 = (double *)(sc + 56);          // and their sums of squares
    const int mi = (int)m, ni = (int)n;
    if (launch_fill_zero(sc, kAlign, stream) != hipSuccess) return -100;
    if (hipMemcpy2DAsync(C0, 8 * (size_t)m, C, 8 * (size_t)ldc, 8 * (size_t)m, (size_t)n,
                         hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return -100;
    if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return -100;
    int rcode = solve_core(m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, rc, kFlagF32Updates, ws,
                           nullptr, nullptr, stream);
    if (rcode) return rcode;
    if (r.max_sweeps > 0) {
        if (launch_norm(A, lda, mi, mi, 1, part, s5 + 1, t5 + 1, stream) != hipSuccess) return -100;
        if (launch_norm(B, ldb, ni, ni, 1, part, s5 + 2, t5 + 2, stream) != hipSuccess) return -100;
        if (launch_norm(C0, mi, mi, ni, 0, part, s5 + 4, t5 + 4, stream) != hipSuccess) return -100;
    }
    for (int sweep = 0; sweep < r.max_sweeps; ++sweep) {
        if (launch_norm(C, ldc, mi, ni, 0, part, s5 + 3, t5 + 3, stream, skip) != hipSuccess) return -100;
        if (launch_neg_exp(s5 + 3, negsy, stream, skip) != hipSuccess) return -100;
        GemmDesc g{};
        g.M = mi; g.N = ni; g.K = mi;                 // D = 2^(-e-sy) C0 - 2^-sy A Y
        g.A = A; g.sAm = 1; g.sAk = lda; g.triA = 1;
        g.B = C; g.sBk = 1; g.sBn = ldc; g.triB = 0;
        g.Cin = C0; g.ldcin = mi;
        g.Out = D; g.ldo = mi;
        g.sa1 = 0; g.sb1 = 1;                         // Y staged as 2^-sy Y
        g.asign = -1.0; g.ae0 = 0; g.ae1 = 0; g.ae2 = 0;
        g.csign = 1.0; g.ce0 = 0; g.ce1 = 1; g.ce2 = -1;
        g.ep1 = negsy; g.ep2 = scale_log2;
        g.mask = 0; g.pat = nullptr; g.ldpat = 1;
        g.skip = skip;
        if (launch_gemm(g, stream) != hipSuccess) return -100;
        g.K = ni;                                     // D -= 2^-sy Y B
        g.A = C; g.sAm = 1; g.sAk = ldc; g.triA = 0;
        g.B = B; g.sBk = 1; g.sBn = ldb; g.triB = 1;
        g.sa1 = 1; g.sb1 = 0;
        g.Cin = D; g.ldcin = mi;
        g.ce1 = 0; g.ce2 = 0;
        if (launch_gemm(g, stream) != hipSuccess) return -100;
        if (launch_norm(D, mi, mi, ni, 0, part, s5 + 0, t5 + 0, stream, skip) != hipSuccess) return -100;
        if (launch_refine_check(s5, t5, scale_log2, r.refine_tol, skip, stream) != hipSuccess) return -100;
        rcode = solve_core(m, n, A, lda, B, ldb, D, m, eD, nullptr, infoD, rsweep, kFlagF32Updates, ws, nullptr,
                           nullptr, stream, skip);
        if (rcode) return rcode;
        if (launch_absmax_exp(D, m, mi, ni, part, sD, stream, skip) != hipSuccess) return -100;
        if (launch_refine_update(C, ldc, D, m, mi, ni, eD, negsy, sD, scale_log2, info, infoD, scale,
                                 stream, skip, sweeps) != hipSuccess)
            return -100;
    }
    if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return -100;
    if (r.counters && hipMemcpyAsync(r.counters + 3, sweeps, sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                     stream) != hipSuccess)
        return -100;
    return 0;
}


// ---------------------------------------------------------------------------------------------
// Batched solves.  Workspace: plans, stage offset tables and the ticket; then one region per
// problem (its layout up to the zeroed state); then the shared per-worker scratch; then the merged
// task list and the problem index of every task.
// ---------------------------------------------------------------------------------------------
struct BLayout {
    int count = 0, workers = 0;
    std::vector<Resolved> r;
    std::vector<Layout> L;
    std::vector<size_t> region;           // offset of problem p's region
    size_t plans = 0, offs = 0, ticket = 0, regions_begin = 0, regions_end = 0, scratch = 0,
           tasks = 0, tprob = 0, total = 0;
    int64_t ntasks = 0;
    // precision form: per problem C0 (the original C) and D (the correction), each m x n
    // column-major; then shared norm partials and per-problem sweep scalars
    bool refine = false;
    int max_sweeps = 0;
    double refine_tol = 0.0;
    std::vector<size_t> c0, d;
    size_t part = 0, eD = 0, negsy = 0, infoD = 0, s5 = 0, t5 = 0, sD = 0, skip = 0;
};

// Returns 0 or the negative argument index that is invalid.
int make_blayout(int32_t count, const int64_t *m, const int64_t *n, const int32_t *tiles,
                 const trsyl_opts *opts, BLayout *B)
{
    B->count = count;
    B->r.resize(count);
    B->L.resize(count);
    B->region.resize(count);
    Resolved base;
    if (int e = resolve(opts, &base, 14)) return e;
    B->refine = base.precision == TRSYL_FP32_REFINE;
    B->max_sweeps = base.max_sweeps;
    B->refine_tol = base.refine_tol;
    B->workers = base.workers ? base.workers : device_cus();
    size_t o = 0;
    B->plans = o; o = align_up(o + sizeof(Plan) * (size_t)count);
    B->offs = o; o = align_up(o + 4 * 5 * (size_t)(count + 1));
    B->ticket = o; o = align_up(o + 4);
    B->regions_begin = o;
    for (int p = 0; p < count; ++p) {
        if (m[p] < 0 || n[p] < 0 || m[p] > (int64_t)INT32_MAX / 2 || n[p] > (int64_t)INT32_MAX / 2) return -2;
        trsyl_opts op;
        if (opts) op = *opts; else trsyl_default_opts(&op);
        if (tiles) { op.tile_m = tiles[2 * p]; op.tile_n = tiles[2 * p + 1]; }
        if (int e = resolve(&op, &B->r[p], 10)) return e;
        B->r[p].precision = TRSYL_FP64;
        B->r[p].scheduler = TRSYL_SCHED_DAG;
        Resolved rr = B->r[p];
        rr.workers = B->workers;
        B->L[p] = make_layout(std::max<int64_t>(m[p], 1), std::max<int64_t>(n[p], 1), rr);
        if (m[p] == 0 || n[p] == 0) { B->L[p].pt = 0; B->L[p].qt = 0; }
        B->region[p] = o;
        o = align_up(o + B->L[p].zero_end);
        B->ntasks += (B->L[p].pt && B->L[p].qt) ? count_tasks(B->L[p].pt, B->L[p].qt, B->r[p].slabs) : 0;
    }
    B->regions_end = o;
    B->scratch = o; o = align_up(o + 8 * (size_t)B->workers * kMaxTile * kMaxTile);
    B->tasks = o; o = align_up(o + 8 * (size_t)B->ntasks);
    B->tprob = o; o = align_up(o + 4 * (size_t)B->ntasks);
    if (B->refine) {
        B->c0.resize(count);
        B->d.resize(count);
        for (int p = 0; p < count; ++p) {
            const size_t mn = 8 * (size_t)m[p] * (size_t)n[p];
            B->c0[p] = o; o = align_up(o + mn);
            B->d[p] = o; o = align_up(o + mn);
        }
        B->part = o; o = align_up(o + 8 * (size_t)kNormParts);
        B->eD = o; o = align_up(o + 8 * (size_t)count);
        B->negsy = o; o = align_up(o + 8 * (size_t)count);
        B->infoD = o; o = align_up(o + 4 * (size_t)count);
        B->s5 = o; o = align_up(o + 4 * 5 * (size_t)count);     // norm exponents: R', A, B, Y, C0
        B->t5 = o; o = align_up(o + 8 * 5 * (size_t)count);     // and sums of squares
        B->sD = o; o = align_up(o + 4 * (size_t)count);
        B->skip = o; o = align_up(o + 4 * (size_t)count);       // converged problems
    }
    B->total = o;
    return 0;
}

// Merged task order: every problem's own topological order (from its list-scheduling
// simulation), interleaved by fractional progress -- the next task is the one whose position in
// its problem's list, divided by that list's length, is smallest (larger problems first on ties).
struct MergedTasks {
    uint64_t *pinned = nullptr;   // tasks, then the uint32 problem indices
    int64_t n = 0;
};
const MergedTasks *get_merged(const BLayout &B, const int64_t *m, const int64_t *n)
{
    static std::mutex mu;
    static std::map<std::vector<int64_t>, MergedTasks *> cache;
    std::vector<int64_t> key;
    key.push_back(B.workers);
    for (int p = 0; p < B.count; ++p) {
        key.push_back(B.L[p].pt); key.push_back(B.L[p].qt); key.push_back(B.r[p].slabs);
        key.push_back(B.r[p].tm); key.push_back(B.r[p].tn);
        key.push_back(update_policy(B.r[p].slabs, B.r[p].flags));
        key.push_back(m[p] * n[p] * (m[p] + n[p]));
    }
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    std::vector<const TaskCache *> lists(B.count, nullptr);
    for (int p = 0; p < B.count; ++p) {
        if (B.L[p].pt && B.L[p].qt) {
            lists[p] = get_tasks(B.L[p].pt, B.L[p].qt, B.r[p].slabs, B.workers, B.r[p].tm, B.r[p].tn,
                                 update_policy(B.r[p].slabs, B.r[p].flags));
            if (!lists[p]) return nullptr;
        }
    }
    typedef std::tuple<double, int64_t, int> Key;    // (fraction, -flops, problem)
    std::priority_queue<Key, std::vector<Key>, std::greater<Key>> q;
    std::vector<size_t> pos(B.count, 0);
    auto push = [&](int p) {
        const size_t len = lists[p]->tasks.size();
        if (pos[p] < len) q.emplace((double)(pos[p] + 1) / (double)len, -(m[p] * n[p] * (m[p] + n[p])), p);
    };
    for (int p = 0; p < B.count; ++p) if (lists[p]) push(p);
    MergedTasks *mt = new MergedTasks;
    mt->n = 0;
    for (int p = 0; p < B.count; ++p) if (lists[p]) mt->n += (int64_t)lists[p]->tasks.size();
    const size_t bytes = 12 * (size_t)B.ntasks + 8;
    if (hipHostMalloc((void **)&mt->pinned, bytes, hipHostMallocDefault) != hipSuccess) { delete mt; return nullptr; }
    uint32_t *prob = (uint32_t *)(mt->pinned + B.ntasks);
    int64_t k = 0;
    while (!q.empty()) {
        const int p = std::get<2>(q.top());
        q.pop();
        mt->pinned[k] = lists[p]->tasks[pos[p]];
        prob[k] = (uint32_t)p;
        ++k;
        ++pos[p];
        push(p);
    }
    if (k != mt->n || mt->n > B.ntasks) { (void)hipHostFree(mt->pinned); delete mt; return nullptr; }
    cache[key] = mt;
    return mt;
}

// One batched solve over the layout BL (plans rebuilt for the given C, scale and info arrays).
int batched_core(const BLayout &BL, int32_t count, const int64_t *m, const int64_t *n, const double *const *A,
                 const int64_t *lda, const double *const *B, const int64_t *ldb, double *const *C,
                 const int64_t *ldc, int64_t *scale_log2, double *scale, int32_t *info, int extra_flags,
                 char *ws, hipEvent_t *ev, hipStream_t stream, const int32_t *skip = nullptr)
{
    // host images of the plans and the stage offset tables
    std::vector<Plan> plans(count);
    std::vector<int32_t> offs(5 * (size_t)(count + 1), 0);
    int32_t *oS = offs.data(), *oA = oS + (count + 1), *oB = oA + (count + 1), *oC = oB + (count + 1),
            *oK = oC + (count + 1);
    for (int p = 0; p < count; ++p) {
        const Layout &L = BL.L[p];
        Resolved rp = BL.r[p];
        rp.flags |= extra_flags;
        Plan P = make_plan(m[p], n[p], A[p], lda[p], B[p], ldb[p], C[p], ldc[p], rp, L, ws + BL.region[p]);
        P.pt = L.pt; P.qt = L.qt;
        P.tasks = nullptr; P.ntasks = 0;
        P.scratch = (double *)(ws + BL.scratch);
        P.ticket = (uint32_t *)(ws + BL.ticket);
        P.e_out = scale_log2 + p;
        P.scale_out = scale ? scale + p : nullptr;
        P.info_out = info + p;
        P.trace = nullptr;
        P.skip = skip ? skip + p : nullptr;
        plans[p] = P;
        const int64_t items = std::max(m[p], n[p]) + 2;
        const int gS = (L.pt && L.qt) ? (int)std::min<int64_t>((items + 255) / 256, 64) : 0;
        oS[p + 1] = oS[p] + gS;
        oA[p + 1] = oA[p] + ((L.pt && L.qt) ? L.pt * L.pt : 0);
        oB[p + 1] = oB[p] + ((L.pt && L.qt) ? L.qt * L.qt : 0);
        oC[p + 1] = oC[p] + L.pt * L.qt;
        oK[p + 1] = oK[p] + ((L.pt && L.qt) ? consistency_per_tile(BL.r[p].tm, BL.r[p].tn) * L.pt * L.qt : 0);
    }
    const MergedTasks *mt = get_merged(BL, m, n);
    if (!mt) return -100;
    if (launch_fill_zero(ws + BL.ticket, BL.regions_end - BL.ticket, stream) != hipSuccess) return -100;
    if (hipMemcpyAsync(ws + BL.plans, plans.data(), sizeof(Plan) * (size_t)count, hipMemcpyHostToDevice,
                       stream) != hipSuccess)
        return -100;
    if (hipMemcpyAsync(ws + BL.offs, offs.data(), 4 * offs.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
        return -100;
    if (BL.ntasks > 0) {
        if (hipMemcpyAsync(ws + BL.tasks, mt->pinned, 8 * (size_t)BL.ntasks, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            hipMemcpyAsync(ws + BL.tprob, mt->pinned + BL.ntasks, 4 * (size_t)BL.ntasks, hipMemcpyHostToDevice,
                           stream) != hipSuccess)
            return -100;
    }
    BatchedLaunch bl{};
    bl.count = count;
    bl.plans = (const Plan *)(ws + BL.plans);
    const int32_t *dof = (const int32_t *)(ws + BL.offs);
    bl.off_structure = dof;
    bl.off_A = dof + (count + 1);
    bl.off_B = dof + 2 * (count + 1);
    bl.off_C = dof + 3 * (count + 1);
    bl.off_consistency = dof + 4 * (count + 1);
    bl.blocks_structure = oS[count];
    bl.blocks_bounds = oA[count] + oB[count] + oC[count];
    bl.blocks_consistency = oK[count];
    bl.tasks = (const uint64_t *)(ws + BL.tasks);
    bl.tprob = (const uint32_t *)(ws + BL.tprob);
    bl.ntasks = mt->n;
    bl.ticket = (uint32_t *)(ws + BL.ticket);
    bl.scratch = (double *)(ws + BL.scratch);
    bl.workers = BL.workers;
    if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return -100;
    if (launch_batched(bl, stream) != hipSuccess) return -100;
    if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return -100;
    return 0;
}

// The precision form over a batch: the batched FP32-update solve, then max_sweeps sweeps, each
// forming every problem's FP64 residual (as in solve_refined), solving all corrections in one
// batched FP32-update solve, and updating every problem.  Per problem the launches and their
// order match solve_refined's, so each result equals the single solve's with the same tiles.
int batched_refined(const BLayout &BL, int32_t count, const int64_t *m, const int64_t *n,
                    const double *const *A, const int64_t *lda, const double *const *B, const int64_t *ldb,
                    double *const *C, const int64_t *ldc, int64_t *scale_log2, double *scale, int32_t *info,
                    char *ws, hipEvent_t *ev, hipStream_t stream)
{
    std::vector<double *> Dp(count);
    std::vector<int64_t> ldd(count);
    for (int p = 0; p < count; ++p) {
        Dp[p] = (double *)(ws + BL.d[p]);
        ldd[p] = std::max<int64_t>(1, m[p]);
        if (m[p] > 0 && n[p] > 0 &&
            hipMemcpy2DAsync(ws + BL.c0[p], 8 * (size_t)m[p], C[p], 8 * (size_t)ldc[p], 8 * (size_t)m[p],
                             (size_t)n[p], hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return -100;
    }
    if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return -100;
    int rcode = batched_core(BL, count, m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, kFlagF32Updates,
                             ws, nullptr, stream);
    if (rcode) return rcode;
    double *part = (double *)(ws + BL.part);
    int64_t *eD = (int64_t *)(ws + BL.eD), *negsy = (int64_t *)(ws + BL.negsy);
    int32_t *infoD = (int32_t *)(ws + BL.infoD), *s5 = (int32_t *)(ws + BL.s5), *sD = (int32_t *)(ws + BL.sD);
    double *t5 = (double *)(ws + BL.t5);
    int32_t *skip = (int32_t *)(ws + BL.skip);
    if (launch_fill_zero(skip, 4 * (size_t)count, stream) != hipSuccess) return -100;
    if (BL.max_sweeps > 0) {
        for (int p = 0; p < count; ++p) {
            if (m[p] == 0 || n[p] == 0) continue;
            const int mi = (int)m[p], ni = (int)n[p];
            if (launch_norm(A[p], lda[p], mi, mi, 1, part, s5 + 5 * p + 1, t5 + 5 * p + 1, stream) != hipSuccess ||
                launch_norm(B[p], ldb[p], ni, ni, 1, part, s5 + 5 * p + 2, t5 + 5 * p + 2, stream) != hipSuccess ||
                launch_norm((const double *)(ws + BL.c0[p]), mi, mi, ni, 0, part, s5 + 5 * p + 4, t5 + 5 * p + 4,
                            stream) != hipSuccess)
                return -100;
        }
    }
    for (int sweep = 0; sweep < BL.max_sweeps; ++sweep) {
        for (int p = 0; p < count; ++p) {
            if (m[p] == 0 || n[p] == 0) continue;
            const int mi = (int)m[p], ni = (int)n[p];
            const int32_t *sk = skip + p;
            if (launch_norm(C[p], ldc[p], mi, ni, 0, part, s5 + 5 * p + 3, t5 + 5 * p + 3, stream, sk) != hipSuccess)
                return -100;
            if (launch_neg_exp(s5 + 5 * p + 3, negsy + p, stream, sk) != hipSuccess) return -100;
            GemmDesc g{};
            g.M = mi; g.N = ni; g.K = mi;                 // D = 2^(-e-sy) C0 - 2^-sy A Y
            g.A = A[p]; g.sAm = 1; g.sAk = lda[p]; g.triA = 1;
            g.B = C[p]; g.sBk = 1; g.sBn = ldc[p]; g.triB = 0;
            g.Cin = (const double *)(ws + BL.c0[p]); g.ldcin = mi;
            g.Out = Dp[p]; g.ldo = mi;
            g.sa1 = 0; g.sb1 = 1;
            g.asign = -1.0; g.ae0 = 0; g.ae1 = 0; g.ae2 = 0;
            g.csign = 1.0; g.ce0 = 0; g.ce1 = 1; g.ce2 = -1;
            g.ep1 = negsy + p; g.ep2 = scale_log2 + p;
            g.mask = 0; g.pat = nullptr; g.ldpat = 1;
            g.skip = sk;
            if (launch_gemm(g, stream) != hipSuccess) return -100;
            g.K = ni;                                     // D -= 2^-sy Y B
            g.A = C[p]; g.sAm = 1; g.sAk = ldc[p]; g.triA = 0;
            g.B = B[p]; g.sBk = 1; g.sBn = ldb[p]; g.triB = 1;
            g.sa1 = 1; g.sb1 = 0;
            g.Cin = Dp[p]; g.ldcin = mi;
            g.ce1 = 0; g.ce2 = 0;
            if (launch_gemm(g, stream) != hipSuccess) return -100;
            if (launch_norm(Dp[p], mi, mi, ni, 0, part, s5 + 5 * p + 0, t5 + 5 * p + 0, stream, sk) != hipSuccess)
                return -100;
            if (launch_refine_check(s5 + 5 * p, t5 + 5 * p, scale_log2 + p, BL.refine_tol, skip + p, stream) !=
                hipSuccess)
                return -100;
        }
        rcode = batched_core(BL, count, m, n, A, lda, B, ldb, Dp.data(), ldd.data(), eD, nullptr, infoD,
                             kFlagF32Updates, ws, nullptr, stream, skip);
        if (rcode) return rcode;
        for (int p = 0; p < count; ++p) {
            if (m[p] == 0 || n[p] == 0) continue;
            const int mi = (int)m[p], ni = (int)n[p];
            if (launch_absmax_exp(Dp[p], mi, mi, ni, part, sD + p, stream, skip + p) != hipSuccess) return -100;
            if (launch_refine_update(C[p], ldc[p], Dp[p], mi, mi, ni, eD + p, negsy + p, sD + p, scale_log2 + p,
                                     info + p, infoD + p, scale ? scale + p : nullptr, stream, skip + p) != hipSuccess)
                return -100;
        }
    }
    if (ev && hipEventRecord(ev[1], stream) != hipSuccess) return -100;
    return 0;
}

}  // namespace

namespace trsyl {

// The solve of trsyl_robust_noalloc on a caller-provided region `ws` of `cap` bytes: FP64, the
// per-front scheduler (no host-built task list), one scratch tile per workgroup of a front.
// Returns 0, a negative argument index, kNoAllocTooLarge when the state does not fit in `cap`, or
// -100 on a launch error.  Allocates nothing.
static int noalloc_resolve(const trsyl_opts *opts, Resolved *r)
{
    if (int e = resolve(opts, r, 12)) return e;
    if (r->precision != TRSYL_FP64) return -12;
    r->scheduler = TRSYL_SCHED_FRONTS;
    r->workers = 1;       // make_layout raises it to the widest front, the only workgroups that need a tile
    return 0;
}

// Bytes of state the no-allocation solve needs (host only, no device call).
int noalloc_need(int64_t m, int64_t n, const trsyl_opts *opts, size_t *need)
{
    Resolved r;
    if (int e = noalloc_resolve(opts, &r)) return e;
    *need = (m > 0 && n > 0) ? make_layout(m, n, r).total : kAlign;
    return 0;
}

int noalloc_solve(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                  int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info, const trsyl_opts *opts,
                  char *ws, size_t cap, hipStream_t stream)
{
    Resolved r;
    if (int e = noalloc_resolve(opts, &r)) return e;
    if (m > 0 && n > 0 && make_layout(m, n, r).total > cap) return kNoAllocTooLarge;
    hipEvent_t *ev = opts ? (hipEvent_t *)opts->profile_events : nullptr;
    return solve_core(m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, r, 0, ws, ev, nullptr, stream);
}

// Argument checks shared by trsyl_robust and trsyl_robust_noalloc (workspace aside).
int check_solve_args(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                     const double *C, int64_t ldc, const int64_t *scale_log2, const int32_t *info)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (m > 0 && bad_ptr(A)) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (n > 0 && bad_ptr(B)) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (m > 0 && n > 0 && bad_ptr(C)) return -7;
    if (ldc < std::max<int64_t>(1, m)) return -8;
    if (bad_ptr(scale_log2)) return -9;
    if (bad_ptr(info)) return -11;
    if (m > (int64_t)INT32_MAX / 2 || n > (int64_t)INT32_MAX / 2) return -1;
    return 0;
}

}  // namespace trsyl

extern "C" {

void trsyl_default_opts(trsyl_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tile_m = kDefaultTile;
    o->tile_n = kDefaultTile;
    o->precision = TRSYL_FP64;
    o->scheduler = TRSYL_SCHED_DAG;
    o->max_sweeps = 3;
    o->refine_tol = 1e-13;
}

const char *trsyl_version(void) { return "trsyl-mi355x 0.1"; }

size_t trsyl_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts)
{
    Resolved r;
    if (m < 0 || n < 0 || resolve(opts, &r, 3)) return 0;
    if (m == 0 || n == 0) return kAlign;
    const size_t core = make_layout(m, n, r).total;
    if (r.precision == TRSYL_FP64) return core;
    return core + refine_extra(m, n);
}

int trsyl_robust(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
                 const trsyl_opts *opts, void *workspace, size_t ws_bytes, trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (int e = check_solve_args(m, n, A, lda, B, ldb, C, ldc, scale_log2, info)) return e;
    Resolved r;
    if (int e = resolve(opts, &r, 12)) return e;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -13;
    const size_t need = trsyl_workspace_size(m, n, opts);
    if (ws_bytes < need) return -14;
    hipEvent_t *ev = opts ? (hipEvent_t *)opts->profile_events : nullptr;
    uint64_t *trace = opts ? opts->trace : nullptr;
    if (r.precision == TRSYL_FP64 || m == 0 || n == 0)
        return solve_core(m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, r, 0, (char *)workspace,
                          ev, trace, stream);
    return solve_refined(m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, r, (char *)workspace, ev,
                         stream);
}

int trsyl_debug_protect_update(int32_t count, const double *in, int32_t *out, trsyl_stream_t s)
{
    if (count < 0) return -1;
    if (count > 0 && (bad_ptr(in) || bad_ptr(out))) return -2;
    return launch_debug_protect(0, count, in, out, (hipStream_t)s) == hipSuccess ? 0 : -100;
}

int trsyl_debug_protect_division(int32_t count, const double *in, int32_t *out, trsyl_stream_t s)
{
    if (count < 0) return -1;
    if (count > 0 && (bad_ptr(in) || bad_ptr(out))) return -2;
    return launch_debug_protect(1, count, in, out, (hipStream_t)s) == hipSuccess ? 0 : -100;
}

int64_t trsyl_debug_task_order(int32_t pt, int32_t qt, int32_t tile_m, int32_t tile_n, int32_t slabs,
                               int32_t workers, int32_t flags, uint64_t *out, int64_t cap)
{
    if (pt < 1 || pt > 4096) return -1;
    if (qt < 1 || qt > 4096 || (int64_t)pt * qt >= (1 << 20)) return -2;
    if (tile_m < 16 || tile_m > 256) return -3;
    if (tile_n < 16 || tile_n > 256) return -4;
    if (slabs < 1 || slabs > 32) return -5;
    if (workers < 1) return -6;
    if (cap < 0 || (cap > 0 && !out)) return -9;
    const std::vector<uint64_t> t =
        build_tasks(pt, qt, slabs, workers, solve_cost(tile_m, tile_n), update_policy(slabs, flags));
    if (!tasks_valid(t, pt, qt, slabs)) return -100;
    for (int64_t i = 0; i < (int64_t)t.size() && i < cap; ++i) out[i] = t[i];
    return (int64_t)t.size();
}


size_t trsyl_batched_workspace_size(int32_t count, const int64_t *m, const int64_t *n, const int32_t *tiles,
                                    const trsyl_opts *opts)
{
    if (count < 0 || (count > 0 && (!m || !n))) return 0;
    BLayout B;
    if (make_blayout(count, m, n, tiles, opts, &B)) return 0;
    return B.total;
}

int trsyl_robust_batched(int32_t count, const int64_t *m, const int64_t *n, const double *const *A,
                         const int64_t *lda, const double *const *B, const int64_t *ldb, double *const *C,
                         const int64_t *ldc, const int32_t *tiles, int64_t *scale_log2, double *scale,
                         int32_t *info, const trsyl_opts *opts, void *workspace, size_t ws_bytes,
                         trsyl_stream_t stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (count < 0) return -1;
    if (count == 0) return 0;
    if (!m || !n) return -2;
    if (!A || !lda) return -4;
    if (!B || !ldb) return -6;
    if (!C || !ldc) return -8;
    if (bad_ptr(scale_log2)) return -11;
    if (bad_ptr(info)) return -13;
    for (int p = 0; p < count; ++p) {
        if (m[p] < 0 || n[p] < 0) return -2;
        if (m[p] > 0 && bad_ptr(A[p])) return -4;
        if (lda[p] < std::max<int64_t>(1, m[p])) return -5;
        if (n[p] > 0 && bad_ptr(B[p])) return -6;
        if (ldb[p] < std::max<int64_t>(1, n[p])) return -7;
        if (m[p] > 0 && n[p] > 0 && bad_ptr(C[p])) return -8;
        if (ldc[p] < std::max<int64_t>(1, m[p])) return -9;
    }
    BLayout BL;
    if (int e = make_blayout(count, m, n, tiles, opts, &BL)) return e;
    if (bad_ptr(workspace) || ((uintptr_t)workspace % kAlign) != 0) return -15;
    if (ws_bytes < BL.total) return -16;
    char *ws = (char *)workspace;
    hipEvent_t *ev = opts ? (hipEvent_t *)opts->profile_events : nullptr;
    if (!BL.refine)
        return batched_core(BL, count, m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, 0, ws, ev, stream);
    return batched_refined(BL, count, m, n, A, lda, B, ldb, C, ldc, scale_log2, scale, info, ws, ev, stream);
}

}  // extern "C"
