/*
 * trsyl.h -- robust solver for the triangular Sylvester equation on AMD Instinct MI355X (gfx950)
 *
 *     A Y + Y B = alpha C,     A (m x m), B (n x n) upper quasi-triangular (real Schur form),
 *
 * after Schwarz & Kjelgaard Mikkelsen, "Robust Task-Parallel Solution of the Triangular
 * Sylvester Equation" (arXiv 1905.10574).  The scale alpha in (0, 1] is chosen on the fly so
 * that no intermediate value exceeds the overflow threshold OMEGA = 2^1022 (Sec. 2, eq. (7)).
 *
 * Conventions shared by every entry point
 *   - All matrix pointers are DEVICE pointers to column-major float64 storage with leading
 *     dimensions (LAPACK layout).  Only the entries of A and B on or above the first
 *     subdiagonal are read.  A nonzero first-subdiagonal entry T(i+1, i) marks a 2x2 diagonal
 *     block (Sec. 1, eq. (4)); two consecutive nonzero subdiagonal entries are an error.
 *   - The caller owns every buffer, including the workspace; the library never allocates
 *     device memory on the solve path.  Size the workspace with the matching *_workspace_size
 *     call, for the same arguments and options.
 *   - Work is enqueued on `stream` and is asynchronous.  Results (Y, the scale exponent, the
 *     status) are written to device memory in stream order.
 *   - alpha is returned as an exact power of two: alpha = 2^-e with integer e >= 0 written to
 *     *scale_log2 (int64), and as a double in *scale (0.0 once e exceeds 1074).  Exponents,
 *     not doubles, carry the scale because strongly growing problems need e far beyond the
 *     double range.
 *   - Return value (synchronous, host): 0 when the work was enqueued, -i when argument i is
 *     invalid (null pointer, negative size, leading dimension too small, workspace too small,
 *     bad option), -100 on a HIP launch error.
 *   - Device status (*info, int32, written in stream order):
 *        0  success
 *        1  a pivot of a small 1x1/2x2 Sylvester solve fell below smin and was replaced by
 *           +-smin (lambda_A + lambda_B = 0 to working precision; Sec. 1 uniqueness
 *           condition); the result solves a nearby problem
 *        2  A or B is not upper quasi-triangular (two consecutive nonzero subdiagonals)
 *        3  non-finite input, an input entry above OMEGA, or a tile of A, B or C (in the
 *           call's tiling, opts->tile_m / tile_n) whose infinity norm exceeds OMEGA: the data
 *           requirement of Alg. 4 (entries at most OMEGA do not imply it; a finer tiling may
 *           accept what a coarser one rejects)
 *        4  the persistent scheduler's watchdog expired (a dependency never resolved)
 *     On status 2 or 3 the contents of C are unspecified.
 *   - Functions are reentrant: concurrent calls need distinct workspaces.
 *   - Host memory: the persistent scheduler (trsyl_robust and the entry points built on it, the
 *     batched solves) follows a static task order that the library computes on the host the first
 *     time it meets a tiling shape (tile counts, tile sizes, slabs, workgroups) and keeps, for the
 *     life of the process, in pinned host memory (hipHostMalloc, 8 bytes per task, e.g. 2 MB for
 *     m = n = 8192 with tile 128; a merged list for each batched problem set), from which each call
 *     copies it into the workspace on the stream.  A first call per shape therefore allocates
 *     pinned host memory and runs the list-scheduling simulation; later calls reuse the list.  The
 *     cache is never trimmed (a list may still be the source of a copy in flight).  The per-front
 *     scheduler and trsyl_robust_noalloc use no task list.
 */
#ifndef TRSYL_H
#define TRSYL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *trsyl_stream_t; /* a hipStream_t; NULL = the null stream */

enum trsyl_precision {
    TRSYL_FP64 = 0,        /* every step in FP64 */
    TRSYL_FP32_REFINE = 1, /* tile updates on FP32 MFMA with power-of-two operand scaling,
                              tile solves / bounds / residual in FP64, iterative refinement */
};

enum trsyl_scheduler {
    TRSYL_SCHED_DAG = 0,    /* one persistent kernel walks the tile dependency graph */
    TRSYL_SCHED_FRONTS = 1, /* one launch per anti-diagonal front (stream ordered) */
};

#define TRSYL_FLAG_ROBUST_SOLVE 1
#define TRSYL_FLAG_PAIRED_UPDATES 4
#define TRSYL_FLAG_DEFERRED_UPDATES 8

typedef struct trsyl_opts {
    int32_t tile_m;      /* tile size for A (rows of Y); 0 = default 128.  Range [16, 256] */
    int32_t tile_n;      /* tile size for B (columns of Y); 0 = tile_m */
    int32_t precision;   /* enum trsyl_precision */
    int32_t scheduler;   /* enum trsyl_scheduler */
    int32_t slabs;       /* row slabs per tile update task; 0 = default (1: whole tiles) */
    int32_t max_sweeps;  /* refinement sweeps for TRSYL_FP32_REFINE; 0 = default 3, < 0 = none */
    double refine_tol;   /* TRSYL_FP32_REFINE: each sweep first evaluates eq. (9) (Sec. 3) of
                            the current (Y, alpha) on the device; once it is <= refine_tol the
                            remaining sweeps do nothing (no host synchronisation).
                            0 = default 1e-13 */
    int32_t workers;     /* persistent workgroups; 0 = one per compute unit */
    int32_t flags;       /* bit 0: force the robust (non-speculative) tile solve.
                            Grouping of the tile updates (Algorithm 3) into tasks, by default one
                            task per update; with slabs = 1 and
                            bit 2 (TRSYL_FLAG_PAIRED_UPDATES): the two updates of a tile whose
                            solved tiles lie on the same anti-diagonal front (which become ready
                            together) run as one two-term update -- one scale decision over both
                            terms (ProtectUpdate with the sum of the terms' bounds), one read and
                            write of the target; both schedulers group the same way, so their
                            results stay bitwise equal;
                            bit 3 (TRSYL_FLAG_DEFERRED_UPDATES): each tile takes all its pending
                            updates as one multi-term update (left-looking; at most 128 terms per
                            task), which reads and writes every target tile once -- in the
                            persistent scheduler; the per-front scheduler then pairs as bit 2. */
    void *profile_events; /* optional host pointer to two caller-owned hipEvent_t: the library
                             records [0] right before and [1] right after the tile-DAG kernel(s)
                             on `stream`, so their elapsed time is the scheduler's duration */
    uint64_t *trace;      /* optional device buffer of 4 * N uint64, N = pt qt + (updates) slabs
                             the length of the task list with one task per update (pt = ceil(m /
                             tile_m), qt = ceil(n / tile_n), updates = qt pt (pt-1)/2 +
                             pt qt (qt-1)/2): for task t of the persistent scheduler, [4t] = task
                             word, [4t+1] = start and [4t+2] = end (100 MHz wall clock), [4t+3] =
                             workgroup; records past the last task (grouped updates make the list
                             shorter) are left as they were */
    uint32_t *counters;   /* optional device buffer of 4 uint32, written on `stream` after the
                             solve: [0] tile solves that ran Algorithm 2 element by element
                             (both faster paths failed), [1] tile updates whose scale decision
                             rescaled the target or the solved tile (scaling events of
                             RobustUpdate, Algorithm 3), [2] tile solves whose unscaled
                             certificate failed, so that the leaf-tiled robust solve ran,
                             [3] TRSYL_FP32_REFINE: refinement sweeps that updated Y (the
                             others stopped at refine_tol); otherwise zero.
                             trsyl_robust, trsyl_robust_adjoint and trsyl_robust_general
                             fill it (for
                             TRSYL_FP32_REFINE: the counts of the first, FP32-update solve);
                             trsyl_robust_batched ignores it */
} trsyl_opts;

/* Fill *opts with the defaults. */
void trsyl_default_opts(trsyl_opts *opts);

/* Workspace bytes needed by trsyl_robust for an m x n problem with these options. */
size_t trsyl_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts);

/*
 * Robust solve of A Y + Y B = alpha C (Algorithm 4, Sec. 2.2): tiles of Y carry their own
 * power-of-two scales; tile solves follow RobustSyl (Algorithm 2), tile updates RobustUpdate
 * (Algorithm 3); the tiles are rescaled consistently to alpha = min alpha_kl at the end.
 *   m, n            orders of A and B (>= 0)
 *   A, lda          device, m x m, lda >= max(1, m), read only
 *   B, ldb          device, n x n, ldb >= max(1, n), read only
 *   C, ldc          device, m x n, ldc >= max(1, m); in: C, out: Y (||Y_kl||_inf <= OMEGA)
 *   scale_log2      device int64[1]: e with alpha = 2^-e
 *   scale           device double[1]: alpha (0.0 when e > 1074); may be NULL
 *   info            device int32[1]: status, see above
 *   opts            host; NULL = defaults
 *   workspace       device, ws_bytes >= trsyl_workspace_size(m, n, opts), 256-byte aligned
 */
int trsyl_robust(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
                 const trsyl_opts *opts, void *workspace, size_t ws_bytes, trsyl_stream_t stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation: trsyl_robust without a workspace argument.
 *   - The solver state lives in a device array of TRSYL_NOALLOC_BYTES (64 MiB) that the library
 *     holds on every GPU it runs on until the process ends; nothing is allocated or freed by the
 *     call (the first call on a device only looks up that device's copy of the array).
 *   - Arguments as for trsyl_robust, opts as well, except: precision must be TRSYL_FP64 (else -12),
 *     the scheduler is always the per-front one (opts->scheduler and opts->workers are ignored) and
 *     opts->trace is ignored.  Results are bit-identical to trsyl_robust's with the same tiles.
 *   - The state grows with the tile counts: about 8 min(p_t, q_t) 257^2 bytes of per-workgroup tiles
 *     plus small per-tile tables (m = n = 8192 with tile 128 uses ~34 MB).  A problem whose state
 *     exceeds TRSYL_NOALLOC_BYTES is rejected with TRSYL_ENOSPACE before anything is enqueued.
 *   - All calls on one GPU share the array and it keeps the last call's contents (each call clears
 *     the state it reads): calls that overlap on one GPU -- from several host threads or on several
 *     streams without ordering between them -- race and give undefined results.
 */
#define TRSYL_NOALLOC_BYTES (64u << 20)
#define TRSYL_ENOSPACE (-201)
int trsyl_robust_noalloc(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                         double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
                         const trsyl_opts *opts, trsyl_stream_t stream);

/*
 * Adjoint solve A^T G + G B^T = alpha W, used for gradients (L = <W, Y> gives dL/dC = alpha_Y G,
 * dL/dA = -G Y^T on A's pattern, dL/dB = -Y^T G).  Same arguments as trsyl_robust with W in C.
 * The transposed problem is mapped onto the forward one by order reversal:
 * P A^T P and Q B^T Q are upper quasi-triangular (P, Q reverse the index order), and
 * G = P Gh Q with (P A^T P) Gh + Gh (Q B^T Q) = alpha P W Q.
 */
size_t trsyl_adjoint_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts);
int trsyl_robust_adjoint(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                         int64_t ldb, double *W, int64_t ldw, int64_t *scale_log2, double *scale,
                         int32_t *info, const trsyl_opts *opts, void *workspace, size_t ws_bytes,
                         trsyl_stream_t stream);

/*
 * Host read-back of a solve's results (the exponent e with alpha = 2^-e, Sec. 2, and the status):
 * waits for `stream`, then copies *scale_log2, *info and, when scale_host is not NULL, *scale from
 * device memory into the host variables.
 *   scale_log2, scale, info           device pointers passed to the solve (scale may be NULL
 *                                     when scale_host is NULL)
 *   e_host, scale_host, info_host     host; scale_host may be NULL
 * Returns 0, -i for a NULL argument i, -100 on a HIP error.
 */
int trsyl_sync_result(const int64_t *scale_log2, const double *scale, const int32_t *info,
                      int64_t *e_host, double *scale_host, int32_t *info_host, trsyl_stream_t stream);

/*
 * General form op(A) Y + isgn Y op(B) = alpha C (the triangular Sylvester equation of Sec. 1 with
 * either coefficient transposed and either sign; with B = A and tranb = 'T' it is the Lyapunov
 * equation A Y + Y A^T = alpha C, which Sec. 1 names as a special case).
 *   trana, tranb    'N': op(X) = X;  'T' (or 'C'): op(X) = X^T
 *   isgn            +1 or -1
 *   other arguments as in trsyl_robust (argument i of this list is reported as -i); A and B are
 *   read only; workspace >= trsyl_general_workspace_size(m, n, opts).
 * A transposed coefficient is mapped onto the forward problem by order reversal as in
 * trsyl_robust_adjoint (P A^T P upper quasi-triangular, the rows of C reversed; Q B^T Q, the
 * columns of C reversed); isgn = -1 solves with -op(B).  'N', 'N', +1 is trsyl_robust.
 */
size_t trsyl_general_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts);
int trsyl_robust_general(char trana, char tranb, int32_t isgn, int64_t m, int64_t n, const double *A,
                         int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                         int64_t *scale_log2, double *scale, int32_t *info, const trsyl_opts *opts,
                         void *workspace, size_t ws_bytes, trsyl_stream_t stream);

/*
 * Bartels-Stewart solve of A X + X B = alpha C for general A, B (Sec. 1): the caller supplies
 * real Schur forms A = U At U^T, B = V Bt V^T (U, V orthogonal; At, Bt upper quasi-triangular,
 * e.g. from LAPACK dgees).  The library forms Ct = U^T C V, solves At Y + Y Bt = alpha Ct with
 * trsyl_robust, and returns X = U Y V^T in C.
 *   U, ldu / V, ldv     device, m x m / n x n, read only
 *   At, ldat / Bt, ldbt device, m x m / n x n, read only (as A, B of trsyl_robust)
 *   C, ldc              device, m x n; in: C, out: X
 *   other arguments as in trsyl_robust (argument i of this list is reported as -i);
 *   workspace >= trsyl_bartels_stewart_workspace_size(m, n, opts).
 * The four orthogonal transforms are FP64 GEMMs that cannot overflow: C, and then Y, enters its
 * first transform times the power of two that brings its Frobenius norm to OMEGA or below (every
 * partial sum of a transformed entry is bounded by that norm), and both shifts are added to e,
 * so X = 2^-e times the solution with e the total exponent.
 */
size_t trsyl_bartels_stewart_workspace_size(int64_t m, int64_t n, const trsyl_opts *opts);
int trsyl_bartels_stewart(int64_t m, int64_t n, const double *U, int64_t ldu, const double *At,
                          int64_t ldat, const double *V, int64_t ldv, const double *Bt, int64_t ldbt,
                          double *C, int64_t ldc, int64_t *scale_log2, double *scale, int32_t *info,
                          const trsyl_opts *opts, void *workspace, size_t ws_bytes,
                          trsyl_stream_t stream);

/*
 * Batched adjoint solve: `count` independent problems A_i^T G_i + G_i B_i^T = alpha_i W_i (the
 * transposed problems whose solutions give the gradients of a loss <W, Y>, an extension beyond the
 * paper), each reversed as in trsyl_robust_adjoint
 * and all solved by one batched forward solve (trsyl_robust_batched).  Arguments as in
 * trsyl_robust_batched, with W (in: W_i, out: G_i) in place of C; workspace >=
 * trsyl_adjoint_batched_workspace_size(count, m, n, tiles, opts).  A problem's results are
 * identical to trsyl_robust_adjoint's with the same tile sizes and options.
 */
size_t trsyl_adjoint_batched_workspace_size(int32_t count, const int64_t *m, const int64_t *n,
                                            const int32_t *tiles, const trsyl_opts *opts);
int trsyl_robust_adjoint_batched(int32_t count, const int64_t *m, const int64_t *n,
                                 const double *const *A, const int64_t *lda, const double *const *B,
                                 const int64_t *ldb, double *const *W, const int64_t *ldw,
                                 const int32_t *tiles, int64_t *scale_log2, double *scale,
                                 int32_t *info, const trsyl_opts *opts, void *workspace,
                                 size_t ws_bytes, trsyl_stream_t stream);

/*
 * Gradient products for L = <W, Y> with Y the scaled forward output (A Y + Y B = alpha_Y C,
 * alpha_Y = 2^-eY held fixed), given the adjoint output G with A^T G + G B^T = 2^-eG W:
 * with Gt = 2^eG G (the unscaled adjoint solution),
 *   dC = alpha_Y Gt,   dA = -Gt Y^T on A's quasi-triangular pattern,
 *   dB = -Y^T Gt on B's pattern (upper triangle plus the subdiagonal entries of 2x2 blocks).
 * eY and eG are read from device memory.  dA (ld ldda), dB (ld lddb), dC (ld lddc) are device
 * outputs and must not alias the inputs.  Needs no workspace.
 */
int trsyl_grad(int64_t m, int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
               const double *Y, int64_t ldy, const int64_t *eY, const double *G, int64_t ldg,
               const int64_t *eG, double *dA, int64_t ldda, double *dB, int64_t lddb, double *dC,
               int64_t lddc, trsyl_stream_t stream);

/*
 * Batched robust solve: `count` independent problems of arbitrary sizes (rectangular allowed) in
 * one launch per stage -- structure, bounds, one persistent tile-DAG kernel over the merged task
 * lists of all problems, finalisation and consistency scaling (Algorithm 4 per problem).  With
 * opts->precision = TRSYL_FP32_REFINE the batch runs the precision form: one batched solve with
 * FP32-MFMA tile updates, then opts->max_sweeps sweeps that form each problem's FP64 residual,
 * solve all corrections in one batched solve and update every problem.
 *   m, n, lda, ldb, ldc   host arrays [count]
 *   A, B, C               host arrays [count] of device pointers (as in trsyl_robust)
 *   tiles                 host array [2 * count] of (tile_m, tile_n) per problem, e.g. from an
 *                         autotuner; NULL = opts->tile_m / tile_n for every problem
 *   scale_log2, scale, info   device arrays [count] (scale may be NULL)
 *   workspace             >= trsyl_batched_workspace_size(count, m, n, tiles, opts), 256-aligned
 * A problem's results are identical to trsyl_robust's with the same tile sizes and options.  The
 * return value
 * is the host argument check only (negative: argument index); per-problem status goes to info[i].
 */
size_t trsyl_batched_workspace_size(int32_t count, const int64_t *m, const int64_t *n,
                                    const int32_t *tiles, const trsyl_opts *opts);
int trsyl_robust_batched(int32_t count, const int64_t *m, const int64_t *n,
                         const double *const *A, const int64_t *lda, const double *const *B,
                         const int64_t *ldb, double *const *C, const int64_t *ldc,
                         const int32_t *tiles, int64_t *scale_log2, double *scale, int32_t *info,
                         const trsyl_opts *opts, void *workspace, size_t ws_bytes,
                         trsyl_stream_t stream);

/*
 * Relative residual of eq. (9), evaluated on the device in FP64 with power-of-two
 * normalisation:  ||alpha C - (A Y + Y B)||_F / ((||A||_F + ||B||_F) ||Y||_F + ||alpha C||_F),
 * alpha = 2^-e read from device memory.  Writes the quotient to *out (device double).
 * workspace >= trsyl_residual_workspace_size(m, n).
 */
size_t trsyl_residual_workspace_size(int64_t m, int64_t n);
int trsyl_residual(int64_t m, int64_t n, const double *A, int64_t lda, const double *B,
                   int64_t ldb, const double *Y, int64_t ldy, const int64_t *e, const double *C,
                   int64_t ldc, double *out, void *workspace, size_t ws_bytes,
                   trsyl_stream_t stream);

/*
 * Diagnostics: evaluate the device versions of ProtectUpdate / ProtectDivision (Sec. 2.1) on
 * `count` argument triples/pairs.  in: device double[3*count] (c, a, y) or double[2*count]
 * (b, t); out: device int32[count] exponents s (zeta = 2^-s).
 */
int trsyl_debug_protect_update(int32_t count, const double *in, int32_t *out, trsyl_stream_t stream);
int trsyl_debug_protect_division(int32_t count, const double *in, int32_t *out, trsyl_stream_t stream);

/*
 * Diagnostics, host only (no device call): the static task order the persistent scheduler
 * follows for a grid of pt x qt tiles (tile sizes tile_m x tile_n, `slabs` row slabs per update,
 * `workers` workgroups, option flags as in trsyl_opts), written to out[0 .. cap) as task words:
 * bits 0..1 kind (0 solve, 1 column update, 2 row update, 3 multi-term update), 2..7 slab,
 * 8..27 target tile i * qt + l, 28..47 source tile (multi-term: number of terms g), 48..63 the
 * update's position in the target's order (multi-term: the first of its g positions).  Returns
 * the number of tasks (which may exceed cap; only cap are written), or a negative argument index.
 */
int64_t trsyl_debug_task_order(int32_t pt, int32_t qt, int32_t tile_m, int32_t tile_n, int32_t slabs,
                               int32_t workers, int32_t flags, uint64_t *out, int64_t cap);

/* Library version string. */
const char *trsyl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TRSYL_H */
