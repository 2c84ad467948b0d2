/*
 * tileqr: tiled Householder QR factorisation on AMD Instinct MI355X (gfx950).
 *
 * The operation is the tiled QR of Buttari, Langou, Kurzak and Dongarra,
 * "A Class of Parallel Tiled Linear Algebra Algorithms for Multicore
 * Architectures", Section 3.2.1 (Algorithm 2): A (m x n) is cut into b x b
 * tiles (b = nb) and factored as A = QR by four tile kernels,
 *   GEQRT  A_kk -> (V_kk, R_kk, T_kk)              QR of a diagonal tile,
 *   LARFB  A_kj <- Q_kk^T A_kj                     its block reflector applied
 *                                                  along tile row k,
 *   TSQRT  [R_kk; A_ik] -> (R_kk, V_ik, T_ik)      QR of a triangle on top of
 *                                                  a square tile,
 *   SSRFB  [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij]     that reflector applied to
 *                                                  the pairs of tiles beside,
 * each accumulating its reflectors in groups of s = ib (inner blocking,
 * Section 3.2.3).  The tasks run as a dependency DAG (Section 4) that a
 * persistent GPU kernel schedules; Q is kept as tile reflectors V plus the
 * triangular T factors of the compact WY form (Section 3.2.1), never formed.
 *
 * Conventions for every entry point:
 *  - Matrix pointers (A, T, B, X) are DEVICE pointers (hipMalloc, or a torch
 *    CUDA tensor's data_ptr), column-major with the given leading dimension,
 *    FP64.  Size arguments and the option/info structs live in host memory.
 *  - The caller allocates and frees A, T, B and X; the library never frees
 *    caller memory.  The library owns its workspace (tile buffer, dependency
 *    counters, ready queues), allocates it lazily on the device current at
 *    the call and keeps it until tileqr_finalize().
 *  - Calls are synchronous: they return once the device work has finished
 *    (so that a device-side status can be reported), unless
 *    TILEQR_FLAG_ASYNC is set.  Work runs on opts->stream (NULL: the null
 *    stream).
 *  - Return value: TILEQR_OK (0) on success; -i when argument i (1-based) is
 *    invalid, in which case nothing is touched (LAPACK INFO style); a
 *    positive tileqr_status otherwise.  A dimension of zero returns 0 at once.
 *  - Each (device, stream) pair gets a workspace of its own, so calls with
 *    TILEQR_FLAG_ASYNC on different streams may overlap on the device.
 *    Calls from several host threads are serialised by a library lock.
 */
#ifndef TILEQR_H
#define TILEQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TILEQR_OK = 0,
    TILEQR_EHIP = 1,        /* a HIP runtime call failed (see tileqr_last_hip_error) */
    TILEQR_ENONFINITE = 2,  /* A holds a NaN or an infinity: nothing factored      */
    TILEQR_ENOCONV = 3,     /* refinement stopped above tol (best iterate returned) */
    TILEQR_ETIMEOUT = 4,    /* scheduler watchdog: no task became ready in time     */
    TILEQR_ENOMEM = 5,      /* workspace allocation failed                          */
    TILEQR_EUNSUPPORTED = 6,/* a valid but unsupported combination (see nb/ib rules)*/
    TILEQR_ESINGULAR = 7,   /* R has an exact zero on its diagonal (solve only)     */
    TILEQR_ENOTSPD = 8      /* tilechol: a leading minor is not positive definite   */
} tileqr_status;

/* Arithmetic of the block-reflector products: LARFB, SSRFB and the updates
 * of the remaining panel columns inside GEQRT and TSQRT.  Reflector
 * generation (norms, tau, beta = the R diagonal) and T, storage, the update
 * of the coupled R rows and the refinement's residuals stay FP64 in every
 * mode.  In a split mode each FP64 operand of the products V^T X and V W is
 * written as a sum of 2 or 3 narrow numbers (x rounded, then the rounded
 * remainders) and the kept partial products run on the narrow MFMAs with
 * FP32 accumulation per 32 rows, summed across rows in FP64.  Split modes
 * take ib = 32 (any supported nb); other ib give TILEQR_EUNSUPPORTED.
 * Entries must stay below about 1e38 in magnitude in the BF16 modes (FP32
 * range); FP16X2 scales every operand column by a power of two. */
typedef enum {
    TILEQR_FP64 = 0,    /* FP64 MFMA                                               */
    TILEQR_BF16X2 = 1,  /* hi+lo BF16 split, 3 products, FP32 accumulation         */
    TILEQR_FP16X2 = 2,  /* hi+lo FP16 split with power-of-two scaling, 3 products  */
    TILEQR_BF16X3 = 3   /* hi+mid+lo BF16 split, 6 products, FP32 accumulation     */
} tileqr_precision;

enum {
    TILEQR_FLAG_ASYNC = 1u << 0,   /* return without synchronising the stream          */
    TILEQR_FLAG_SERIAL = 1u << 1,  /* run the tasks one launch each in Algorithm 2's
                                      loop order instead of the DAG scheduler          */
    TILEQR_FLAG_TRACE = 1u << 2,   /* record one trace event per task (tileqr_trace)   */
    TILEQR_FLAG_SHUFFLE = 1u << 3, /* DAG scheduler pops ready tasks in a seeded
                                      pseudo-random order (schedule-independence test) */
    TILEQR_FLAG_TIMING = 1u << 4,  /* time each stage with HIP events on the call's
                                      stream (tileqr_last_timing)                      */
    TILEQR_FLAG_NO_GRAPH = 1u << 5,/* tileqr_factor_batched: launch the kernels directly
                                      instead of replaying a captured HIP graph        */
    TILEQR_FLAG_CHECK = 1u << 6    /* tileqr_solve_ls: also estimate the factorisation's
                                      backward error (tileqr_info.beta_fact_est)       */
};

typedef struct {
    int precision;        /* tileqr_precision                                        */
    int64_t nb, ib;       /* tile size b and inner block s; 0 = pick automatically   */
    int max_iter;         /* refinement iterations in tileqr_solve_ls (<= 64)        */
    double tol;           /* refinement target for the backward error                */
    void *stream;         /* hipStream_t; NULL = null stream                         */
    unsigned flags;       /* TILEQR_FLAG_*                                           */
    uint64_t seed;        /* seed of TILEQR_FLAG_SHUFFLE                             */
    int64_t spin_limit;   /* scheduler watchdog: idle polls without progress before
                             TILEQR_ETIMEOUT; 0 = default (several seconds)          */
    int64_t workers;      /* update-worker workgroups of the DAG scheduler; 0 = as many
                             as fit beside the panel worker                          */
    int64_t drop_edge;    /* test hook for the watchdog: the task with this id skips
                             its first successor release; -1 (default) = none        */
    int64_t panel_workers;/* panel-role workgroups of the DAG scheduler (GEQRT, TSQRT);
                             0 = automatic: in proportion to the panel flops for a
                             batch, and for one matrix split into panel tasks (at
                             least 16, at most nb/ib per tile step); one matrix
                             with whole tile kernels: 16 with up to 32 tile
                             steps, else 8                                         */
    int64_t panel_tasks;  /* DAG tasks per GEQRT and TSQRT: 1 (the whole tile
                             kernel) or nb / ib (one per inner panel, which lets
                             the panel chains of a step overlap; with ib = 32
                             each panel's update of every later strip of its
                             tile is then a task of its own); 0 = automatic
                             (one matrix with at most 32 tile steps: nb / ib,
                             otherwise 1)                                           */
    int64_t apply_group;  /* inner panels per workgroup when tileqr_solve_ls applies
                             Q or Q^T: 1, 2, 4 or 8, dividing nb / ib; 0 =
                             automatic (larger for matrices with many tile steps
                             per row block).  The result does not depend on it */
} tileqr_opts;

/* Blocking and schedule of a factorisation, as chosen by tileqr_tune. */
typedef struct {
    int64_t nb, ib;           /* tile size and inner block                           */
    int64_t panel_workers;    /* tileqr_opts.panel_workers                           */
    int64_t workers;          /* tileqr_opts.workers (update workgroups)             */
    double ms;                /* device time of the best trial                       */
} tileqr_tuning;

typedef struct {
    int iterations;       /* refinement steps taken                                  */
    int converged;        /* 1 if the backward error reached tol                     */
    double eta;           /* stopping measure of the returned X (see tileqr_solve_ls):
                             eta_ls, and for m == n the larger of eta_ls, eta_inf    */
    double eta_hist[65];  /* the stopping measure after 0, 1, ... iterations         */
    int64_t nb, ib;       /* blocking used                                           */
    double ms_factor;     /* device time of the factorisation                        */
    double ms_total;      /* device time of the whole call                           */
    double eta_ls;        /* ||A^T (B - A X)||_2 / (||A||_F (||A||_F ||X||_2 +
                             ||B||_2)) of the returned X, worst column               */
    double eta_inf;       /* m == n: ||B - A X||_inf / (||A||_inf ||X||_inf) of the
                             returned X, worst column (the solution backward error
                             of Section 3.2.4); 0 for m > n                          */
    double beta_fact_est; /* with TILEQR_FLAG_CHECK: ||A - Q [R; 0]||_F / ||A||_F
                             estimated from `probes` Gaussian probe vectors z
                             (E ||E z||^2 = ||E||_F^2), else -1                      */
    int probes;           /* probe vectors behind beta_fact_est                      */
    double ms_worker;     /* device time of the factorisation kernel(s) alone
                             (within ms_factor, which adds the layout conversion
                             and the scheduler set-up)                             */
} tileqr_info;

/* Fill *opts with the defaults: FP64, automatic nb/ib, max_iter 30,
 * tol 1e-14, null stream, no flags, drop_edge -1. */
void tileqr_opts_default(tileqr_opts *opts);

/* Supported blockings: nb in {64, 128, 256} and ib in {16, 32} (so nb % ib
 * == 0: the paper takes b/s integral, Section 3.2.3).  Returns 1 if (nb, ib)
 * is supported, else 0. */
int tileqr_blocking_supported(int64_t nb, int64_t ib);

/* Blocking the library picks for an m x n factorisation in the given
 * precision when nb = ib = 0 (ib = 32 in the split modes).  Writes nb and
 * ib; returns 0. */
int tileqr_choose_blocking(int64_t m, int64_t n, int precision, int64_t *nb, int64_t *ib);

/* Number of doubles the T factors of an m x n factorisation occupy:
 * one ib x nb block (nb/ib upper-triangular ib x ib blocks, Section 3.2.3)
 * per tile (i, k) with k < min(p, q), k <= i < p, where p = ceil(m/nb),
 * q = ceil(n/nb).  0 for an empty matrix or unsupported blocking. */
size_t tileqr_t_size(int64_t m, int64_t n, int64_t nb, int64_t ib);

/*
 * Factor A = QR in place (Section 3.2.1, Algorithm 2; reflector sign
 * beta = -sign(alpha) ||x|| with sign(0) = +1, tau = 0 when the column below
 * the diagonal is already zero).
 *   m, n   >= 0 (m < n allowed: min(p, q) tile steps)
 *   A      device, m x n, leading dimension lda >= max(1, m); overwritten by
 *          R (upper triangle of rows 0..min(m,n)-1) and the tile reflectors:
 *          V_kk in the strict lower triangle of each diagonal tile, V_ik
 *          (i > k) filling the tiles below it.  This is the tiled layout of
 *          the paper (Section 3.2.1), not LAPACK's: use Q only through
 *          tileqr_apply_q / tileqr_apply_qt with the same nb, ib and T.
 *   nb, ib blocking (see tileqr_blocking_supported); 0, 0 = automatic is not
 *          allowed here because T is sized by the caller
 *   T      device, >= tileqr_t_size(m, n, nb, ib) doubles, written; its
 *          internal layout is private to the library.
 * Errors: -1 m, -2 n, -3 A (NULL with m, n > 0), -4 lda, -5 nb, -6 ib,
 *         -7 T; TILEQR_ENONFINITE if A holds NaN/Inf (A then unchanged).
 */
int tileqr_factor(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib,
                  double *T);

/* tileqr_factor with options (schedule, stream, flags, precision of the
 * two GEMM-shaped kernels).  opts may be NULL (defaults); opts->nb/ib are
 * ignored (the explicit arguments rule).  Argument 8 is opts (-8 for an
 * unknown precision); TILEQR_EUNSUPPORTED for a split precision with
 * ib != 32. */
int tileqr_factor_ex(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib,
                     double *T, const tileqr_opts *opts);

/* Size of the fixed device array tileqr_factor_noalloc takes its workspace
 * from (64 MiB per device, held from the library's load to the end of the
 * process). */
#define TILEQR_NOALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels, schedule and result (bit for bit) as tileqr_factor_ex,
 * but no hipMalloc, hipFree or other allocating call is made: the tile
 * workspace, the status word, the scheduler's counters and queues and (split
 * precisions) the split images of V and T are carved from one fixed device
 * array of TILEQR_NOALLOC_SCRATCH_BYTES per device.  A shape whose workspace
 * does not fit (p q nb^2 doubles of tiles, 4 bytes per task id and per task,
 * the split images) returns TILEQR_ENOMEM before anything is launched, A
 * untouched; every shape up to 2048 x 2048 fits at each supported blocking
 * and precision.  TILEQR_FLAG_TRACE and TILEQR_FLAG_TIMING are not supported
 * here (TILEQR_EUNSUPPORTED).  The array is shared by every call on the
 * device and keeps the last call's contents (each call clears what must
 * start at zero): calls that overlap on one device (TILEQR_FLAG_ASYNC calls
 * on two streams, or from two host threads) race and must not be issued.
 */
int tileqr_factor_noalloc(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib,
                          double *T, const tileqr_opts *opts);

/*
 * B := Q^T B (tileqr_apply_qt) or B := Q B (tileqr_apply_q) for Q of a
 * previous tileqr_factor(m, n, A, lda, nb, ib, T).  Q^T applies, for each
 * tile step k in ascending order, the diagonal reflector (as LARFB does) and
 * then the coupled reflectors of tiles i = k+1.. in ascending order (as SSRFB
 * does); Q applies the same operators transposed in reverse order.
 *   nrhs >= 0; B device, m x nrhs, ldb >= max(1, m), overwritten.
 * Errors: -1 m, -2 n, -3 nrhs, -4 A, -5 lda, -6 nb, -7 ib, -8 T, -9 B, -10 ldb.
 */
int tileqr_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                    int64_t nb, int64_t ib, const double *T, double *B, int64_t ldb);
int tileqr_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                   int64_t nb, int64_t ib, const double *T, double *B, int64_t ldb);

/*
 * Least squares X = argmin ||B - A X||_2 for m >= n and A of full column
 * rank, one column per right-hand side.  A and B are left untouched (the
 * library factors a copy).  The solution is first R^{-1} (Q^T B)(0:n); then,
 * as Section 3.2.4 advises (check the backward error of a solve, refine
 * when needed), it is refined in FP64 on the original A until the stopping
 * measure is <= opts->tol, stagnates (two steps that fail to halve it), or
 * max_iter steps are taken; the best iterate is returned.  The stopping
 * measure is eta_ls = ||A^T (B - A X)||_2 / (||A||_F (||A||_F ||X||_2 +
 * ||B||_2)) (worst column); for m == n it is the larger of eta_ls and the
 * paper's eta_inf = ||B - A X||_inf / (||A||_inf ||X||_inf).  Refinement for
 * m > n is on the augmented system (residuals f = B - R - A X and
 * g = -A^T R in FP64, corrections through the factors); for m == n, whose
 * least-squares residual is zero, it is classical refinement
 * dX = R^{-1} Q^T (B - A X).  With a split precision the factorisation's
 * block-reflector products run in that arithmetic and the refinement wins
 * back the FP64 backward error; with TILEQR_FP64 the first solution
 * normally meets tol already.  With TILEQR_FLAG_CHECK the factorisation's
 * backward error is estimated from Gaussian probes (info->beta_fact_est);
 * its cost is outside ms_factor but inside ms_total.
 *   X device, n x nrhs, ldx >= max(1, n), written.  info may be NULL.
 * Errors: -1 m, -2 n (n > m), -3 nrhs, -4 A, -5 lda, -6 B, -7 ldb, -8 X,
 *         -9 ldx, -10 opts; TILEQR_ENOCONV (best iterate in X) when the
 *         refinement does not reach tol; TILEQR_ESINGULAR for a zero R_jj.
 */
int tileqr_solve_ls(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *X, int64_t ldx,
                    const tileqr_opts *opts, tileqr_info *info);

/*
 * Factor `batch` independent matrices in one persistent launch: one global
 * task space over all of them (Section 4's DAG, one per matrix).
 *   m, n, lda, nb, ib : host arrays of `batch` entries (nb/ib may be NULL:
 *                       tileqr_choose_blocking per matrix)
 *   A, T              : host arrays of `batch` device pointers; T[i] holds
 *                       tileqr_t_size(m[i], n[i], nb[i], ib[i]) doubles.
 * Each result equals, bit for bit, tileqr_factor on that matrix alone with
 * the same nb, ib and precision.  Matrices with different (nb, ib) form
 * groups, one persistent launch each (nb = ib = NULL: one (nb, ib) for the
 * whole batch, tileqr_tune's if it has seen these shapes, else by size).
 * The launch sequence (layout conversion, scheduler set-up, workers,
 * conversion back) is captured into a HIP graph on first use and replayed
 * while the shapes, blocking and options stay the same; the matrix and T
 * pointers are read from device memory at run time, so new pointers need no
 * new capture.  opts->stream orders the call; TILEQR_FLAG_ASYNC returns
 * without waiting (status then unchecked), TILEQR_FLAG_NO_GRAPH launches
 * directly, TILEQR_FLAG_SERIAL and TILEQR_FLAG_TRACE are not supported here
 * (TILEQR_EUNSUPPORTED).  With NaN/Inf in any matrix no matrix is written
 * (TILEQR_ENONFINITE).
 * Errors: -1 batch, -2 m, -3 n, -4 A, -5 lda, -6 nb, -7 ib, -8 T, -9 opts
 * (for an array argument: the first bad entry).
 */
int tileqr_factor_batched(int64_t batch, const int64_t *m, const int64_t *n,
                          double *const *A, const int64_t *lda, const int64_t *nb,
                          const int64_t *ib, double *const *T, const tileqr_opts *opts);

/*
 * Tree reduction of the panels of a tall matrix (m >= n), an extension of
 * Section 3.2.1's Algorithm 2, whose flat chain of TSQRT makes the panel of
 * every step a chain of ceil(m / nb) tasks.  The rows are cut into `leaves`
 * row blocks of h rows (h the largest multiple of nb with leaves * h <= m;
 * the last block takes the rest; every block needs at least max(n, nb)
 * rows); each block is factored by Algorithm 2 (all blocks in one
 * tileqr_factor_batched launch, one task per inner panel unless
 * opts->panel_tasks says otherwise, a quarter of the CUs on the panels
 * unless opts->panel_workers says otherwise), then the blocks' triangles R
 * are merged level by level, up to four at a time, by the QR of the stack
 * [R_1; ...; R_k] (kn x n) with the same tile kernels (the merges of a level
 * in one batched launch; a lone block passes up unchanged).
 *   A (m x n, lda >= m): on return R in the upper triangle of rows 0..n-1;
 *     below the diagonal of every block's first rows its reflectors (the
 *     other blocks' first n rows hold their own R, used by the merges).
 *   F (device, tileqr_tree_size doubles): the blocks' T factors, then every
 *     merge's stacked matrix (leading dimension kn) and T.
 *   opts: FP64 only; stream (the call returns with its work done); the
 *     scheduler options apply to the batched launches.
 * Q^T B and Q B (B m x nrhs, ldb >= m) follow the same order: each block's
 * Q^T on its rows, then each merge's on the first n rows of its blocks (the
 * leftmost block of a merged group carries the group).  (Q^T B)(0:n) is
 * in B's first n rows, as with tileqr_apply_qt.
 * tileqr_solve_ls_tree: X (n x nrhs, ldx >= n) = R^{-1} (Q^T B)(0:n), the
 * FP64 least-squares solution, from copies of A and B; *ms (may be NULL)
 * gets the device time of the call.
 * tileqr_tree_size returns 0 for impossible arguments.  Errors as
 * tileqr_factor_ex; -7 leaves (a block would be too short) for the factor,
 * -8 for the applies, -12 for the solve; TILEQR_EUNSUPPORTED for a split
 * precision, TILEQR_FLAG_SERIAL or TILEQR_FLAG_TRACE.
 */
size_t tileqr_tree_size(int64_t m, int64_t n, int64_t nb, int64_t ib, int64_t leaves);
int tileqr_factor_tree(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib, int64_t leaves,
                       double *F, const tileqr_opts *opts);
int tileqr_apply_qt_tree(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb, int64_t ib,
                         int64_t leaves, const double *F, double *B, int64_t ldb);
int tileqr_apply_q_tree(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb, int64_t ib,
                        int64_t leaves, const double *F, double *B, int64_t ldb);
int tileqr_solve_ls_tree(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                         int64_t ldb, double *X, int64_t ldx, int64_t nb, int64_t ib, int64_t leaves,
                         const tileqr_opts *opts, double *ms);

/* Outcome of a tileqr_solve_ls_batched call. */
typedef struct {
    int64_t converged;      /* matrices whose backward error reached tol         */
    int64_t not_converged;  /* matrices returned with their best iterate         */
    int max_iterations;     /* most refinement steps any matrix took             */
    double max_eta;         /* largest backward error over the batch             */
    double ms_factor;       /* device time of the batched factorisation          */
    double ms_total;        /* device time of the whole call                     */
} tileqr_batch_info;

/*
 * Least squares for `batch` independent systems min ||b_i - A_i x_i||_2,
 * one right-hand side each (m_i >= n_i), the batched counterpart of
 * tileqr_solve_ls: the matrices are factored together as in
 * tileqr_factor_batched (a copy in the library's tiles; A_i and b_i are not
 * written), in opts->precision, then one workgroup per matrix forms
 * (Q^T b)(0:n), solves with R and refines with FP64 residuals on A_i
 * (Bjorck's augmented-system refinement for m > n, classical refinement for
 * m == n) until its own backward error (eta_ls, and for m == n the larger of
 * eta_ls and eta_inf, as in tileqr_solve_ls) is <= opts->tol, for at most
 * opts->max_iter steps, stopping early after two steps that do not halve it
 * (Section 3.2.4 advises checking the backward error and refining).
 *   m, n, lda      : host arrays of `batch` entries (n_i = 0: nothing done)
 *   A, b, x        : host arrays of `batch` device pointers; A_i column-major
 *                    m_i x n_i, b_i m_i entries, x_i n_i entries (written:
 *                    the iterate with the smallest backward error)
 *   opts           : precision, tol, max_iter, stream; opts->nb and ib both
 *                    0 (the tuner's or the default blocking for the batch)
 *                    or a blocking used for every matrix
 *   eta, iterations: optional HOST arrays of `batch` entries receiving each
 *                    matrix's backward error and refinement steps
 *   info           : optional summary (synchronous call)
 * Returns TILEQR_ENOCONV if some matrix stayed above tol (its best iterate is
 * in x_i), TILEQR_ESINGULAR for an exact zero on some R's diagonal,
 * TILEQR_ENONFINITE for NaN/Inf in some A_i (nothing solved).
 * Errors: -1 batch, -2 m, -3 n (n > m), -4 A, -5 lda, -6 b, -7 x, -8 opts
 * (TILEQR_FLAG_ASYNC, _SERIAL and _TRACE give TILEQR_EUNSUPPORTED).
 */
int tileqr_solve_ls_batched(int64_t batch, const int64_t *m, const int64_t *n,
                            const double *const *A, const int64_t *lda, const double *const *b,
                            double *const *x, const tileqr_opts *opts, double *eta,
                            int32_t *iterations, tileqr_batch_info *info);

/*
 * Autotuner: times trial factorisations of synthetic matrices with the given
 * shapes (batch >= 1; batch = 1 tunes one m x n matrix) in the given
 * precision on the current device, over every supported (nb, ib) and a few
 * splits of the workgroups between the panel and update roles, one untimed
 * warm-up run and then `trials` timed runs each (best time counts).  The
 * fastest choice is written to *best and
 * remembered in the tuner's table, keyed by the device's architecture and
 * compute-unit count, the precision and the multiset of shapes, for the rest
 * of the process (or longer, with tileqr_tune_save): tileqr_factor_batched
 * with nb = ib = NULL and tileqr_solve_ls / tileqr_choose_blocking with
 * automatic blocking use it, for exactly these shapes and, failing that, for
 * shapes of the same size class: the same precision and the same ceil(log2)
 * of the batch size, of the flop-weighted typical min(m, n) and of the
 * largest m and n (the paper tunes b and s per problem size, Section 5).
 * Allocates scratch device memory for the trial matrices (freed before
 * returning).
 * Errors: -1 batch, -2 m, -3 n, -4 precision, -5 trials, -6 best.
 */
int tileqr_tune(int64_t batch, const int64_t *m, const int64_t *n, int precision, int trials,
                tileqr_tuning *best);

/*
 * The tuner's table on disk: tileqr_tune_save writes every entry (of any
 * device kind) to the text file `path`, one line each; tileqr_tune_load adds
 * the entries of such a file to the table (replacing entries with the same
 * device kind and shapes).  Host only; no device is needed.  Return the
 * number of entries written / read, or -1 (path NULL), -2 (the file cannot
 * be opened or written), -3 (tileqr_tune_load: a malformed line; nothing is
 * loaded).
 */
int64_t tileqr_tune_save(const char *path);
int64_t tileqr_tune_load(const char *path);

/*
 * Query the table as the automatic blocking does, for a device of
 * architecture `arch` (e.g. "gfx950") with `cu` compute units: 1 and *out
 * set if an entry for exactly these shapes or for their size class exists,
 * else 0.  Host only.  Errors: -1 arch, -3 batch, -4 m, -5 n, -6 precision,
 * -7 out.
 */
int tileqr_tune_lookup(const char *arch, int cu, int64_t batch, const int64_t *m, const int64_t *n,
                       int precision, tileqr_tuning *out);

/* Empty the tuner's table. */
void tileqr_tune_clear(void);

/* Operation counts.  tileqr_flops_lapack: 2mn^2 - 2n^3/3 (m >= n; the
 * mirror formula for m < n), the count the paper reports rates with
 * (Section 5).  tileqr_flops_tiled: the tiled algorithm's own count from
 * its per-kernel costs (Section 3.2.3), which exceeds it by about s/(4b). */
double tileqr_flops_lapack(int64_t m, int64_t n);
double tileqr_flops_tiled(int64_t m, int64_t n, int64_t nb, int64_t ib);

/* Tasks of the DAG (Section 4) for a p x q tile grid with `strips` column
 * strips per tile (LARFB and SSRFB split by columns) and `panels` inner
 * panels per tile (GEQRT and TSQRT split into their ib-column panels; the
 * scheduler uses strips = nb / 32, panels = nb / ib; strips = panels = 1:
 * the paper's tasks).  With panels == strips > 1 (ib = 32) the panel tasks
 * only factor their panel and each later strip of the tile (or tile pair)
 * gets the panel's reflector in a task of its own, PUPD.  counts[0..4]
 * receive the numbers of GEQRT, TSQRT, LARFB, SSRFB and PUPD tasks;
 * returns their sum.  Host only, no GPU needed. */
int64_t tileqr_dag_counts(int64_t p, int64_t q, int64_t strips, int64_t panels, int64_t counts[5]);

/* Host-side check of the dependency rules the scheduler uses: executes the
 * DAG of a p x q grid (strips and panels as for tileqr_dag_counts) in
 * `trials` random topological orders (seeded) on a
 * symbolic tile-version model and checks that every task sees each tile in
 * the state Algorithm 2's loop order would give it.  Also checks that
 * in-degrees equal the number of predecessors that release each task.
 * Also checks that the per-queue task counts the scheduler derives by index
 * ranges equal the tasks each ready queue receives.  Returns 0 if all pass,
 * else the 1-based number of the failing trial (trials + 1 for a queue count
 * mismatch).  Host only. */
int tileqr_dag_selfcheck(int64_t p, int64_t q, int64_t strips, int64_t panels, int64_t trials, uint64_t seed);

/* Trace of the last factorisation run with TILEQR_FLAG_TRACE: up to `cap`
 * events copied to host memory, 10 int64 each: {type, k, i, j, strip (the
 * inner panel for GEQRT and TSQRT),
 * worker, t_pop, t_start, t_body_end, t_end} (types 0 GEQRT, 1 TSQRT,
 * 2 LARFB, 3 SSRFB, 4 PUPD, whose j field holds its inner panel;
 * worker = (role << 16) | workgroup; times in ticks of
 * the device wall clock, tileqr_trace_clock_hz per second: when the task
 * was taken from its queue, when its body started after the acquire fence,
 * when the body ended, and when the release fence and the successor
 * updates were done).  Returns the number of events available. */
int64_t tileqr_trace(int64_t *events, int64_t cap);
double tileqr_trace_clock_hz(void);

/* Device times in milliseconds of the stages of the last tileqr_factor_ex
 * call made with TILEQR_FLAG_TIMING (synchronous): ms[0] layout conversion
 * in, ms[1] scheduler set-up, ms[2] the factorisation kernel(s) (the
 * persistent worker, or all launches of the serial driver), ms[3] layout
 * conversion out.  Returns 0, or TILEQR_EUNSUPPORTED if no timed call ran. */
int tileqr_last_timing(double ms[4]);

/* Measured matrix-core peak of the current device, a diagnostic for
 * reading the factorisation's rates (the rates of Section 5 are quoted
 * against the machine's peak): a full-chip launch in which every wave
 * issues long chains of independent MFMAs of one kind, timed with HIP
 * events (best of three after a warm-up).  kind 0: FP64 16x16x4 (the FP64
 * products); 1: BF16 16x16x32 and 2: FP16 16x16x32 with FP32 accumulation
 * (the split products).  Writes TFLOP/s (2 flops per multiply-add) to
 * *tflops.  Errors: -1 kind, -2 tflops. */
int tileqr_mfma_peak(int kind, double *tflops);

const char *tileqr_status_string(int status);
const char *tileqr_last_hip_error(void);

/* Release the library workspace on every device it was allocated on. */
int tileqr_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* TILEQR_H */
