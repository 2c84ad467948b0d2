/*
 * tilechol: tiled Cholesky factorisation A = L L^T of a symmetric positive
 * definite matrix on one AMD Instinct MI355X (gfx950), the first of the three
 * tiled algorithms of Buttari, Langou, Kurzak and Dongarra, "A Class of
 * Parallel Tiled Linear Algebra Algorithms for Multicore Architectures":
 * Section 3.1, Algorithm 1.  The lower triangle is cut into nb x nb tiles;
 * the factorisation is the DAG of three kernels, scheduled dynamically
 * (Section 4) by a persistent GPU kernel:
 *   POTF2(k)      A_kk -> L_kk, the Cholesky factor of the diagonal tile;
 *   TRSM(k, i)    L_ik = A_ik L_kk^{-T}, i > k;
 *   GSMM(k, i, j) A_ij <- A_ij - L_ik L_jk^T, k < j <= i (on a diagonal
 *                 tile only its lower triangle).
 * L overwrites the lower triangle of A; the strict upper triangle is neither
 * read nor written (the paper stores L in place of the tiles of A).
 *
 * Shares the status codes, the options structure and the library (and its
 * workspace) with tileqr.h.  All matrix pointers are DEVICE pointers,
 * column-major FP64.
 */
#ifndef TILECHOL_H
#define TILECHOL_H

#include <stddef.h>
#include <stdint.h>

#include "tileqr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t minor;        /* TILEQR_ENOTSPD: the order (1-based) of the first
                             leading minor found not positive definite (its
                             pivot was not a positive number, or was NaN);
                             else 0                                             */
    int64_t nb;           /* tile size used                                     */
    double ms_factor;     /* device time of the call (layout in, scheduler
                             set-up, factorisation, layout out)                 */
    double ms_worker;     /* device time of the factorisation kernel alone      */
} tilechol_info;

/*
 * L L^T = A for the n x n symmetric positive definite matrix whose lower
 * triangle is in A (leading dimension lda >= max(1, n)); L overwrites that
 * lower triangle.  nb: 64 or 128, or 0 to choose (64 up to n = 512, else
 * 128).  n need not be a multiple of nb: the last diagonal tile is completed
 * with the identity, which changes none of L.
 * opts (may be NULL): precision must be TILEQR_FP64 (else
 * TILEQR_EUNSUPPORTED); stream orders the call; flags TILEQR_FLAG_ASYNC
 * (return without waiting; status and info unchecked), TILEQR_FLAG_SERIAL
 * (one workgroup runs the tasks in Algorithm 1's loop order),
 * TILEQR_FLAG_SHUFFLE (randomised queue choice, for testing: the result is
 * bitwise the same as in every other order), TILEQR_FLAG_TIMING (info
 * times); workers and spin_limit as for tileqr_factor_ex.  info (may be
 * NULL): host memory.
 * Returns TILEQR_OK; TILEQR_ENONFINITE (NaN or Inf in the lower triangle:
 * nothing written); TILEQR_ENOTSPD (info->minor set; A is left unchanged);
 * TILEQR_ETIMEOUT; TILEQR_EHIP; TILEQR_ENOMEM; or -1 n, -2 A, -3 lda, -4 nb,
 * -5 opts for an invalid argument (nothing touched).
 */
int tilechol_factor(int64_t n, double *A, int64_t lda, int64_t nb, const tileqr_opts *opts,
                    tilechol_info *info);

/*
 * X with A X = B, from the factor tilechol_factor left in L (the lower
 * triangle of the n x n column-major array L, leading dimension
 * ldl >= max(1, n); its strict upper triangle is not read): the forward
 * solve L Y = B, then the back solve L^T X = Y -- the use of the factor
 * L L^T = A of Section 3.1 (LAPACK's DPOTRS).  B (n x nrhs, leading
 * dimension ldb >= max(1, n)) is overwritten with X.  Both solves run on
 * FP64 MFMA by 64-row blocks over nb x nb tiles of L^T (nb 64 or 128, or 0 to
 * choose as tilechol_factor does; any nb works with any factor).
 * opts (may be NULL): precision must be TILEQR_FP64 (else
 * TILEQR_EUNSUPPORTED); stream orders the call; TILEQR_FLAG_ASYNC returns
 * without waiting (status unchecked); spin_limit as for tileqr_factor_ex.
 * Returns TILEQR_OK; TILEQR_ESINGULAR (an exact zero on the diagonal of L;
 * B then holds no solution); TILEQR_ETIMEOUT; TILEQR_EHIP; TILEQR_ENOMEM; or
 * -1 n, -2 nrhs, -3 L, -4 ldl, -5 B, -6 ldb, -7 nb, -8 opts for an invalid
 * argument (nothing touched).
 */
int tilechol_solve(int64_t n, int64_t nrhs, const double *L, int64_t ldl, double *B, int64_t ldb, int64_t nb,
                   const tileqr_opts *opts);

/* Tasks of Algorithm 1 on a p x p tile grid (host only): returns the total
 * and, if counts != NULL, writes {POTF2, TRSM, GSMM} counts. */
int64_t tilechol_dag_counts(int64_t p, int64_t *counts);

/* Host-only check of the scheduler's task graph for a p x p tile grid:
 * every task's in-degree equals the number of successor lists it appears
 * in, and `trials` executions in random topological orders (seeded) run
 * every task once, each after the tasks Algorithm 1 makes it depend on (the
 * last writer of each tile it reads or writes).  Returns 0 if all pass, else
 * a positive code naming the first failed check. */
int tilechol_dag_selfcheck(int64_t p, int64_t trials, uint64_t seed);

#ifdef __cplusplus
}
#endif

#endif /* TILECHOL_H */
