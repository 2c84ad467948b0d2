/*
 * tilelu: tiled LU factorisation with tiled pairwise pivoting on one AMD
 * Instinct MI355X (gfx950), the third tiled algorithm of Buttari, Langou,
 * Kurzak and Dongarra, "A Class of Parallel Tiled Linear Algebra Algorithms
 * for Multicore Architectures": Section 3.2.2, Algorithm 3, with the inner
 * blocking of Section 3.2.3.  The n x n matrix is cut into nb x nb tiles; the
 * factorisation is the DAG of four kernels, scheduled dynamically (Section 4)
 * by a persistent GPU kernel:
 *   GETRF(k)       P_kk A_kk = L_kk U_kk (partial pivoting inside the tile);
 *   GESSM(k, j)    A_kj <- L_kk^{-1} P_kk A_kj, j > k;
 *   TSTRF(k, i)    the LU of [U_kk; A_ik] with pivoting between U_kk's
 *                  diagonal entry and A_ik's column, by inner panels of ib
 *                  columns, i > k;
 *   SSSSM(k, i, j) [A_kj; A_ij] <- L_ik^{-1} P_ik [A_kj; A_ij].
 * Storage follows the paper: U overwrites the tiles on and right of the
 * diagonal (the upper triangle), L_kk the strictly lower part of A_kk, the
 * multipliers of TSTRF the tile A_ik; the upper part of L_ik (ib x ib unit
 * lower triangles, one per inner panel) and the pivots are kept in caller
 * memory apart.  Pivot conventions (0-based, within the tile): GETRF
 * ipiv[j] = the row exchanged with row j at step j; TSTRF piv[j] = j (U_kk's
 * row kept) or nb + r (exchanged with row r of A_ik).  Ties go to the first
 * candidate (U_kk's entry before the rows of A_ik, lower rows first).
 *
 * Shares the status codes, the options and the library with tileqr.h.  All
 * matrix pointers are DEVICE pointers, column-major FP64.
 */
#ifndef TILELU_H
#define TILELU_H

#include <stddef.h>
#include <stdint.h>

#include "tileqr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t minor;        /* TILEQR_ESINGULAR: the 1-based global column that
                             had no nonzero pivot; else 0                       */
    double ms_factor;     /* device time of the call                            */
    double ms_worker;     /* device time of the factorisation kernel(s)         */
} tilelu_info;

/* Doubles of the Lup area and int32 entries of the pivot area for an n x n
 * factorisation with tiles nb and inner block ib (p = ceil(n / nb)): Lup is
 * p * p * ib * nb (tile (i, k) at (k p + i) ib nb, row-major ib x nb: row
 * j - l0 of the panel starting at l0, column c of the tile), piv is p * p * nb
 * (tile (i, k), i >= k, at (k p + i) nb).  0 for unsupported sizes. */
size_t tilelu_lup_size(int64_t n, int64_t nb, int64_t ib);
size_t tilelu_piv_size(int64_t n, int64_t nb);

/*
 * Algorithm 3 on the n x n matrix A (lda >= max(1, n)); nb = 64 and ib in
 * {16, 32}.  n need not be a multiple of nb: the last diagonal tile is
 * completed with the identity (the caller's arrays see only the n x n
 * part; Lup and piv are sized for the padded grid).
 * opts (may be NULL): precision TILEQR_FP64 only; stream; flags
 * TILEQR_FLAG_ASYNC, TILEQR_FLAG_SERIAL (Algorithm 3's loop order, one step
 * and kernel at a time: the reference order of the tests), TILEQR_FLAG_SHUFFLE,
 * TILEQR_FLAG_TIMING; workers, spin_limit, seed as for tileqr_factor_ex.
 * info (may be NULL): host memory.
 * Returns TILEQR_OK; TILEQR_ENONFINITE (NaN or Inf in A: nothing written);
 * TILEQR_ESINGULAR (a column with no nonzero pivot: info->minor, A left
 * unchanged); TILEQR_ETIMEOUT; TILEQR_EHIP; TILEQR_ENOMEM;
 * TILEQR_EUNSUPPORTED (nb, ib or precision); or -1 n, -2 A, -3 lda, -4 nb,
 * -5 ib, -6 Lup (NULL or not 16-byte aligned), -7 piv, -8 opts for an
 * invalid argument.
 */
int tilelu_factor(int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib, double *Lup, int32_t *piv,
                  const tileqr_opts *opts, tilelu_info *info);

typedef struct {
    int iterations;       /* refinement corrections applied                      */
    int converged;        /* 1 if the backward error reached tol                 */
    double eta;           /* the returned X's largest (over the columns)
                             ||b - A x||_inf / (||A||_inf ||x||_inf)             */
    int64_t minor;        /* TILEQR_ESINGULAR from the factorisation: as in
                             tilelu_info                                        */
} tilelu_solve_info;

/*
 * X with A X = B for the n x n column-major A (lda >= max(1, n), not
 * modified) and nrhs >= 0 right-hand sides B (ldb >= max(1, n)): the
 * tiled LU of Algorithm 3 with tiled pairwise pivoting (nb 64, inner panels
 * ib 16 or 32, 0 choosing 16) computed into the library's workspace, the
 * factor's transformations applied to B in the factorisation's order
 * (GESSM(k) on row block k, then SSSSM(k, i) on row blocks k and i), the back
 * solve with U, then classical refinement with FP64 residuals: Section 3.2.4
 * notes that tiled pairwise pivoting is not guaranteed stable and advises
 * checking the backward error ||b - A x||_inf / (||A||_inf ||x||_inf) and
 * refining.  The right-hand sides are taken 64 columns at a time, each
 * block with its own refinement, which stops at opts->tol (default 1e-14)
 * for every column, after opts->max_iter corrections (<= 64), or after two
 * corrections that fail to halve the error; the best iterate goes to X
 * (ldx >= max(1, n)).
 * opts (may be NULL): precision must be TILEQR_FP64 and TILEQR_FLAG_ASYNC is
 * not accepted (TILEQR_EUNSUPPORTED: the refinement decides on the host);
 * stream, workers, spin_limit, TILEQR_FLAG_SERIAL / _SHUFFLE as for
 * tilelu_factor.  info (may be NULL): host memory.
 * Returns TILEQR_OK; TILEQR_ENOCONV (best iterate in X); TILEQR_ESINGULAR;
 * TILEQR_ENONFINITE; TILEQR_ETIMEOUT; TILEQR_EHIP; TILEQR_ENOMEM; or -1 n,
 * -2 nrhs, -3 A, -4 lda, -5 B, -6 ldb, -7 X, -8 ldx, -9 ib, -10 opts for an
 * invalid argument (nothing written).
 */
int tilelu_solve(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B, int64_t ldb, double *X,
                 int64_t ldx, int64_t ib, const tileqr_opts *opts, tilelu_solve_info *info);

/* Tasks of Algorithm 3 on a p x p tile grid (host only): the total, and
 * {GETRF, GESSM, TSTRF, SSSSM} counts if counts != NULL. */
int64_t tilelu_dag_counts(int64_t p, int64_t *counts);

/* Host-only check of the scheduler's task graph (as tilechol_dag_selfcheck):
 * in-degrees against successor lists, and random topological orders against
 * Algorithm 3's order of writes to every tile.  0 if all pass. */
int tilelu_dag_selfcheck(int64_t p, int64_t trials, uint64_t seed);

#ifdef __cplusplus
}
#endif

#endif /* TILELU_H */
