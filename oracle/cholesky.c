/*
 * Oracle for the tiled Cholesky factorisation: TEST INFRASTRUCTURE ONLY.  It
 * is linked and called by the test suite and the benchmark's checks, never by
 * the library, and shares no code, header or constant with the GPU path.
 *
 * What it computes.  The tiled algorithm of the paper (Section 3.1,
 * Algorithm 1: POTF2 on a diagonal tile, TRSM on the tiles below it, GSMM on
 * the trailing tiles) is a reordering of the Cholesky factorisation
 * A = L L^T of a symmetric positive definite A, L lower triangular with a
 * positive diagonal.  So the oracle is that definition written out, one
 * column at a time (the textbook inner-product form, no blocking):
 *   L[j][j] = sqrt(A[j][j] - sum_{k<j} L[j][k]^2)
 *   L[i][j] = (A[i][j] - sum_{k<j} L[i][k] L[j][k]) / L[j][j],  i > j,
 * each sum taken in increasing k.  Only the lower triangle of A is read; the
 * strict upper triangle is neither read nor written.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math), so every product and sum
 * is an individually rounded IEEE-754 double operation.
 *
 * Pointers are host memory, column-major with the given leading dimension.
 *
 * Parity status: pinned by the CPU tests (exact integer factors, the 2 x 2
 * closed form, brute force in high precision, LAPACK cross-checks, L L^T = A,
 * power-of-four scaling, the order of the first minor that is not positive
 * definite); not "parity unpinned".
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define AT(M, ld, r, c) ((M)[(size_t)(c) * (size_t)(ld) + (size_t)(r)])

/*
 * Overwrites the lower triangle of A (n x n, leading dimension lda) with L.
 * Returns 0 on success; -1 (n < 0), -2 (A NULL with n > 0), -3 (lda < n);
 * or j + 1 > 0 when the pivot of column j, A[j][j] - sum_k L[j][k]^2, is not
 * a positive number (the leading minor of order j + 1 is not positive
 * definite, or the input holds NaN): columns 0 .. j-1 then hold L, the rest
 * of the lower triangle is partly updated.
 */
int oracle_potrf_lower(int64_t n, double *A, int64_t lda)
{
    if (n < 0) return -1;
    if (n > 0 && A == NULL) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    for (int64_t j = 0; j < n; ++j) {
        double d = AT(A, lda, j, j);
        for (int64_t k = 0; k < j; ++k) d -= AT(A, lda, j, k) * AT(A, lda, j, k);
        if (!(d > 0.0)) return (int)(j + 1);
        const double ljj = sqrt(d);
        AT(A, lda, j, j) = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = AT(A, lda, i, j);
            for (int64_t k = 0; k < j; ++k) s -= AT(A, lda, i, k) * AT(A, lda, j, k);
            AT(A, lda, i, j) = s / ljj;
        }
    }
    return 0;
}

/*
 * Solves A X = B with the factor of oracle_potrf_lower (L in the lower
 * triangle of F): L Y = B by forward substitution, then L^T X = Y by back
 * substitution, each in increasing (then decreasing) row order.  B (n x nrhs,
 * ldb) is overwritten with X.  Returns 0, or -i for a bad argument i.
 */
int oracle_potrs_lower(int64_t n, int64_t nrhs, const double *F, int64_t ldf, double *B, int64_t ldb)
{
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && F == NULL) return -3;
    if (ldf < (n > 1 ? n : 1)) return -4;
    if (n > 0 && nrhs > 0 && B == NULL) return -5;
    if (ldb < (n > 1 ? n : 1)) return -6;
    for (int64_t c = 0; c < nrhs; ++c) {
        double *b = B + (size_t)c * (size_t)ldb;
        for (int64_t i = 0; i < n; ++i) {
            double s = b[i];
            for (int64_t k = 0; k < i; ++k) s -= AT(F, ldf, i, k) * b[k];
            b[i] = s / AT(F, ldf, i, i);
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int64_t k = i + 1; k < n; ++k) s -= AT(F, ldf, k, i) * b[k];
            b[i] = s / AT(F, ldf, i, i);
        }
    }
    return 0;
}
