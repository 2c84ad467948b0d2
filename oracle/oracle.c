/*
 * Oracle: plain, slow, single-threaded FP64 Householder QR and the operations
 * built on it.  TEST INFRASTRUCTURE ONLY: it is linked and called by the test
 * suite, by the smoke check and by the CPU-baseline leg of the benchmark, never
 * by the library.  It shares no code, header or constant with the GPU path.
 *
 * What it computes.  The tiled algorithm of the paper (Section 3.2.1,
 * Algorithm 2: GEQRT / LARFB / TSQRT / SSRFB on b x b tiles) is an exact
 * reformulation of the Householder QR factorisation A = QR (Q orthogonal, R
 * upper triangular) as an updating factorisation (Section 3.2).  So the
 * oracle is that plain definition written out: one Householder reflector per
 * column, applied to the remaining columns straight away (no blocking, no WY
 * accumulation, no reordering).  Q is kept as the n reflectors
 * H_j = I - tau_j v_j v_j^T with v_j(j) = 1 stored below the diagonal, the
 * classical LAPACK storage.
 *
 * Reflector convention (the paper only refers to the compact WY technique
 * and fixes no sign): for x = [alpha; x2],
 *   beta  = -sign(alpha) * ||x||  with sign(+-0) = +1,
 *   tau   = (beta - alpha) / beta, v = [1; x2 / (alpha - beta)],
 *   tau   = 0 and nothing changes when ||x2|| = 0 (even for alpha < 0).
 * Norms are computed with a scaled two-pass sum so that no intermediate
 * overflows or underflows.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math), so every
 * product and sum is an individually rounded IEEE-754 double operation.
 *
 * Every pointer is host memory, column-major with the given leading
 * dimension.  Functions return 0 on success and -i for a bad argument i.
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, exact integer cases, brute force in high precision, LAPACK
 * cross-checks and invariants); none is "parity unpinned".
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#define AT(M, ld, r, c) ((M)[(size_t)(c) * (size_t)(ld) + (size_t)(r)])

/* Euclidean norm of x[0..len) with a scaling pass: scale = max |x_i|,
 * result = scale * sqrt(sum (x_i / scale)^2).  Exact zero for a zero vector. */
static double scaled_norm(const double *x, int64_t len, int64_t stride)
{
    double scale = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double a = fabs(x[i * stride]);
        if (a > scale) scale = a;
    }
    if (scale == 0.0) return 0.0;
    double sum = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double t = x[i * stride] / scale;
        sum += t * t;
    }
    return scale * sqrt(sum);
}

/*
 * Householder QR of the m x n matrix A (in place).  On return the upper
 * triangle of A[0:min(m,n), :] holds R, the part below the diagonal holds the
 * reflector tails v_j(j+1:m), and tau[0:min(m,n)] the reflector scalars.
 * This is the factorisation A = QR that every tile kernel of Section 3.2.1
 * contributes to (DGEQRT/DTSQRT produce R, DLARFB/DSSRFB apply Q^T).
 */
int oracle_geqr2(int64_t m, int64_t n, double *A, int64_t lda, double *tau)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (lda < (m > 1 ? m : 1)) return -4;
    int64_t kmax = m < n ? m : n;
    for (int64_t j = 0; j < kmax; ++j) {
        double alpha = AT(A, lda, j, j);
        double *x = &AT(A, lda, j + 1, j);
        int64_t len = m - j - 1;
        double xnorm = scaled_norm(x, len, 1);
        if (xnorm == 0.0) {
            tau[j] = 0.0;           /* H_j = I: column already reduced */
            continue;
        }
        double h = hypot(alpha, xnorm);
        double beta = (alpha >= 0.0) ? -h : h;
        double t = (beta - alpha) / beta;
        double scal = 1.0 / (alpha - beta);
        for (int64_t r = 0; r < len; ++r) x[r] *= scal;
        AT(A, lda, j, j) = beta;
        tau[j] = t;
        /* Apply H_j = I - tau v v^T to columns j+1..n-1, rows j..m-1. */
        for (int64_t c = j + 1; c < n; ++c) {
            double w = AT(A, lda, j, c);
            for (int64_t r = 0; r < len; ++r) w += x[r] * AT(A, lda, j + 1 + r, c);
            double tw = t * w;
            AT(A, lda, j, c) -= tw;
            for (int64_t r = 0; r < len; ++r) AT(A, lda, j + 1 + r, c) -= x[r] * tw;
        }
    }
    return 0;
}

/* Apply one reflector (v stored below the diagonal of column j of A, implicit
 * 1 on the diagonal) to the rows j..m-1 of every column of B. */
static void apply_reflector(int64_t m, int64_t j, const double *A, int64_t lda,
                            double t, int64_t nrhs, double *B, int64_t ldb)
{
    if (t == 0.0) return;
    const double *v = &AT(A, lda, j + 1, j);
    int64_t len = m - j - 1;
    for (int64_t c = 0; c < nrhs; ++c) {
        double w = AT(B, ldb, j, c);
        for (int64_t r = 0; r < len; ++r) w += v[r] * AT(B, ldb, j + 1 + r, c);
        double tw = t * w;
        AT(B, ldb, j, c) -= tw;
        for (int64_t r = 0; r < len; ++r) AT(B, ldb, j + 1 + r, c) -= v[r] * tw;
    }
}

/* B := Q^T B = H_{k-1} ... H_1 H_0 B  (reflectors applied in ascending order,
 * the order in which the factorisation applied them to A).  k = min(m, n). */
int oracle_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                    const double *tau, double *B, int64_t ldb)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (ldb < (m > 1 ? m : 1)) return -8;
    int64_t kmax = m < n ? m : n;
    for (int64_t j = 0; j < kmax; ++j) apply_reflector(m, j, A, lda, tau[j], nrhs, B, ldb);
    return 0;
}

/* B := Q B = H_0 H_1 ... H_{k-1} B  (each H_j is symmetric, so Q B applies
 * the same reflectors in descending order). */
int oracle_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                   const double *tau, double *B, int64_t ldb)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (ldb < (m > 1 ? m : 1)) return -8;
    int64_t kmax = m < n ? m : n;
    for (int64_t j = kmax - 1; j >= 0; --j) apply_reflector(m, j, A, lda, tau[j], nrhs, B, ldb);
    return 0;
}

/* Solve R X = C by back substitution, R the n x n upper triangle of R
 * (leading dimension ldr), C overwritten by X (n x nrhs).  Returns j+1 > 0
 * when R(j,j) == 0 (singular, C untouched), else 0. */
int oracle_trsv_upper(int64_t n, const double *R, int64_t ldr, int64_t nrhs,
                      double *C, int64_t ldc)
{
    if (n < 0) return -1;
    if (ldr < (n > 1 ? n : 1)) return -3;
    if (nrhs < 0) return -4;
    if (ldc < (n > 1 ? n : 1)) return -6;
    for (int64_t j = 0; j < n; ++j)
        if (AT(R, ldr, j, j) == 0.0) return (int)(j + 1);
    for (int64_t c = 0; c < nrhs; ++c) {
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = AT(C, ldc, i, c);
            for (int64_t k = i + 1; k < n; ++k) s -= AT(R, ldr, i, k) * AT(C, ldc, k, c);
            AT(C, ldc, i, c) = s / AT(R, ldr, i, i);
        }
    }
    return 0;
}

/*
 * Least squares min ||B - A X||_2 for m >= n, A of full column rank:
 *   Q R = A,  C = Q^T B,  R X = C[0:n],  residual computed from the original A.
 * A and B are left untouched; the work copies are allocated here.
 * X is n x nrhs (leading dimension ldx); Rres (m x nrhs, leading dimension
 * ldr, may be NULL) receives B - A X.
 */
int oracle_lstsq(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double *X, int64_t ldx,
                 double *Rres, int64_t ldr)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (ldb < (m > 1 ? m : 1)) return -7;
    if (ldx < (n > 1 ? n : 1)) return -9;
    if (Rres && ldr < (m > 1 ? m : 1)) return -11;
    double *F = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (size_t)(n > 0 ? n : 1));
    double *C = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (size_t)(nrhs > 0 ? nrhs : 1));
    double *tau = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!F || !C || !tau) { free(F); free(C); free(tau); return 1; }
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < m; ++r) AT(F, m, r, c) = AT(A, lda, r, c);
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t r = 0; r < m; ++r) AT(C, m, r, c) = AT(B, ldb, r, c);
    int info = oracle_geqr2(m, n, F, m > 1 ? m : 1, tau);
    if (info == 0) info = oracle_apply_qt(m, n, nrhs, F, m > 1 ? m : 1, tau, C, m > 1 ? m : 1);
    if (info == 0) info = oracle_trsv_upper(n, F, m > 1 ? m : 1, nrhs, C, m > 1 ? m : 1);
    if (info == 0) {
        for (int64_t c = 0; c < nrhs; ++c)
            for (int64_t r = 0; r < n; ++r) AT(X, ldx, r, c) = AT(C, m, r, c);
        if (Rres) {
            for (int64_t c = 0; c < nrhs; ++c)
                for (int64_t r = 0; r < m; ++r) {
                    double s = AT(B, ldb, r, c);
                    for (int64_t k = 0; k < n; ++k) s -= AT(A, lda, r, k) * AT(X, ldx, k, c);
                    AT(Rres, ldr, r, c) = s;
                }
        }
    }
    free(F); free(C); free(tau);
    return info;
}
