/*
 * Oracle for the tiled LU factorisation with tiled pairwise pivoting: TEST
 * INFRASTRUCTURE ONLY.  It is called by the test suite, never by the
 * library, and shares no code, header or constant with the GPU path.
 *
 * What it computes.  Gaussian elimination with tiled pairwise pivoting
 * (Section 3.2.2, Algorithm 3, named GETWP in the stability discussion) is
 * its own elimination order, not plain partial pivoting, so the oracle takes
 * Algorithm 3's steps in the paper's order on b x b tiles (n = p b), each
 * kernel written out plainly:
 *   GETRF(k)       Gaussian elimination with partial pivoting of A_kk (the
 *                  result of LAPACK's blocked dgetrf, written unblocked):
 *                  P_kk A_kk = L_kk U_kk, pivots ipiv[j] (row swapped with j
 *                  at step j, whole rows of the tile), L_kk unit lower;
 *   GESSM(k, j)    A_kj <- L_kk^{-1} P_kk A_kj;
 *   TSTRF(k, i)    the LU of [U_kk; A_ik] with pivoting between the diagonal
 *                  entry U_kk[j][j] and the column of A_ik, by inner panels
 *                  of s columns (Section 3.2.3 applied to LU): in panel
 *                  [l0, l0 + s), column j picks the largest magnitude among
 *                  U[j][j] and A[0..b)[j] (the first one on ties, U first);
 *                  a pivot in A row r swaps U row j and A row r from column
 *                  j on, and moves A row r's multipliers of the panel's
 *                  earlier columns to L_up (U row j holds zeros there; L_kk
 *                  keeps the strictly lower part of the diagonal tile); the
 *                  multipliers A[:, j] / U[j][j] are stored in A's column j
 *                  and update the rest of the panel; the columns right of
 *                  the panel are then updated as a block: U rows of the panel
 *                  by the unit lower s x s triangle L_up, then every A row by
 *                  its multipliers.
 *                  piv[j] = j (U row kept) or b + r (swapped with A row r);
 *   SSSSM(k, i, j) [A_kj; A_ij] <- L_ik^{-1} P_ik [A_kj; A_ij], panel by
 *                  panel in the same order: the swaps of the panel, then the
 *                  panel's rows of A_kj by L_up, then A_ij by the multipliers.
 * The factor overwrites A (U in the upper triangle of the tiles on and right
 * of the diagonal, L_kk below the diagonal of A_kk, the multipliers of
 * TSTRF in A_ik); L_up (s x b per tile (i, k), i > k: the b/s unit lower
 * s x s triangles side by side, row-major, strictly lower entries) and the
 * pivots (b per tile (i, k), i >= k) are kept apart, as the paper does.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math).  Host memory, column-major.
 *
 * Parity status: pinned by the CPU tests (one tile = LAPACK's dgetrf, no
 * pivoting = plain LU, b = 1 = pairwise pivoting by hand, exact integer
 * cases, solves against LAPACK, a mutation test); not "parity unpinned".
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define AT(M, ld, r, c) ((M)[(size_t)(c) * (size_t)(ld) + (size_t)(r)])

static void swap_rows(double *A, int64_t lda, int64_t r1, int64_t r2, int64_t c0, int64_t c1)
{
    for (int64_t c = c0; c < c1; ++c) {
        const double t = AT(A, lda, r1, c);
        AT(A, lda, r1, c) = AT(A, lda, r2, c);
        AT(A, lda, r2, c) = t;
    }
}

/* GETRF: GEPP of the b x b tile at T (leading dimension ld).  Returns 0 or
 * j + 1 when column j has no nonzero pivot. */
static int getrf_tile(int64_t b, double *T, int64_t ld, int32_t *ipiv)
{
    for (int64_t j = 0; j < b; ++j) {
        int64_t p = j;
        for (int64_t r = j + 1; r < b; ++r)
            if (fabs(AT(T, ld, r, j)) > fabs(AT(T, ld, p, j))) p = r;
        ipiv[j] = (int32_t)p;
        if (AT(T, ld, p, j) == 0.0) return (int)(j + 1);
        if (p != j) swap_rows(T, ld, j, p, 0, b);
        const double d = AT(T, ld, j, j);
        for (int64_t r = j + 1; r < b; ++r) AT(T, ld, r, j) = AT(T, ld, r, j) / d;
        for (int64_t c = j + 1; c < b; ++c)
            for (int64_t r = j + 1; r < b; ++r) AT(T, ld, r, c) -= AT(T, ld, r, j) * AT(T, ld, j, c);
    }
    return 0;
}

/* GESSM: X <- L^{-1} P X for the b x nc block X, with L and P of GETRF. */
static void gessm_tile(int64_t b, int64_t nc, const double *L, int64_t ldl, const int32_t *ipiv, double *X,
                       int64_t ldx)
{
    for (int64_t j = 0; j < b; ++j)
        if (ipiv[j] != j) swap_rows(X, ldx, j, ipiv[j], 0, nc);
    for (int64_t c = 0; c < nc; ++c)
        for (int64_t j = 0; j < b; ++j)
            for (int64_t r = j + 1; r < b; ++r) AT(X, ldx, r, c) -= AT(L, ldl, r, j) * AT(X, ldx, j, c);
}

/* TSTRF on [U; A]: U the upper triangle (diagonal included) of the b x b
 * tile at Ut (its strictly lower part, L_kk, is neither read nor written), A
 * the b x b tile at At; inner panels of s columns.  Lup: s x b row-major, the
 * triangle of the panel holding column c in column c, row j - l0 for panel
 * row j.  Returns 0 or j + 1 when column j has only zeros to pivot on. */
static int tstrf_tile(int64_t b, int64_t s, double *Ut, int64_t ldu, double *At, int64_t lda, double *Lup,
                      int32_t *piv)
{
    for (int64_t i = 0; i < s * b; ++i) Lup[i] = 0.0;
    for (int64_t l0 = 0; l0 < b; l0 += s) {
        const int64_t l1 = l0 + s;
        for (int64_t j = l0; j < l1; ++j) {
            int64_t p = -1;                    /* -1: the U row */
            double best = fabs(AT(Ut, ldu, j, j));
            for (int64_t r = 0; r < b; ++r)
                if (fabs(AT(At, lda, r, j)) > best) {
                    best = fabs(AT(At, lda, r, j));
                    p = r;
                }
            if (best == 0.0) return (int)(j + 1);
            if (p >= 0) {
                /* U row j <-> A row p from column j on; the A row's
                 * multipliers of the panel's earlier columns move to L_up
                 * (U row j is zero there). */
                for (int64_t c = j; c < b; ++c) {
                    const double t = AT(Ut, ldu, j, c);
                    AT(Ut, ldu, j, c) = AT(At, lda, p, c);
                    AT(At, lda, p, c) = t;
                }
                for (int64_t c = l0; c < j; ++c) {
                    Lup[(j - l0) * b + c] = AT(At, lda, p, c);
                    AT(At, lda, p, c) = 0.0;
                }
                piv[j] = (int32_t)(b + p);
            } else {
                piv[j] = (int32_t)j;
            }
            const double d = AT(Ut, ldu, j, j);
            /* Multipliers of the A rows; the panel's later columns updated. */
            for (int64_t r = 0; r < b; ++r) AT(At, lda, r, j) = AT(At, lda, r, j) / d;
            for (int64_t c = j + 1; c < l1; ++c)
                for (int64_t r = 0; r < b; ++r) AT(At, lda, r, c) -= AT(At, lda, r, j) * AT(Ut, ldu, j, c);
        }
        /* The columns right of the panel: U's panel rows by L_up (forward),
         * then the A rows by their multipliers. */
        for (int64_t c = l1; c < b; ++c) {
            for (int64_t r = l0; r < l1; ++r)
                for (int64_t q = l0; q < r; ++q) AT(Ut, ldu, r, c) -= Lup[(r - l0) * b + q] * AT(Ut, ldu, q, c);
            for (int64_t q = l0; q < l1; ++q)
                for (int64_t r = 0; r < b; ++r) AT(At, lda, r, c) -= AT(At, lda, r, q) * AT(Ut, ldu, q, c);
        }
    }
    return 0;
}

/* SSSSM: [X1; X2] <- L^{-1} P [X1; X2] (X1, X2 b x nc) with the
 * transformation of TSTRF (multipliers in L2 = the factored A tile, L_up,
 * pivots), panel by panel. */
static void ssssm_tile(int64_t b, int64_t s, int64_t nc, const double *L2, int64_t ldl, const double *Lup,
                       const int32_t *piv, double *X1, int64_t ld1, double *X2, int64_t ld2)
{
    for (int64_t l0 = 0; l0 < b; l0 += s) {
        const int64_t l1 = l0 + s;
        for (int64_t j = l0; j < l1; ++j)
            if (piv[j] >= b) {
                const int64_t p = piv[j] - b;
                for (int64_t c = 0; c < nc; ++c) {
                    const double t = AT(X1, ld1, j, c);
                    AT(X1, ld1, j, c) = AT(X2, ld2, p, c);
                    AT(X2, ld2, p, c) = t;
                }
            }
        for (int64_t c = 0; c < nc; ++c) {
            for (int64_t r = l0; r < l1; ++r)
                for (int64_t q = l0; q < r; ++q) AT(X1, ld1, r, c) -= Lup[(r - l0) * b + q] * AT(X1, ld1, q, c);
            for (int64_t q = l0; q < l1; ++q)
                for (int64_t r = 0; r < b; ++r) AT(X2, ld2, r, c) -= AT(L2, ldl, r, q) * AT(X1, ld1, q, c);
        }
    }
}

/*
 * Algorithm 3 on the n x n matrix A (n = p b, b % s == 0).  Lup: p * p * s * b
 * doubles (block (i, k) at ((k p + i) s b)); piv: p * p * b ints (tile (i, k)
 * at (k p + i) b).  Returns 0; -1 n, -2 b, -3 s, -4 A, -5 lda, -6 Lup, -7 piv
 * for a bad argument; or j + 1 > 0 when global column j had no nonzero pivot
 * (the factorisation stops there).
 */
int oracle_tile_lu(int64_t n, int64_t b, int64_t s, double *A, int64_t lda, double *Lup, int32_t *piv)
{
    if (n < 0) return -1;
    if (b < 1 || (n > 0 && n % b != 0)) return -2;
    if (s < 1 || b % s != 0) return -3;
    if (n > 0 && A == NULL) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (n > 0 && Lup == NULL) return -6;
    if (n > 0 && piv == NULL) return -7;
    const int64_t p = n / b;
#define TILE(i, j) (A + (size_t)(j) * b * (size_t)lda + (size_t)(i) * b)
    for (int64_t k = 0; k < p; ++k) {
        int32_t *pk = piv + ((size_t)k * p + k) * b;
        int info = getrf_tile(b, TILE(k, k), lda, pk);
        if (info) return (int)(k * b + info);
        for (int64_t j = k + 1; j < p; ++j) gessm_tile(b, b, TILE(k, k), lda, pk, TILE(k, j), lda);
        for (int64_t i = k + 1; i < p; ++i) {
            double *lup = Lup + ((size_t)k * p + i) * s * b;
            int32_t *pi = piv + ((size_t)k * p + i) * b;
            info = tstrf_tile(b, s, TILE(k, k), lda, TILE(i, k), lda, lup, pi);
            if (info) return (int)(k * b + info);
            for (int64_t j = k + 1; j < p; ++j)
                ssssm_tile(b, s, b, TILE(i, k), lda, lup, pi, TILE(k, j), lda, TILE(i, j), lda);
        }
    }
#undef TILE
    return 0;
}

/*
 * Solve A X = B with the factor of oracle_tile_lu: the transformations of
 * Algorithm 3 applied to B's row blocks in the same order (GESSM's on block
 * k, SSSSM's on blocks k and i), then back substitution with U (the upper
 * triangle of F).  B (n x nrhs, ldb) is overwritten with X.
 */
int oracle_tile_lu_solve(int64_t n, int64_t b, int64_t s, const double *F, int64_t ldf, const double *Lup,
                         const int32_t *piv, int64_t nrhs, double *B, int64_t ldb)
{
    if (n < 0) return -1;
    if (b < 1 || (n > 0 && n % b != 0)) return -2;
    if (s < 1 || b % s != 0) return -3;
    if (n > 0 && (F == NULL || Lup == NULL || piv == NULL)) return -4;
    if (ldf < (n > 1 ? n : 1) || ldb < (n > 1 ? n : 1)) return -5;
    if (nrhs < 0 || (n > 0 && nrhs > 0 && B == NULL)) return -6;
    const int64_t p = n / b;
    for (int64_t k = 0; k < p; ++k) {
        const double *Lkk = F + (size_t)k * b * (size_t)ldf + (size_t)k * b;
        gessm_tile(b, nrhs, Lkk, ldf, piv + ((size_t)k * p + k) * b, B + (size_t)k * b, ldb);
        for (int64_t i = k + 1; i < p; ++i) {
            const double *Lik = F + (size_t)k * b * (size_t)ldf + (size_t)i * b;
            ssssm_tile(b, s, nrhs, Lik, ldf, Lup + ((size_t)k * p + i) * s * b, piv + ((size_t)k * p + i) * b,
                       B + (size_t)k * b, ldb, B + (size_t)i * b, ldb);
        }
    }
    for (int64_t c = 0; c < nrhs; ++c) {
        double *x = B + (size_t)c * (size_t)ldb;
        for (int64_t r = n - 1; r >= 0; --r) {
            double t = x[r];
            for (int64_t q = r + 1; q < n; ++q) t -= AT(F, ldf, r, q) * x[q];
            x[r] = t / AT(F, ldf, r, r);
        }
    }
    return 0;
}
