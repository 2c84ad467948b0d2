"""Pins of the Cholesky oracle (oracle/cholesky.c) against facts fixed by the
mathematics: exact integer factors, the 2 x 2 closed form (a golden file),
brute force at 50 digits, LAPACK's dpotrf and cho_solve, L L^T = A,
power-of-four scaling, and the order of the first minor that is not positive
definite.  ``test_chol_mutants_are_caught`` plants plausible mistakes in a copy
of the oracle and requires the battery to catch each one.
"""
import os
import shutil
import subprocess
import tempfile

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from conftest import ROOT, load_golden

EPS = np.finfo(np.float64).eps


def spd(seed, n, kappa=1e3):
    """A = U diag(s) U^T with U orthogonal (QR of a Gaussian matrix, numpy)
    and s log-spaced from 1 to 1/kappa."""
    g = np.random.default_rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((n, n)))
    s = np.logspace(0, -np.log10(kappa), n)
    A = (U * s) @ U.T
    return (A + A.T) / 2


def int_lower(seed, n, hi=9):
    g = np.random.default_rng(seed)
    L = np.tril(g.integers(-hi, hi + 1, (n, n))).astype(np.float64)
    L[np.arange(n), np.arange(n)] = g.integers(1, hi + 1, n)
    return L


# ------------------------------------------------------------------ battery

def check_exact_integer(O):
    # Integer L with a positive integer diagonal: every step of the textbook
    # recurrence is exact, so the factor comes back bitwise; so does x from
    # L L^T x = b with integer x.
    for seed, n in ((1, 3), (2, 6), (3, 11)):
        L0 = int_lower(seed, n)
        A = L0 @ L0.T
        L, info = O.potrf(A)
        assert info == 0 and np.array_equal(L, L0), (seed, n)
        x = np.arange(1, n + 1, dtype=np.float64) - n // 2
        assert np.array_equal(O.potrs(L, A @ x), x), (seed, n)


def check_closed_form_2x2(O):
    gold = load_golden("cholesky_2x2.txt")
    L, info = O.potrf(np.array(gold["A1"]).reshape(2, 2))
    assert info == 0 and np.array_equal(L.ravel(), np.array(gold["L1"]))
    L, info = O.potrf(np.array(gold["A2"]).reshape(2, 2))
    assert info == 0
    assert np.allclose(L.ravel(), np.array(gold["L2"]), rtol=2 * EPS, atol=0)
    _, info = O.potrf(np.array(gold["A3"]).reshape(2, 2))
    assert info == int(gold["info3"][0])


def check_brute_force_mpmath(O):
    mpmath.mp.dps = 50
    for seed, n in ((4, 5), (5, 8)):
        A = spd(seed, n, 1e4)
        L, info = O.potrf(A)
        assert info == 0
        Lm = mpmath.cholesky(mpmath.matrix(A.tolist()))
        Lx = np.array([[float(Lm[i, j]) for j in range(n)] for i in range(n)])
        assert np.linalg.norm(L - Lx) <= 1e-15 * 1e2 * n * np.linalg.norm(Lx), (seed, n)


def check_vs_lapack(O):
    for seed, n in ((6, 40), (7, 97)):
        A = spd(seed, n, 1e5)
        L, info = O.potrf(A)
        assert info == 0
        Ll = np.linalg.cholesky(A)
        assert np.linalg.norm(L - Ll) <= 1e-15 * 1e3 * np.linalg.norm(Ll), (seed, n)
        B = np.random.default_rng(seed).standard_normal((n, 3))
        X = O.potrs(L, B)
        Xl = scipy.linalg.cho_solve((Ll, True), B)
        assert np.linalg.norm(X - Xl) <= 1e-15 * 1e6 * np.linalg.norm(Xl), (seed, n)


def check_llt_is_a(O):
    for seed, n in ((8, 64), (9, 130)):
        A = spd(seed, n, 1e6)
        L, info = O.potrf(A)
        assert info == 0
        assert np.all(np.diag(L) > 0) and np.array_equal(L, np.tril(L))
        assert np.linalg.norm(A - L @ L.T) <= 4 * n * EPS * np.linalg.norm(A), (seed, n)


def check_power_of_four_scaling(O):
    # sqrt(4^e x) = 2^e sqrt(x) and every quotient and product scales by a
    # power of two exactly: the factor of 4^e A is 2^e L, bitwise.
    A = spd(10, 23, 1e3)
    L, _ = O.potrf(A)
    for e in (-20, 7, 300):
        Ls, info = O.potrf(A * 4.0 ** e)
        assert info == 0 and np.array_equal(Ls, L * 2.0 ** e), e


def check_first_bad_minor(O):
    # The order of the first leading minor that is not positive definite, as
    # LAPACK's dpotrf reports it.
    for seed, n, k in ((11, 9, 4), (12, 16, 1), (13, 16, 16)):
        A = spd(seed, n, 10.0)
        A[k - 1, k - 1] -= 3.0 * A[k - 1, k - 1] + 5.0      # breaks the minor of order k
        _, info = O.potrf(A)
        _, info_l = scipy.linalg.lapack.dpotrf(A, lower=1)
        assert info == info_l == k, (seed, n, k, info, info_l)


def check_upper_triangle_ignored(O):
    # Only the lower triangle is read and written: NaN above the diagonal
    # changes nothing and stays where it was.
    A = spd(14, 12, 1e2)
    L, _ = O.potrf(A)
    F = np.asfortranarray(A.copy())
    iu = np.triu_indices(12, 1)
    F[iu] = np.nan
    info = O.L.oracle_potrf_lower(12, oracle._ptr(F), 12)
    assert info == 0
    assert np.array_equal(np.tril(F), L)
    assert np.all(np.isnan(F[iu]))


BATTERY = [check_exact_integer, check_closed_form_2x2, check_brute_force_mpmath, check_vs_lapack,
           check_llt_is_a, check_power_of_four_scaling, check_first_bad_minor, check_upper_triangle_ignored]


@pytest.mark.parametrize("check", BATTERY, ids=lambda f: f.__name__)
def test_chol_oracle_pin(check):
    check(oracle.chol_default())


def test_chol_bad_arguments_and_empty():
    O = oracle.chol_default()
    d = np.zeros(4)
    p = oracle._ptr(d)
    assert O.L.oracle_potrf_lower(-1, p, 1) == -1
    assert O.L.oracle_potrf_lower(2, None, 2) == -2
    assert O.L.oracle_potrf_lower(2, p, 1) == -3
    assert O.L.oracle_potrf_lower(0, p, 1) == 0
    assert O.L.oracle_potrs_lower(2, 1, p, 1, p, 2) == -4
    L, info = O.potrf(np.zeros((0, 0)))
    assert info == 0 and L.shape == (0, 0)
    _, info = O.potrf(np.array([[np.nan]]))
    assert info == 1


# ---------------------------------------------------------- mutation test

MUTANTS = {
    "pivot_sign": ("d -= AT(A, lda, j, k) * AT(A, lda, j, k);", "d += AT(A, lda, j, k) * AT(A, lda, j, k);"),
    "pivot_drops_last": ("for (int64_t k = 0; k < j; ++k) d -=", "for (int64_t k = 0; k + 1 < j; ++k) d -="),
    "offdiag_transposed": ("s -= AT(A, lda, i, k) * AT(A, lda, j, k);", "s -= AT(A, lda, i, k) * AT(A, lda, k, j);"),
    "offdiag_wrong_row": ("s -= AT(A, lda, i, k) * AT(A, lda, j, k);", "s -= AT(A, lda, i, k) * AT(A, lda, i, k);"),
    "divide_by_pivot": ("AT(A, lda, i, j) = s / ljj;", "AT(A, lda, i, j) = s / d;"),
    "reads_upper": ("double s = AT(A, lda, i, j);", "double s = AT(A, lda, j, i);"),
    "info_off_by_one": ("if (!(d > 0.0)) return (int)(j + 1);", "if (!(d > 0.0)) return (int)j;"),
    "forward_transposed": ("for (int64_t k = 0; k < i; ++k) s -= AT(F, ldf, i, k) * b[k];",
                           "for (int64_t k = 0; k < i; ++k) s -= AT(F, ldf, k, i) * b[k];"),
    "back_wrong_order": ("for (int64_t i = n - 1; i >= 0; --i) {", "for (int64_t i = 0; i < n; ++i) {"),
}


def _build_chol_mutant(tmp, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "cholesky.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path_c = os.path.join(tmp, f"{name}.c")
    path_so = os.path.join(tmp, f"lib{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", "-o", path_so, path_c,
                    "-lm"], check=True)
    return path_so


def test_chol_mutants_are_caught():
    tmp = tempfile.mkdtemp(prefix="chol_mut_")
    try:
        survivors = []
        for name, (old, new) in MUTANTS.items():
            O = oracle.CholOracle(_build_chol_mutant(tmp, name, old, new))
            caught = False
            for check in BATTERY:
                try:
                    check(O)
                except (AssertionError, ValueError, np.linalg.LinAlgError, ZeroDivisionError):
                    caught = True
                    break
            if not caught:
                survivors.append(name)
        assert not survivors, f"planted mistakes not caught by any pin: {survivors}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
