"""Pins of the tiled LU oracle (oracle/lu.c, Algorithm 3 with tiled pairwise
pivoting) against facts fixed by the mathematics and the paper: one tile is
Gaussian elimination with partial pivoting (LAPACK's dgetrf, same pivots);
1 x 1 tiles are pairwise pivoting, worked by hand (a golden file); a matrix
that needs no pivoting gives the plain LU factors; the inner blocking s only
regroups the same elimination (same U and pivots for every s); the solve
agrees with LAPACK's; and a mutation test plants plausible mistakes in a copy
of the oracle and requires the battery to catch each one.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg

import oracle
from conftest import ROOT, load_golden

EPS = np.finfo(np.float64).eps


def gauss(seed, n):
    return np.random.default_rng(seed).standard_normal((n, n))


def check_one_tile_is_gepp(O):
    for seed, n, s in ((1, 16, 4), (2, 64, 16), (3, 48, 48)):
        A = gauss(seed, n)
        F, _, piv, info = O.tile_lu(A, n, s)
        lu, pv = scipy.linalg.lu_factor(A)
        assert info == 0 and np.array_equal(piv[0, 0], pv), (seed, n)
        assert np.linalg.norm(F - lu) <= 1e2 * n * EPS * np.linalg.norm(lu), (seed, n)


def check_pairwise_by_hand(O):
    g = load_golden("tile_lu_pairwise_3x3.txt")
    A = np.array(g["A"]).reshape(3, 3)
    F, Lup, piv, info = O.tile_lu(A, 1, 1)
    assert info == 0
    assert np.allclose(F.ravel(), np.array(g["F"]), rtol=4 * EPS, atol=4 * EPS)
    assert list(piv[0, :, 0]) == [int(v) for v in g["piv_k0"]]
    assert list(piv[1, 1:, 0]) == [int(v) for v in g["piv_k1"]]
    assert list(piv[2, 2:, 0]) == [int(v) for v in g["piv_k2"]]
    assert np.all(Lup == 0.0)


def check_no_pivoting_is_plain_lu(O):
    # Column diagonal dominance survives elimination, so every pivot is the
    # diagonal entry: the tiled factor is the plain LU (Doolittle) factor,
    # which LAPACK also returns (no swaps).
    for seed, n, b, s in ((4, 64, 16, 4), (5, 96, 32, 8)):
        A = gauss(seed, n)
        A += np.diag(np.abs(A).sum(axis=0) + 1.0)
        F, Lup, piv, info = O.tile_lu(A, b, s)
        lu, pv = scipy.linalg.lu_factor(A)
        assert info == 0 and np.array_equal(pv, np.arange(n))
        assert np.all(Lup == 0.0)
        for k in range(n // b):
            for i in range(k, n // b):
                assert np.array_equal(piv[k, i], np.arange(b)), (k, i)
        assert np.linalg.norm(F - lu) <= 1e2 * n * EPS * np.linalg.norm(lu), (seed, n)


def check_inner_blocking_regroups(O):
    # s changes where the multipliers are kept, not the elimination: U and
    # the pivots agree for every s, and so do the solutions.
    for seed, n, b in ((6, 96, 32), (7, 128, 64)):
        A = gauss(seed, n)
        xr = np.random.default_rng(seed).standard_normal(n)
        ref = None
        for s in (b, b // 2, 8, 4):
            F, Lup, piv, info = O.tile_lu(A, b, s)
            assert info == 0
            x = O.tile_lu_solve(F, Lup, piv, b, s, A @ xr)
            if ref is None:
                ref = (np.triu(F), piv, x)
            else:
                assert np.array_equal(piv, ref[1]), (seed, s)
                assert np.linalg.norm(np.triu(F) - ref[0]) <= 1e2 * n * EPS * np.linalg.norm(ref[0]), (seed, s)
                assert np.linalg.norm(x - ref[2]) <= 1e6 * n * EPS * np.linalg.norm(ref[2]), (seed, s)


def check_solve_vs_lapack(O):
    for seed, n, b, s in ((8, 64, 16, 4), (9, 120, 8, 2), (10, 128, 32, 32), (11, 192, 64, 16)):
        A = gauss(seed, n)
        B = np.random.default_rng(seed + 100).standard_normal((n, 3))
        F, Lup, piv, info = O.tile_lu(A, b, s)
        assert info == 0
        X = O.tile_lu_solve(F, Lup, piv, b, s, B)
        Xl = scipy.linalg.solve(A, B)
        kappa = np.linalg.cond(A)
        assert np.linalg.norm(X - Xl) <= 1e2 * n * EPS * kappa * np.linalg.norm(Xl), (seed, n, b, s)
        eta = np.abs(B - A @ X).max(axis=0) / (np.abs(A).sum(axis=1).max() * np.abs(X).max(axis=0))
        assert eta.max() <= 1e-14, (seed, eta.max())


def check_ties_keep_the_diagonal(O):
    # Equal magnitudes: the first candidate wins, U's diagonal entry before
    # the rows below.  By hand, with 1 x 1 tiles: [[1, 2], [1, 3]] keeps row 0
    # (multiplier 1, A_11 = 3 - 2 = 1).  [[1, 0, 0], [2, 1, 0], [-2, 0, 1]]:
    # step 0 swaps rows 0 and 1 (|2| > |1|; multiplier 0.5, row 1 becomes
    # [-0.5, 0]), then keeps the new row 0 against the tie |-2| (multiplier -1,
    # row 2 becomes [1, 1]); step 1 swaps rows 1 and 2 in columns 1..2
    # (|1| > |-0.5|; multiplier -0.5, last entry 0 - (-0.5)(1) = 0.5), the
    # step-0 multipliers staying in column 0.
    F, _, piv, info = O.tile_lu(np.array([[1.0, 2.0], [1.0, 3.0]]), 1, 1)
    assert info == 0 and piv[0, 1, 0] == 0
    assert np.array_equal(F, np.array([[1.0, 2.0], [1.0, 1.0]]))
    F, _, piv, info = O.tile_lu(np.array([[1.0, 0.0, 0.0], [2.0, 1.0, 0.0], [-2.0, 0.0, 1.0]]), 1, 1)
    assert info == 0 and [piv[0, 1, 0], piv[0, 2, 0], piv[1, 2, 0]] == [1, 0, 1]
    assert np.array_equal(F, np.array([[2.0, 1.0, 0.0], [0.5, 1.0, 1.0], [-1.0, -0.5, 0.5]]))


def check_singular_column_reported(O):
    # An exact zero column leaves no pivot: the 1-based global column.
    A = gauss(12, 64)
    A[:, 37] = 0.0
    _, _, _, info = O.tile_lu(A, 16, 4)
    assert info == 38


BATTERY = [check_one_tile_is_gepp, check_pairwise_by_hand, check_ties_keep_the_diagonal, check_no_pivoting_is_plain_lu,
           check_inner_blocking_regroups, check_solve_vs_lapack, check_singular_column_reported]


@pytest.mark.parametrize("check", BATTERY, ids=lambda f: f.__name__)
def test_lu_oracle_pin(check):
    check(oracle.lu_default())


def test_lu_bad_arguments():
    O = oracle.lu_default()
    A = gauss(13, 8)
    with pytest.raises(ValueError):
        O.tile_lu(A, 3, 1)            # b does not divide n
    with pytest.raises(ValueError):
        O.tile_lu(A, 4, 3)            # s does not divide b
    F, _, _, info = O.tile_lu(np.zeros((0, 0)), 4, 2)
    assert info == 0


MUTANTS = {
    "getrf_pivot_min": ("if (fabs(AT(T, ld, r, j)) > fabs(AT(T, ld, p, j))) p = r;",
                        "if (fabs(AT(T, ld, r, j)) < fabs(AT(T, ld, p, j))) p = r;"),
    "getrf_swap_partial": ("if (p != j) swap_rows(T, ld, j, p, 0, b);", "if (p != j) swap_rows(T, ld, j, p, j, b);"),
    "gessm_no_swap": ("if (ipiv[j] != j) swap_rows(X, ldx, j, ipiv[j], 0, nc);", "(void)ipiv;"),
    "tstrf_ties_to_a": ("if (fabs(AT(At, lda, r, j)) > best) {", "if (fabs(AT(At, lda, r, j)) >= best) {"),
    "tstrf_keeps_multipliers": ("Lup[(j - l0) * b + c] = AT(At, lda, p, c);\n                    AT(At, lda, p, c) = 0.0;",
                                "Lup[(j - l0) * b + c] = AT(At, lda, p, c);"),
    "tstrf_no_lup_update": ("for (int64_t q = l0; q < r; ++q) AT(Ut, ldu, r, c) -= Lup[(r - l0) * b + q] * AT(Ut, ldu, q, c);",
                            "(void)0;"),
    "tstrf_swap_from_panel": ("for (int64_t c = j; c < b; ++c) {\n                    const double t = AT(Ut, ldu, j, c);",
                              "for (int64_t c = j + 1; c < b; ++c) {\n                    const double t = AT(Ut, ldu, j, c);"),
    "ssssm_sign": ("for (int64_t r = 0; r < b; ++r) AT(X2, ld2, r, c) -= AT(L2, ldl, r, q) * AT(X1, ld1, q, c);",
                   "for (int64_t r = 0; r < b; ++r) AT(X2, ld2, r, c) += AT(L2, ldl, r, q) * AT(X1, ld1, q, c);"),
    "solve_skips_ssssm": ("ssssm_tile(b, s, nrhs, Lik, ldf,", "if (0) ssssm_tile(b, s, nrhs, Lik, ldf,"),
}


def _build_lu_mutant(tmp, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "lu.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path_c = os.path.join(tmp, f"{name}.c")
    path_so = os.path.join(tmp, f"lib{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", "-w", "-o", path_so, path_c,
                    "-lm"], check=True)
    return path_so


def test_lu_mutants_are_caught():
    tmp = tempfile.mkdtemp(prefix="lu_mut_")
    try:
        survivors = []
        for name, (old, new) in MUTANTS.items():
            O = oracle.LUOracle(_build_lu_mutant(tmp, name, old, new))
            caught = False
            for check in BATTERY:
                try:
                    check(O)
                except (AssertionError, ValueError, np.linalg.LinAlgError, ZeroDivisionError, FloatingPointError):
                    caught = True
                    break
            if not caught:
                survivors.append(name)
        assert not survivors, f"planted mistakes not caught by any pin: {survivors}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
