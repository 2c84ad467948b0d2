"""Pins of the CPU oracle against facts fixed by the mathematics, not by itself.

Each check would fail on a plausible mistake in the oracle: a wrong reflector
sign (closed forms, exact integer case), a dropped tau or a wrong index in the
update (Q^T A = [R; 0], R^T R = A^T A, brute force), a reversed application
order (Q^T Q z = z, thin Q vs LAPACK), a wrong back substitution (least
squares vs LAPACK).  ``test_mutants_are_caught`` plants such mistakes in a
copy of the oracle and checks that the battery catches every one.
"""
import os
import re
import shutil
import subprocess
import tempfile

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from conftest import ROOT, load_golden
from paper_0709_1272_amd import synth

EPS = np.finfo(np.float64).eps


# ------------------------------------------------------------------ battery
# Each check takes an oracle.Oracle instance so the mutation test can rerun
# the same battery against a planted-mistake build.

def check_2x2_closed_form(O):
    g = load_golden("householder_2x2.txt")
    A = np.array(g["A"]).reshape(2, 2)
    F, tau = O.geqr2(A)
    R = oracle.r_factor(F)
    np.testing.assert_allclose(R.ravel(), g["R"], rtol=2 * EPS, atol=2 * EPS)
    np.testing.assert_allclose(tau, g["tau"], rtol=2 * EPS, atol=0)
    np.testing.assert_allclose([1.0, F[1, 0]], g["v"], rtol=2 * EPS, atol=0)
    # H e_1, H e_2 from the stored reflector, compared with the printed H.
    H = O.apply_q(F[:, :1].copy(), tau[:1], np.eye(2))
    np.testing.assert_allclose(H.ravel(), g["H"], rtol=4 * EPS, atol=4 * EPS)


def check_3x3_integer(O):
    g = load_golden("householder_3x3_integer.txt")
    A = np.array(g["A"]).reshape(3, 3)
    F, tau = O.geqr2(A)
    np.testing.assert_allclose(oracle.r_factor(F).ravel(), g["R"], rtol=0, atol=16 * EPS)
    # Q = -M/3 exactly, so Q^T A = R and Q (R) = A.
    QR = O.apply_q(F, tau, oracle.r_factor(F))
    np.testing.assert_allclose(QR, A, rtol=0, atol=32 * EPS)


def check_single_column(O):
    rng = np.random.default_rng(11)
    for a0 in (2.5, -2.5, 0.0, -0.0):
        a = rng.standard_normal(7)
        a[0] = a0
        F, tau = O.geqr2(a.reshape(-1, 1))
        sgn = 1.0 if a0 >= 0 else -1.0      # sign(+0) = sign(-0) = +1
        ref = -sgn * np.linalg.norm(a)
        assert abs(F[0, 0] - ref) <= 4 * EPS * abs(ref), (a0, F[0, 0], ref)


def check_upper_triangular_is_fixed(O):
    rng = np.random.default_rng(3)
    A = np.triu(rng.standard_normal((9, 6)))
    A[2, 2] = -abs(A[2, 2])   # a negative diagonal entry must stay untouched too
    F, tau = O.geqr2(A)
    assert np.all(tau == 0.0)
    assert np.array_equal(F, A)


def check_power_of_two_scaling(O):
    A = synth.uniform(5, 13, 9)
    F0, t0 = O.geqr2(A)
    for e in (-20, 7, 30):
        F1, t1 = O.geqr2(A * 2.0 ** e)
        R0, R1 = oracle.r_factor(F0), oracle.r_factor(F1)
        assert np.array_equal(R1, R0 * 2.0 ** e)
        assert np.array_equal(np.tril(F1, -1), np.tril(F0, -1))
        assert np.array_equal(t1, t0)


def check_gram(O):
    A = synth.uniform(8, 40, 25)
    F, _ = O.geqr2(A)
    R = oracle.r_factor(F)
    G = A.T @ A
    assert np.linalg.norm(R.T @ R - G) <= 64 * EPS * np.linalg.norm(G)


def check_qt_a_is_r(O):
    A = synth.uniform(9, 30, 17)
    F, tau = O.geqr2(A)
    QtA = O.apply_qt(F, tau, A)
    RR = np.zeros_like(A)
    RR[:17] = oracle.r_factor(F)
    assert np.linalg.norm(QtA - RR) <= 64 * EPS * np.linalg.norm(A)


def check_q_roundtrip(O):
    A = synth.uniform(10, 21, 13)
    F, tau = O.geqr2(A)
    z = np.random.default_rng(1).standard_normal((21, 3))
    back = O.apply_qt(F, tau, O.apply_q(F, tau, z))
    assert np.linalg.norm(back - z) <= 64 * EPS * np.linalg.norm(z)
    # Q^T applied twice is not the identity unless the order is right:
    Qt = O.apply_qt(F, tau, np.eye(21))
    Q = O.apply_q(F, tau, np.eye(21))
    assert np.linalg.norm(Qt - Q.T) <= 64 * EPS * 21


def check_thin_q_vs_lapack(O):
    A = synth.uniform(12, 24, 10)
    F, tau = O.geqr2(A)
    Qo = O.thin_q(F, tau)
    Ql, Rl = np.linalg.qr(A)          # LAPACK dgeqrf + dorgqr
    s = np.sign(np.diag(Rl)) * np.sign(np.diag(oracle.r_factor(F)))
    assert np.linalg.norm(Qo - Ql * s[None, :]) <= 256 * EPS * np.sqrt(10)


def check_r_vs_lapack(O):
    for (m, n, seed) in ((50, 50, 0), (77, 31, 1), (20, 35, 2)):
        A = synth.uniform(seed, m, n)
        F, tau = O.geqr2(A)
        h, tau_l = np.linalg.qr(A, mode="raw")   # LAPACK storage, transposed
        Fl = h.T
        Rl = np.triu(Fl[: min(m, n)])
        R = oracle.r_factor(F)
        # Same reflector convention as LAPACK: the signs agree too.
        assert np.array_equal(np.sign(np.diag(R)), np.sign(np.diag(Rl)))
        assert np.linalg.norm(R - Rl) <= 64 * EPS * np.linalg.norm(Rl)
        np.testing.assert_allclose(tau, tau_l, rtol=1e-13, atol=1e-15)


def check_brute_force_mpmath(O):
    mpmath.mp.dps = 50
    rng = np.random.default_rng(21)
    for (m, n) in ((3, 3), (5, 4), (8, 8), (8, 3), (6, 1)):
        A = rng.uniform(-1, 1, (m, n))
        F, _ = O.geqr2(A)
        R = oracle.r_factor(F)
        R = R * oracle.row_signs(R)[:, None]
        # R with a positive diagonal is the Cholesky factor of A^T A
        # (computed here at 50 digits from the exact double entries of A).
        Am = mpmath.matrix(A.tolist())
        L = mpmath.cholesky(Am.T * Am)
        Rm = np.array([[float(L[j, i]) for j in range(n)] for i in range(n)])
        kappa = np.linalg.cond(A)
        assert np.linalg.norm(R - Rm) <= 64 * EPS * kappa * np.linalg.norm(Rm), (m, n)


def check_lstsq_vs_lapack(O):
    A, b, x_true = synth.svd_matrix(4, 60, 20, 1e4)
    x, r = O.lstsq(A, b)
    xl = scipy.linalg.lstsq(A, b, lapack_driver="gelsy")[0]
    assert np.linalg.norm(x - xl) <= 1e4 * 64 * EPS * np.linalg.norm(xl)
    np.testing.assert_allclose(r, b - A @ x, rtol=0, atol=64 * EPS * np.linalg.norm(b))
    assert oracle.eta_ls(A, x, b) <= 1e-15


def check_invariants_moderate(O):
    A = synth.uniform(0, 256, 256)
    F, tau = O.geqr2(A)
    assert O.beta_fact(A, F, tau) <= 1e-14
    assert oracle.beta_orth(O.thin_q(F, tau)) <= 1e-14 * 256


BATTERY = [check_2x2_closed_form, check_3x3_integer, check_single_column,
           check_upper_triangular_is_fixed, check_power_of_two_scaling, check_gram,
           check_qt_a_is_r, check_q_roundtrip, check_thin_q_vs_lapack, check_r_vs_lapack,
           check_brute_force_mpmath, check_lstsq_vs_lapack, check_invariants_moderate]


@pytest.mark.parametrize("check", BATTERY, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check(oracle.default())


# ------------------------------------------------------------ degenerate cases

def test_empty_and_bad_arguments():
    O = oracle.default()
    F, tau = O.geqr2(np.zeros((0, 3)))
    assert tau.size == 0
    F, tau = O.geqr2(np.zeros((4, 0)))
    assert tau.size == 0
    import ctypes
    buf = np.zeros(4)
    p = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert O.L.oracle_geqr2(-1, 2, p, 1, p) == -1
    assert O.L.oracle_geqr2(2, -1, p, 2, p) == -2
    assert O.L.oracle_geqr2(3, 1, p, 2, p) == -4


def test_zero_column_gives_identity_reflector():
    A = synth.uniform(2, 10, 4)
    A[:, 1] = A[:, 0] * 3.0      # rank deficient: column 1 is reduced to zero below row 1
    F, tau = oracle.geqr2(A)
    assert abs(F[1, 1]) <= 64 * EPS * np.linalg.norm(A)
    assert np.all(np.isfinite(F))


def test_wide_matrix():
    A = synth.uniform(6, 7, 12)
    F, tau = oracle.geqr2(A)
    assert tau.size == 7
    RR = oracle.r_factor(F)
    QR = oracle.apply_q(F, tau, RR)
    assert np.linalg.norm(QR - A) <= 64 * EPS * np.linalg.norm(A)


def test_singular_triangle_reported():
    R = np.triu(np.ones((3, 3)))
    R[1, 1] = 0.0
    with pytest.raises(ValueError):
        oracle.trsv_upper(R, np.ones(3))


# ---------------------------------------------------------------- mutations

MUTANTS = {
    "beta_sign": ("double beta = (alpha >= 0.0) ? -h : h;", "double beta = (alpha >= 0.0) ? h : -h;"),
    "dropped_tau": ("double tw = t * w;\n            AT(A, lda, j, c) -= tw;",
                    "double tw = w;\n            AT(A, lda, j, c) -= tw;"),
    "dot_index": ("w += x[r] * AT(A, lda, j + 1 + r, c);", "w += x[r] * AT(A, lda, j + r, c);"),
    "tau_formula": ("double t = (beta - alpha) / beta;", "double t = (alpha - beta) / beta;"),
    "vector_scale": ("double scal = 1.0 / (alpha - beta);", "double scal = 1.0 / (beta - alpha);"),
    "apply_order": ("for (int64_t j = 0; j < kmax; ++j) apply_reflector(",
                    "for (int64_t j = kmax - 1; j >= 0; --j) apply_reflector("),
    "norm_square": ("return scale * sqrt(sum);", "return scale * sum;"),
    "backsub_index": ("s -= AT(R, ldr, i, k) * AT(C, ldc, k, c);", "s -= AT(R, ldr, k, i) * AT(C, ldc, k, c);"),
    "zero_norm_flip": ("tau[j] = 0.0;           /* H_j = I", "AT(A, lda, j, j) = -alpha; tau[j] = 0.0; /* H_j = I"),
}


def _build_mutant(tmp, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path_c = os.path.join(tmp, f"{name}.c")
    path_so = os.path.join(tmp, f"lib{name}.so")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", "-o",
                    path_so, path_c, "-lm"], check=True)
    return path_so


def test_mutants_are_caught():
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        survivors = []
        for name, (old, new) in MUTANTS.items():
            O = oracle.Oracle(_build_mutant(tmp, name, old, new))
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


# ------------------------------------------------------------ metric pins
# The error measures of oracle/metrics.py against values worked out by hand
# from their definitions (tests/golden/metrics.txt).  Each check takes a
# namespace holding the metric functions, so that the mutation test below can
# run the same checks on a copy with a planted mistake.

def _mat(g, key, rows):
    v = np.array(g[key])
    return v.reshape(rows, -1)


def check_metric_r_diff(M):
    g = load_golden("metrics.txt")
    for case in ("rdiff1", "rdiff2", "rdiff3"):
        got = M.r_diff(_mat(g, case + "_test", 2), _mat(g, case + "_ref", 2))
        assert abs(got - g[case][0]) <= 4 * EPS, (case, got, g[case][0])


def check_metric_beta_orth(M):
    g = load_golden("metrics.txt")
    for case in ("orth1", "orth2"):
        got = M.beta_orth(_mat(g, case + "_q", 3))
        assert abs(got - g[case][0]) <= 8 * EPS * max(1.0, g[case][0]), (case, got)


def check_metric_beta_fact(M):
    g = load_golden("metrics.txt")
    for case in ("fact1", "fact2"):
        got = M.beta_fact(_mat(g, case + "_a", 2), _mat(g, case + "_qr", 2))
        assert abs(got - g[case][0]) <= 4 * EPS, (case, got)


def check_metric_eta_inf(M):
    g = load_golden("metrics.txt")
    A, x = _mat(g, "inf1_a", 2), np.array(g["inf1_x"])
    got = M.eta_inf(A, x, np.array(g["inf1_b"]))
    assert abs(got - g["inf1"][0]) <= 4 * EPS, got
    assert M.eta_inf(A, x, np.array(g["inf2_b"])) == g["inf2"][0]


def check_metric_eta_ls(M):
    g = load_golden("metrics.txt")
    A, b = _mat(g, "ls1_a", 3), np.array(g["ls1_b"])
    assert M.eta_ls(A, np.array(g["ls1_xopt"]), b) == g["ls1_xopt_eta"][0]
    got = M.eta_ls(A, np.array(g["ls1_x"]), b)
    assert abs(got - g["ls1"][0]) <= 4 * EPS, got
    A, b = _mat(g, "ls2_a", 3), np.array(g["ls2_b"])
    got = M.eta_ls(A, np.array(g["ls2_x"]), b)
    assert abs(got - g["ls2"][0]) <= 1e-14, got
    assert M.eta_ls(A, np.array(g["ls2_xopt"]), b) <= 1e-16


METRIC_BATTERY = [check_metric_r_diff, check_metric_beta_orth, check_metric_beta_fact,
                  check_metric_eta_inf, check_metric_eta_ls]


@pytest.mark.parametrize("check", METRIC_BATTERY, ids=lambda f: f.__name__)
def test_metric_pin(check):
    from oracle import metrics
    check(metrics)


METRIC_MUTANTS = {
    "unsigned_rows": ("Rt = R_test[:k] * row_signs(R_test)[:k, None]", "Rt = R_test[:k]"),
    "unsigned_ref": ("Rr = R_ref[:k] * row_signs(R_ref)[:k, None]", "Rr = R_ref[:k]"),
    "sign_of_zero": ("d[d == 0] = 1.0", "pass"),
    "r_diff_unnormalised": ("return float(np.linalg.norm(Rt - Rr) / (den if den > 0 else 1.0))",
                            "return float(np.linalg.norm(Rt - Rr))"),
    "orth_outer_gram": ("np.linalg.norm(Qthin.T @ Qthin - np.eye(n))",
                        "np.linalg.norm(Qthin @ Qthin.T - np.eye(Qthin.shape[0]))"),
    "orth_two_norm": ("np.linalg.norm(Qthin.T @ Qthin - np.eye(n))", "np.linalg.norm(Qthin.T @ Qthin - np.eye(n), 2)"),
    "fact_wrong_denominator": ("den = np.linalg.norm(A)\n    return float(np.linalg.norm(A - QR)",
                               "den = np.linalg.norm(QR)\n    return float(np.linalg.norm(A - QR)"),
    "inf_one_norm_of_a": ("np.linalg.norm(A, np.inf) * np.linalg.norm(x, np.inf)",
                          "np.linalg.norm(A, 1) * np.linalg.norm(x, np.inf)"),
    "inf_two_norm_of_r": ("float(np.linalg.norm(r, np.inf) / den)", "float(np.linalg.norm(r) / den)"),
    "inf_two_norm_of_x": ("np.linalg.norm(A, np.inf) * np.linalg.norm(x, np.inf)",
                          "np.linalg.norm(A, np.inf) * np.linalg.norm(x)"),
    "ls_dropped_b": ("den = nA * (nA * np.linalg.norm(x) + np.linalg.norm(b))", "den = nA * (nA * np.linalg.norm(x))"),
    "ls_spectral_norm": ("nA = np.linalg.norm(A)\n", "nA = np.linalg.norm(A, 2)\n"),
    "ls_residual_not_projected": ("float(np.linalg.norm(A.T @ r) / den)", "float(np.linalg.norm(r) / den)"),
    "ls_residual_sign": ("r = b - A @ x\n    nA", "r = b + A @ x\n    nA"),
}


def test_metric_mutants_are_caught():
    import types
    src = open(os.path.join(ROOT, "oracle", "metrics.py")).read()
    survivors = []
    for name, (old, new) in METRIC_MUTANTS.items():
        assert src.count(old) == 1, f"mutation anchor for {name} not unique"
        mod = types.ModuleType("metrics_" + name)
        exec(compile(src.replace(old, new), f"metrics_{name}.py", "exec"), mod.__dict__)
        caught = False
        for check in METRIC_BATTERY:
            try:
                check(mod)
            except (AssertionError, ValueError, np.linalg.LinAlgError):
                caught = True
                break
        if not caught:
            survivors.append(name)
    assert not survivors, f"planted mistakes in the metrics not caught by any pin: {survivors}"
