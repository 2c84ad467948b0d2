"""Oracles for the tiled Householder QR and the tiled Cholesky factorisation:
TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library never does, and nothing here imports the
library: the two share no code.

``oracle.c`` holds the arithmetic (unblocked Householder QR, application of
Q and Q^T, back substitution, least squares), ``cholesky.c`` the plain
column-by-column Cholesky factorisation and its solve, ``lu.c`` the tiled LU
factorisation with tiled pairwise pivoting (Algorithm 3's steps) and its
solve.  This module marshals
numpy arrays into them.  The error measures used to assess a factorisation or a
solution (``r_diff``, ``beta_fact``, ``beta_orth``, ``eta_inf``, ``eta_ls``)
are defined in ``metrics.py`` and re-exported here.
"""
import ctypes
import os

import numpy as np

from . import build as _build

class Oracle:
    """The C oracle loaded from one shared library (the default build, or a
    copy the mutation tests compile with a planted mistake)."""

    def __init__(self, path=None):
        if path is None:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = ctypes.CDLL(path)
        i64, dp, ci = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.oracle_geqr2.argtypes = [i64, i64, dp, i64, dp]
        L.oracle_geqr2.restype = ci
        for f in (L.oracle_apply_qt, L.oracle_apply_q):
            f.argtypes = [i64, i64, i64, dp, i64, dp, dp, i64]
            f.restype = ci
        L.oracle_trsv_upper.argtypes = [i64, dp, i64, i64, dp, i64]
        L.oracle_trsv_upper.restype = ci
        L.oracle_lstsq.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64]
        L.oracle_lstsq.restype = ci
        self.L = L

    def geqr2(self, A):
        """Householder QR of A (m x n).  Returns (F, tau) with F in LAPACK
        storage: R in the upper triangle, reflector tails below the diagonal."""
        F = _fortran(A)
        m, n = F.shape
        tau = np.zeros(max(min(m, n), 1))
        info = self.L.oracle_geqr2(m, n, _ptr(F), max(m, 1), _ptr(tau))
        if info != 0:
            raise ValueError(f"oracle_geqr2 info={info}")
        return F, tau[: min(m, n)]

    def _apply(self, fn, F, tau, B):
        m, n = F.shape
        B = _fortran(B.reshape(m, -1) if B.ndim == 1 else B)
        t = np.ascontiguousarray(tau, dtype=np.float64)
        if t.size == 0:
            t = np.zeros(1)
        info = fn(m, n, B.shape[1], _ptr(F), max(m, 1), _ptr(t), _ptr(B), max(m, 1))
        if info != 0:
            raise ValueError(f"oracle apply info={info}")
        return B

    def apply_qt(self, F, tau, B):
        """Q^T B for the factorisation (F, tau)."""
        return self._apply(self.L.oracle_apply_qt, F, tau, B)

    def apply_q(self, F, tau, B):
        """Q B for the factorisation (F, tau)."""
        return self._apply(self.L.oracle_apply_q, F, tau, B)

    def trsv_upper(self, R, C):
        n = R.shape[0]
        R = _fortran(R)
        C = _fortran(C.reshape(n, -1) if C.ndim == 1 else C)
        info = self.L.oracle_trsv_upper(n, _ptr(R), max(n, 1), C.shape[1], _ptr(C), max(n, 1))
        if info != 0:
            raise ValueError(f"oracle_trsv_upper info={info}")
        return C

    def lstsq(self, A, B):
        """Least-squares solution X of min ||B - A X|| (m >= n, full rank) and
        the residual B - A X, both from the oracle's Householder QR."""
        A = _fortran(A)
        m, n = A.shape
        vec = B.ndim == 1
        B = _fortran(B.reshape(m, -1) if vec else B)
        nrhs = B.shape[1]
        X = np.zeros((max(n, 1), nrhs), order="F")
        Res = np.zeros((max(m, 1), nrhs), order="F")
        info = self.L.oracle_lstsq(m, n, nrhs, _ptr(A), max(m, 1), _ptr(B), max(m, 1),
                                   _ptr(X), max(n, 1), _ptr(Res), max(m, 1))
        if info != 0:
            raise ValueError(f"oracle_lstsq info={info}")
        X, Res = X[:n], Res[:m]
        if vec:
            return X[:, 0], Res[:, 0]
        return X, Res

    def thin_q(self, F, tau):
        m, n = F.shape
        k = min(m, n)
        E = np.zeros((m, k))
        E[np.arange(k), np.arange(k)] = 1.0
        return self.apply_q(F, tau, E)

    def beta_fact(self, A, F, tau):
        """beta_fact of this oracle's own factorisation (Q [R; 0] by apply_q)."""
        m, n = A.shape
        RR = np.zeros((m, n))
        k = min(m, n)
        RR[:k] = r_factor(F)
        return beta_fact(A, self.apply_q(F, tau, RR))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran(a):
    return np.array(a, dtype=np.float64, order="F", copy=True)


def r_factor(F):
    """The min(m,n) x n upper-trapezoidal R held in F."""
    m, n = F.shape
    k = min(m, n)
    return np.triu(F[:k, :])


_default = None


def default():
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def geqr2(A):
    return default().geqr2(A)


def apply_qt(F, tau, B):
    return default().apply_qt(F, tau, B)


def apply_q(F, tau, B):
    return default().apply_q(F, tau, B)


def trsv_upper(R, C):
    return default().trsv_upper(R, C)


def lstsq(A, B):
    return default().lstsq(A, B)


def thin_q(F, tau):
    return default().thin_q(F, tau)


def oracle_beta_fact(A, F, tau):
    return default().beta_fact(A, F, tau)


# ----------------------------------------------------------------- Cholesky

class CholOracle:
    """The C Cholesky oracle (cholesky.c) from one shared library (the
    default build, or a mutant the tests compile)."""

    def __init__(self, path=None):
        if path is None:
            path = _build.CHOL_LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.CHOL_SRC):
                _build.build(force=False)
        L = ctypes.CDLL(path)
        i64, dp, ci = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.oracle_potrf_lower.argtypes = [i64, dp, i64]
        L.oracle_potrf_lower.restype = ci
        L.oracle_potrs_lower.argtypes = [i64, i64, dp, i64, dp, i64]
        L.oracle_potrs_lower.restype = ci
        self.L = L

    def potrf(self, A):
        """(L, info): the Cholesky factor of the lower triangle of A (L lower
        triangular, zeros above) and 0; or, when the leading minor of order
        info > 0 is not positive definite, the partial result and info."""
        F = _fortran(A)
        n = F.shape[0]
        info = self.L.oracle_potrf_lower(n, _ptr(F), max(n, 1))
        if info < 0:
            raise ValueError(f"oracle_potrf_lower info={info}")
        return np.tril(F), info

    def potrs(self, Lf, B):
        """X with L L^T X = B for the factor of potrf."""
        F = _fortran(Lf)
        n = F.shape[0]
        vec = B.ndim == 1
        X = _fortran(B.reshape(n, -1) if vec else B)
        info = self.L.oracle_potrs_lower(n, X.shape[1], _ptr(F), max(n, 1), _ptr(X), max(n, 1))
        if info != 0:
            raise ValueError(f"oracle_potrs_lower info={info}")
        return X[:, 0] if vec else X


_chol = None


def chol_default():
    global _chol
    if _chol is None:
        _chol = CholOracle()
    return _chol


def potrf(A):
    return chol_default().potrf(A)


def potrs(Lf, B):
    return chol_default().potrs(Lf, B)


# ------------------------------------------------------------------- LU

class LUOracle:
    """The C tiled-LU oracle (lu.c) from one shared library (the default
    build, or a mutant the tests compile)."""

    def __init__(self, path=None):
        if path is None:
            path = _build.LU_LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.LU_SRC):
                _build.build(force=False)
        L = ctypes.CDLL(path)
        i64, dp, ci = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_tile_lu.argtypes = [i64, i64, i64, dp, i64, dp, ip]
        L.oracle_tile_lu.restype = ci
        L.oracle_tile_lu_solve.argtypes = [i64, i64, i64, dp, i64, dp, ip, i64, dp, i64]
        L.oracle_tile_lu_solve.restype = ci
        self.L = L

    def tile_lu(self, A, b, s):
        """Algorithm 3 on A (n x n, n = p b): (F, Lup, piv, info) with F the
        factored matrix (U above, L_kk and the TSTRF multipliers below), Lup
        (p, p, s, b) and piv (p, p, b) indexed [k][i], info 0 or the 1-based
        column that had no nonzero pivot."""
        F = _fortran(A)
        n = F.shape[0]
        p = n // b if b else 0
        Lup = np.zeros((max(p, 1), max(p, 1), s, b))
        piv = np.zeros((max(p, 1), max(p, 1), b), dtype=np.int32)
        info = self.L.oracle_tile_lu(n, b, s, _ptr(F), max(n, 1), _ptr(Lup),
                                     piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if info < 0:
            raise ValueError(f"oracle_tile_lu info={info}")
        return F, Lup, piv, info

    def tile_lu_solve(self, F, Lup, piv, b, s, B):
        n = F.shape[0]
        vec = B.ndim == 1
        X = _fortran(B.reshape(n, -1) if vec else B)
        info = self.L.oracle_tile_lu_solve(n, b, s, _ptr(_fortran(F)), max(n, 1), _ptr(np.ascontiguousarray(Lup)),
                                           np.ascontiguousarray(piv).ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           X.shape[1], _ptr(X), max(n, 1))
        if info != 0:
            raise ValueError(f"oracle_tile_lu_solve info={info}")
        return X[:, 0] if vec else X


_lu = None


def lu_default():
    global _lu
    if _lu is None:
        _lu = LUOracle()
    return _lu


def tile_lu(A, b, s):
    return lu_default().tile_lu(A, b, s)


def tile_lu_solve(F, Lup, piv, b, s, B):
    return lu_default().tile_lu_solve(F, Lup, piv, b, s, B)


# ----------------------------------------------------------------- metrics
# The error measures live in metrics.py (pure numpy) and are re-exported here.
from .metrics import beta_fact, beta_orth, eta_inf, eta_ls, r_diff, row_signs  # noqa: E402,F401
