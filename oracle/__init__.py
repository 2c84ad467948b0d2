"""Oracle for the tiled Householder QR: TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library never does, and nothing here imports the
library: the two share no code.

``oracle.c`` holds the arithmetic (unblocked Householder QR, application of
Q and Q^T, back substitution, least squares).  This module marshals numpy
arrays into it and adds the error measures used to assess a factorisation:

* ``beta_fact``  = ||A - Q [R; 0]||_F / ||A||_F       (factorisation residual)
* ``beta_orth``  = ||Q_thin^T Q_thin - I_n||_F        (loss of orthogonality)
* ``eta_inf``    = ||b - A x||_inf / (||A||_inf ||x||_inf), the square-system
  backward error of the paper (Section 3.2.4, the solution backward error of
  the stability experiments),
* ``eta_ls``     = ||A^T (b - A x)||_2 / (||A||_F (||A||_F ||x||_2 + ||b||_2)),
  a normwise least-squares backward-error measure (the paper defines only the
  square-system one; this is the reading used for m > n).
* ``r_diff``     = ||D_g R_g - D_o R_o||_F / ||R_o||_F with D = diag(sign R_jj),
  sign(0) = +1: R compared up to row signs, since R of a full-rank matrix is
  unique up to the signs of its rows.
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


# ----------------------------------------------------------------- metrics

def row_signs(R):
    d = np.sign(np.diag(R)).astype(np.float64)
    d[d == 0] = 1.0
    return d


def r_diff(R_test, R_ref):
    """||D_t R_t - D_r R_r||_F / ||R_r||_F  (R up to row signs)."""
    k = min(R_ref.shape)
    Rt = R_test[:k] * row_signs(R_test)[:, None]
    Rr = R_ref[:k] * row_signs(R_ref)[:, None]
    den = np.linalg.norm(Rr)
    return float(np.linalg.norm(Rt - Rr) / (den if den > 0 else 1.0))


def beta_fact(A, QR):
    """||A - QR||_F / ||A||_F given the product QR already formed."""
    den = np.linalg.norm(A)
    return float(np.linalg.norm(A - QR) / (den if den > 0 else 1.0))


def beta_orth(Qthin):
    n = Qthin.shape[1]
    return float(np.linalg.norm(Qthin.T @ Qthin - np.eye(n)))


def eta_inf(A, x, b):
    """Square-system normwise backward error in the infinity norm."""
    r = b - A @ x
    den = np.linalg.norm(A, np.inf) * np.linalg.norm(x, np.inf)
    return float(np.linalg.norm(r, np.inf) / den) if den > 0 else float("inf")


def eta_ls(A, x, b):
    """Normwise least-squares backward-error measure for one right-hand side."""
    r = b - A @ x
    nA = np.linalg.norm(A)
    den = nA * (nA * np.linalg.norm(x) + np.linalg.norm(b))
    return float(np.linalg.norm(A.T @ r) / den) if den > 0 else 0.0
