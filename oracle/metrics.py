"""Error measures of the oracle: TEST INFRASTRUCTURE ONLY.

Plain numpy, FP64, one definition per function, no blocking or reordering.
They measure a factorisation or a solution, whichever path produced it:

* ``r_diff``     ||D_t R_t - D_r R_r||_F / ||R_r||_F with D = diag(sign R_jj)
                 and sign(0) = +1.  R of a full-rank matrix is unique up to
                 the signs of its rows (the tiled algorithm of Section 3.2.1
                 flips them relative to the unblocked one), so R is compared
                 after making every diagonal entry non-negative.
* ``beta_fact``  ||A - Q R||_F / ||A||_F, the factorisation backward error
                 (Section 3.2.4 measures the factorisation this way, in the
                 infinity norm for LU; the Frobenius norm is taken here).
* ``beta_orth``  ||Q^T Q - I_n||_F for the n columns of Q given: the loss of
                 orthogonality of the thin factor.
* ``eta_inf``    ||b - A x||_inf / (||A||_inf ||x||_inf), the backward error of
                 a solution that Section 3.2.4 uses for square systems.
* ``eta_ls``     ||A^T (b - A x)||_2 / (||A||_F (||A||_F ||x||_2 + ||b||_2)), a
                 normwise measure for least squares (m > n), where b - A x does
                 not vanish at the solution; the paper defines only the
                 square-system measure, so this is a reading, zero exactly at
                 the least-squares solution.

Each is pinned in tests/test_oracle_pins.py by values worked out by hand
(tests/golden/metrics.txt) and by planted mistakes that those values catch.
"""
import numpy as np


def row_signs(R):
    """sign(R_jj) per row with sign(0) = +1."""
    d = np.sign(np.diag(R)).astype(np.float64)
    d[d == 0] = 1.0
    return d


def r_diff(R_test, R_ref):
    """||D_t R_t - D_r R_r||_F / ||R_r||_F  (R up to row signs)."""
    k = min(R_ref.shape)
    Rt = R_test[:k] * row_signs(R_test)[:k, None]
    Rr = R_ref[:k] * row_signs(R_ref)[:k, None]
    den = np.linalg.norm(Rr)
    return float(np.linalg.norm(Rt - Rr) / (den if den > 0 else 1.0))


def beta_fact(A, QR):
    """||A - QR||_F / ||A||_F given the product QR already formed."""
    den = np.linalg.norm(A)
    return float(np.linalg.norm(A - QR) / (den if den > 0 else 1.0))


def beta_orth(Qthin):
    """||Q^T Q - I_n||_F for an m x n matrix Q."""
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
