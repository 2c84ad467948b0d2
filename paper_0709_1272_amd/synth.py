"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers; it holds none of the factorisation's
arithmetic.  Every generator uses numpy's PCG64 (``default_rng(seed)``) and
draws an (m, n) array in C order before it is copied to column-major, so the
values do not depend on the storage layout.  The same host bytes feed the
oracle and the GPU path.

Workloads (the paper's QR runs use random dense matrices; its stability
experiments draw entries with randn):

* ``uniform``      entries i.i.d. uniform(-1, 1)            (square FP64 QR)
* ``svd_matrix``   A = U diag(s) V^T with random orthogonal U, V and s
                   log-spaced from 1 to 1/kappa              (least squares)
* ``svd_matrix_haar_device``  the same construction at sizes where a host QR
                   of a Gaussian matrix is too slow: U and V are the Q factors
                   of Gaussian matrices (Haar-distributed, column signs fixed)
                   computed on the GPU by torch.linalg.qr   (large least squares)
* ``svd_matrix_device``  the same spectrum with structured orthogonal factors:
                   U and V are products of normalised Walsh-Hadamard
                   transforms, random signs and random permutations (dense and
                   exactly orthogonal), built on the GPU with torch
* ``batch_sizes`` / ``batch_matrices``  m ~ U{32..768}, n ~ U{16..m},
                   entries N(0, 1)                           (batched QR)
* ``batch_ls``     the same matrices, then one consistent right-hand side
                   each, b_i = A_i x_i with x_i ~ N(0, 1)    (batched least squares)
* ``spd_matrix``   A = U diag(s) U^T, symmetric positive definite with
                   eigenvalues log-spaced from 1 to 1/kappa  (Cholesky)
* ``spd_matrix_device``  the same spectrum with the structured orthogonal U of
                   ``svd_matrix_device``, built on the GPU   (large Cholesky)
"""
import numpy as np


def uniform(seed, m, n):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, (m, n)))


def normal(seed, m, n):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)))


def _orthonormal_columns(rng, m, n):
    """Orthonormal m x n basis from the QR of a Gaussian matrix (input
    construction only), column signs fixed so that diag(R) > 0."""
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def svd_matrix(seed, m, n, kappa, nrhs=1, noise=1e-6):
    """(A, b, x_true): A = U diag(s) V^T, s = logspace(0, -log10(kappa), n),
    x_true ~ N(0,1) (n x nrhs), b = A x_true + noise * N(0,1) (m x nrhs).
    With nrhs == 1, x_true and b are vectors."""
    rng = np.random.default_rng(seed)
    U = _orthonormal_columns(rng, m, n)
    V = _orthonormal_columns(rng, n, n)
    s = np.logspace(0.0, -np.log10(kappa), n)
    A = np.asfortranarray((U * s[None, :]) @ V.T)
    x = rng.standard_normal((n, nrhs))
    b = A @ x + noise * rng.standard_normal((m, nrhs))
    if nrhs == 1:
        return A, np.ascontiguousarray(b[:, 0]), np.ascontiguousarray(x[:, 0])
    return A, np.asfortranarray(b), np.asfortranarray(x)


def _hadamard(M, dim):
    """Normalised Walsh-Hadamard transform of M (torch, power-of-two size)
    along dimension `dim`, in log2(n) butterfly passes."""
    import torch
    n = M.shape[dim]
    x = M if dim == 0 else M.t()
    x = x.contiguous()
    cols = x.shape[1]
    h = 1
    while h < n:
        y = x.view(n // (2 * h), 2, h, cols)
        x = torch.stack((y[:, 0] + y[:, 1], y[:, 0] - y[:, 1]), dim=1).view(n, cols)
        h *= 2
    x = x * (1.0 / float(n) ** 0.5)
    return x if dim == 0 else x.t().contiguous()


def svd_matrix_device(seed, n, kappa, nrhs=1, noise=1e-6, device="cuda"):
    """(A, B, X) as torch tensors on `device`, A n x n with singular values
    logspace(0, -log10(kappa), n): A = U diag(s) V^T with U = H D1 P1 H D2 and
    V^T = H D3 P2 H D4 (H the normalised Walsh-Hadamard matrix, D random
    signs, P random permutations; n a power of two).  A is returned as a
    contiguous (n, n) tensor holding A column-major (that is, A^T row-major);
    X ~ N(0, 1) (n x nrhs) and B = A X + noise N(0, 1), both column-major
    (nrhs, n)."""
    import torch
    assert n & (n - 1) == 0, "n must be a power of two"
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sign = lambda: torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int64).to(torch.float64) * 2 - 1
    perm = lambda: torch.randperm(n, generator=g, device=device)
    d1, d2, d3, d4 = sign(), sign(), sign(), sign()
    p1, p2 = perm(), perm()
    s = torch.logspace(0.0, -float(torch.log10(torch.tensor(kappa))), n, dtype=torch.float64, device=device)
    # M = U diag(s): columns of diag(s) scaled by d2 ... built row by row
    M = torch.diag(s * d2)                      # D2 S
    M = _hadamard(M, 0)                         # H D2 S
    M = M[p1]                                   # P1 H D2 S
    M = M * d1[:, None]                         # D1 P1 H D2 S
    M = _hadamard(M, 0)                         # U S
    M = _hadamard(M, 1)                         # U S H
    M = M * d3[None, :]
    M = M[:, p2]
    M = _hadamard(M, 1)
    M = M * d4[None, :]                         # U S V^T
    X = torch.randn((n, nrhs), generator=g, device=device, dtype=torch.float64)
    B = M @ X + noise * torch.randn((n, nrhs), generator=g, device=device, dtype=torch.float64)
    return M.t().contiguous(), B.t().contiguous(), X.t().contiguous()


def svd_matrix_haar_device(seed, m, n, kappa, nrhs=1, noise=1e-6, device="cuda"):
    """(A, B, X) as torch tensors on `device`: A m x n = U diag(s) V^T with U
    (m x n) and V (n x n) the orthonormal factors of the QR of Gaussian
    matrices (Haar distributed once the column signs make diag(R) positive),
    computed on the GPU by torch.linalg.qr; s = logspace(0, -log10(kappa), n);
    X ~ N(0, 1) (n x nrhs); B = A X + noise N(0, 1) (m x nrhs).  A is returned
    as a contiguous (n, m) tensor holding A column-major; B (nrhs, m) and
    X (nrhs, n) column-major likewise.  Seeded with a torch generator on the
    device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar(rows, cols):
        G = torch.randn((rows, cols), generator=g, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(G)
        del G
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        del R
        return Q * d[None, :]

    U = haar(m, n)
    V = haar(n, n)
    s = torch.logspace(0.0, -float(torch.log10(torch.tensor(kappa, dtype=torch.float64))), n, dtype=torch.float64,
                       device=device)
    U.mul_(s[None, :])
    # A^T = V (U diag(s))^T, stored row-major: that is A column-major.
    At = V @ U.t()
    del U, V
    X = torch.randn((nrhs, n), generator=g, device=device, dtype=torch.float64)
    Bt = X @ At + noise * torch.randn((nrhs, m), generator=g, device=device, dtype=torch.float64)
    return At.contiguous(), Bt.contiguous(), X.contiguous()


def spd_matrix(seed, n, kappa=1e3):
    """Symmetric positive definite n x n: A = U diag(s) U^T with U the
    orthogonal factor of a Gaussian matrix and s = logspace(0, -log10 kappa, n);
    exactly symmetric (the mean of A and A^T), column-major."""
    rng = np.random.default_rng(seed)
    U = _orthonormal_columns(rng, n, n)
    s = np.logspace(0.0, -np.log10(kappa), n)
    A = (U * s[None, :]) @ U.T
    return np.asfortranarray((A + A.T) / 2.0)


def spd_matrix_device(seed, n, kappa=1e6, device="cuda"):
    """Symmetric positive definite n x n on `device` (n a power of two):
    A = U diag(s) U^T with U = H D1 P1 H D2 (H the normalised Walsh-Hadamard
    matrix, D random signs, P a random permutation) and
    s = logspace(0, -log10 kappa, n); returned as a contiguous (n, n) tensor
    (A is symmetric, so row- and column-major agree), exactly symmetric."""
    import torch
    assert n & (n - 1) == 0, "n must be a power of two"
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sign = lambda: torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int64).to(torch.float64) * 2 - 1
    d1, d2 = sign(), sign()
    p1 = torch.randperm(n, generator=g, device=device)
    s = torch.logspace(0.0, -float(torch.log10(torch.tensor(kappa))), n, dtype=torch.float64, device=device)
    # M = U diag(sqrt(s)), then A = M M^T.
    M = torch.diag(torch.sqrt(s) * d2)          # D2 S^(1/2)
    M = _hadamard(M, 0)                         # H D2 S^(1/2)
    M = M[p1]                                   # P1 H D2 S^(1/2)
    M = M * d1[:, None]                         # D1 P1 H D2 S^(1/2)
    M = _hadamard(M, 0)                         # U S^(1/2)
    A = M @ M.t()
    del M
    A = (A + A.t()) * 0.5
    return A.contiguous()


def batch_sizes(seed, count=4000, m_lo=32, m_hi=768, n_lo=16):
    """Sizes of the batched workload: m ~ U{m_lo..m_hi}, then n_i ~ U{n_lo..m_i}."""
    rng = np.random.default_rng(seed)
    m = rng.integers(m_lo, m_hi + 1, size=count)
    n = np.array([rng.integers(n_lo, mi + 1) for mi in m])
    return m.astype(np.int64), n.astype(np.int64), rng


def batch_matrices(seed, count=4000, m_lo=32, m_hi=768, n_lo=16):
    """List of column-major N(0,1) matrices with the sizes of ``batch_sizes``,
    drawn in order from the same generator."""
    m, n, rng = batch_sizes(seed, count, m_lo, m_hi, n_lo)
    mats = [np.asfortranarray(rng.standard_normal((int(mi), int(ni)))) for mi, ni in zip(m, n)]
    return m, n, mats


def batch_ls(seed, count=4000, m_lo=32, m_hi=768, n_lo=16):
    """(m, n, mats, bs, xs): ``batch_matrices`` drawn first, then from the same
    generator x_i ~ N(0, 1) (n_i entries) in order, and b_i = A_i x_i."""
    m, n, rng = batch_sizes(seed, count, m_lo, m_hi, n_lo)
    mats = [np.asfortranarray(rng.standard_normal((int(mi), int(ni)))) for mi, ni in zip(m, n)]
    xs = [rng.standard_normal(int(ni)) for ni in n]
    bs = [A @ x for A, x in zip(mats, xs)]
    return m, n, mats, bs, xs


def qr_flops(m, n):
    """LAPACK operation count of a Householder QR, 2 m n^2 - 2 n^3 / 3 (m >= n);
    for m < n the count of the m x m leading part plus the update of the rest."""
    m = float(m)
    n = float(n)
    if m >= n:
        return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    return 2.0 * n * m * m - 2.0 * m ** 3 / 3.0
