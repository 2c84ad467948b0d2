"""Probe estimates of the factorisation invariants at sizes where Q cannot be
formed (test tooling; torch on the GPU computes A Z and R Z, the library's
tileqr_apply_q / tileqr_apply_qt apply Q).

For E = A - Q [R; 0] and a Gaussian z, E ||E z||^2 = ||E||_F^2, so with k
probes ||E||_F ~ sqrt(sum_i ||E z_i||^2 / k); likewise for the thin Gram error
[I 0] Q^T Q [I; 0] - I_n.

The products A Z and R Z are formed with the contracted index cut into
chunks of 256 whose partial products are added with error-free
transformations (two-sum, compensation carried separately): a plain FP64
product with 32768 terms rounds at about sqrt(n) u relative, which is the
size of the backward error being measured at that order.
"""
import torch

CHUNK = 256


def compensated_matmul(Zt, M, chunk=CHUNK):
    """Zt @ M (Zt (k, n), M (n, m)) with the partial products over chunks of
    the contracted index summed by two-sum with a separate compensation."""
    s = None
    c = None
    for c0 in range(0, Zt.shape[1], chunk):
        p = Zt[:, c0:c0 + chunk] @ M[c0:c0 + chunk, :]
        if s is None:
            s = p
            c = torch.zeros_like(p)
            continue
        t = s + p
        bp = t - s
        c += (s - (t - bp)) + (p - bp)
        s = t
    return s + c


def gaussian(k, n, seed, device="cuda"):
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((k, n), generator=g, device=device, dtype=torch.float64)


def a_times(At, Zt):
    """A Z for column-major A in tensor At (n, m) and Z column-major (k, n):
    the result column-major (k, m)."""
    return compensated_matmul(Zt, At)


def beta_fact_probe(tq, Ft, T, m, n, nb, ib, AZt, Zt):
    """||A - Q [R; 0]||_F / ||A||_F estimate: AZt = A Z taken before the
    factorisation, Ft the factored matrix (column-major, (n, m)), ||A||_F
    from normA."""
    k = Zt.shape[0]
    # R Z with R = triu of the leading n x n block: column-major R^T is the
    # lower triangle of Ft[:, :n].
    RtT = torch.tril(Ft[:, :n])            # (n, n) tensor = R^T row-major
    W = torch.zeros((k, m), dtype=torch.float64, device=Ft.device)
    W[:, :n] = compensated_matmul(Zt, RtT)   # (R Z)^T
    del RtT
    tq.check(tq.apply_q(m, n, k, Ft.data_ptr(), m, nb, ib, T.data_ptr(), W.data_ptr(), m), "apply_q")
    D = W - AZt
    return float(torch.linalg.norm(D) / k ** 0.5)


def beta_orth_probe(tq, Ft, T, m, n, nb, ib, k=8, seed=7):
    """||Q_thin^T Q_thin - I_n||_F estimate through apply_q then apply_qt."""
    Z = gaussian(k, n, seed, Ft.device)
    W = torch.zeros((k, m), dtype=torch.float64, device=Ft.device)
    W[:, :n] = Z
    tq.check(tq.apply_q(m, n, k, Ft.data_ptr(), m, nb, ib, T.data_ptr(), W.data_ptr(), m), "apply_q")
    tq.check(tq.apply_qt(m, n, k, Ft.data_ptr(), m, nb, ib, T.data_ptr(), W.data_ptr(), m), "apply_qt")
    E = W[:, :n] - Z
    return float(torch.linalg.norm(E) / k ** 0.5)


def factor_invariants(tq, At, m, n, nb, ib, k=8, seed=3, opts=None):
    """Factor the column-major A in At (destroyed) and return
    (beta_fact_est, beta_orth_est, T)."""
    Z = gaussian(k, n, seed, At.device)
    AZ = a_times(At, Z)
    normA = float(torch.linalg.norm(At))
    T = tq.factor_tensor(At, m, nb, ib, opts)
    torch.cuda.synchronize()
    bf = beta_fact_probe(tq, At, T, m, n, nb, ib, AZ, Z) / normA
    bo = beta_orth_probe(tq, At, T, m, n, nb, ib, k=k)
    return bf, bo, T
