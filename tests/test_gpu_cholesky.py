"""GPU tests of the tiled Cholesky factorisation (tilechol_factor, through the
C-ABI) against the Cholesky oracle (plain column-by-column factorisation).

The factor of a symmetric positive definite matrix is unique, so L is
compared with the oracle's normwise within a bound from the arithmetic
(c n u kappa), and the backward error ||A - L L^T||_F / ||A||_F is held to
1e-14.  Every order of the DAG gives the same bits as Algorithm 1's loop
order; the strict upper triangle is never touched; a matrix that is not
positive definite reports the order of its first bad leading minor.
tilechol_solve is checked against the oracle's forward and back
substitution with the same L and by its backward error.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_0709_1272_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def tq():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0709_1272_amd import tileqr
    return tileqr


@pytest.fixture(scope="module")
def tc(tq):
    from paper_0709_1272_amd import tilechol
    return tilechol


def factor(tq, tc, A, nb=0, **opt):
    n = A.shape[0]
    At = tq.to_device(A)
    o = tq.opts(**opt)
    rc, info = tc.factor_tensor(At, n, nb, o)
    torch.cuda.synchronize()
    return rc, tq.to_host(At, n), info


@pytest.mark.parametrize("n,nb,kappa", [(64, 64, 1e2), (100, 64, 1e3), (128, 64, 1e4), (128, 128, 1e4),
                                        (300, 64, 1e5), (300, 128, 1e5), (517, 128, 1e6), (1024, 128, 1e3),
                                        (2000, 128, 1e6)])
def test_factor_vs_oracle(tq, tc, n, nb, kappa):
    A = synth.spd_matrix(n + nb, n, kappa)
    rc, F, info = factor(tq, tc, A, nb)
    assert rc == tq.OK and info.nb == nb
    L = np.tril(F)
    Lo, oinfo = oracle.potrf(A)
    assert oinfo == 0
    err = np.linalg.norm(L - Lo) / np.linalg.norm(Lo)
    bwd = np.linalg.norm(A - L @ L.T) / np.linalg.norm(A)
    print(f"n={n} nb={nb} kappa={kappa:.0e}: |L - L_oracle|/|L| = {err:.2e}, backward {bwd:.2e}")
    assert np.all(np.diag(L) > 0)
    assert err <= 4 * n * EPS * kappa
    assert bwd <= 1e-14


def test_upper_triangle_untouched(tq, tc):
    # Only the lower triangle is read or written: NaN above the diagonal
    # stays, bit for bit, and changes no entry of L.
    n = 333
    A = synth.spd_matrix(5, n, 1e3)
    rc, F, _ = factor(tq, tc, A, 64)
    assert rc == tq.OK
    B = A.copy()
    iu = np.triu_indices(n, 1)
    B[iu] = np.nan
    rc, G, _ = factor(tq, tc, B, 64)
    assert rc == tq.OK
    assert np.array_equal(np.tril(G), np.tril(F))
    assert np.all(np.isnan(G[iu]))


@pytest.mark.parametrize("n,nb", [(700, 64), (1000, 128), (129, 128)])
def test_dag_bitwise_equals_algorithm_order(tq, tc, n, nb):
    # The persistent scheduler, in its own order and in randomised ones,
    # gives bitwise the result of Algorithm 1's loop order.
    A = synth.spd_matrix(7, n, 1e4)
    rc, ref, _ = factor(tq, tc, A, nb, flags=tq.FLAG_SERIAL)
    assert rc == tq.OK
    rc, F, _ = factor(tq, tc, A, nb)
    assert rc == tq.OK and np.array_equal(F, ref)
    for seed in (1, 2, 3):
        rc, F, _ = factor(tq, tc, A, nb, flags=tq.FLAG_SHUFFLE, seed=seed, workers=1 + 37 * seed)
        assert rc == tq.OK and np.array_equal(F, ref), seed


@pytest.mark.parametrize("n,nb,k", [(200, 64, 1), (200, 64, 64), (200, 64, 65), (450, 128, 300), (450, 128, 450)])
def test_not_positive_definite(tq, tc, n, nb, k):
    # The order of the first leading minor that is not positive definite, as
    # the oracle and LAPACK's dpotrf report it; A is left as it was.
    A = synth.spd_matrix(11, n, 10.0)
    A[k - 1, k - 1] -= 3.0 * A[k - 1, k - 1] + 5.0
    _, oinfo = oracle.potrf(A)
    _, linfo = scipy.linalg.lapack.dpotrf(A, lower=1)
    assert oinfo == linfo == k
    for flags in (0, tq.FLAG_SERIAL):
        rc, F, info = factor(tq, tc, A, nb, flags=flags)
        assert rc == tq.ENOTSPD and info.minor == k, (flags, info.minor)
        assert np.array_equal(F, A)


def test_nonfinite_input(tq, tc):
    A = synth.spd_matrix(12, 150, 1e2)
    A[120, 7] = np.inf
    rc, F, _ = factor(tq, tc, A, 64)
    assert rc == tq.ENONFINITE
    assert np.array_equal(F, A)


def test_default_blocking_and_tiny(tq, tc):
    for n in (1, 2, 31, 65):
        A = synth.spd_matrix(13 + n, n, 1e2)
        rc, F, info = factor(tq, tc, A)
        assert rc == tq.OK and info.nb == 64
        Lo, _ = oracle.potrf(A)
        assert np.linalg.norm(np.tril(F) - Lo) <= 1e-13 * np.linalg.norm(Lo)
    A = synth.spd_matrix(14, 600, 1e2)
    rc, _, info = factor(tq, tc, A)
    assert rc == tq.OK and info.nb == 128


def test_timing_and_lda(tq, tc):
    # A leading dimension larger than n; TILEQR_FLAG_TIMING fills the times.
    n, lda = 500, 531
    A = synth.spd_matrix(15, n, 1e3)
    Ap = np.zeros((lda, n))
    Ap[:n] = A
    At = torch.tensor(np.ascontiguousarray(Ap.T), device="cuda")
    info = tc.CholInfo()
    rc = tc.factor(n, At.data_ptr(), lda, 128, tq.opts(flags=tq.FLAG_TIMING), info)
    torch.cuda.synchronize()
    assert rc == tq.OK and info.ms_factor > 0 and 0 < info.ms_worker <= info.ms_factor
    F = At.cpu().numpy().T
    assert np.array_equal(F[n:], np.zeros((lda - n, n)))
    Lo, _ = oracle.potrf(A)
    assert np.linalg.norm(np.tril(F[:n]) - Lo) <= 4 * n * EPS * 1e3 * np.linalg.norm(Lo)


@pytest.mark.parametrize("n", [16384, 32768])
def test_full_size_sampled(tq, tc, n):
    # The benchmark's sizes: the leading 512 x 512 block of L depends only on
    # the leading block of A, so it is compared with the oracle's factor of
    # that block; the backward error is estimated with Gaussian probes,
    # ||A z - L (L^T z)|| / (||A||_F ||z||) over 4 probes.
    A = synth.spd_matrix_device(3, n, 1e6, device="cuda")       # symmetric: rows = columns
    lead = A[:512, :512].cpu().numpy()
    At = A.clone()
    info = tc.CholInfo()
    rc = tc.factor(n, At.data_ptr(), n, 128, tq.opts(flags=tq.FLAG_TIMING), info)
    torch.cuda.synchronize()
    assert rc == tq.OK
    print(f"n={n}: {info.ms_factor:.1f} ms ({tc.flops(n) / info.ms_factor / 1e9:.1f} TF/s)")
    # At holds L column-major, i.e. L^T row-major.
    Lt = torch.triu(At)                                            # L^T as a row-major tensor
    Lo, oinfo = oracle.potrf(lead)
    assert oinfo == 0
    Lg = Lt[:512, :512].t().cpu().numpy()
    assert np.linalg.norm(Lg - Lo) <= 4 * 512 * EPS * 1e6 * np.linalg.norm(Lo)
    # ||A - L L^T||_F ~ sqrt(sum_i ||(A - L L^T) z_i||^2 / k) for Gaussian z_i;
    # the products summed with compensation (a plain FP64 product over n
    # terms rounds at about the size of what is measured).
    from gpu_probes import compensated_matmul, gaussian
    k = 4
    Zt = gaussian(k, n, 5)
    AZ = compensated_matmul(Zt, A)                  # (A Z)^T, A symmetric
    V = compensated_matmul(Zt, Lt.t())              # (L^T Z)^T
    W = compensated_matmul(V, Lt)                   # (L L^T Z)^T
    est = float(torch.linalg.norm(AZ - W) / k ** 0.5 / torch.linalg.norm(A))
    print(f"n={n}: ||A - L L^T||_F / ||A||_F estimate {est:.2e}")
    assert est <= 1e-14


def solve_on_device(tq, tc, F, B, nb=0, ldl=None, ldb=None, **opt):
    """tilechol_solve with the factored array F (host) and right-hand sides B;
    returns (status, X)."""
    n, nrhs = B.shape
    ldl = ldl or n
    ldb = ldb or n
    Fp = np.zeros((ldl, n))
    Fp[:n] = F
    Bp = np.zeros((ldb, nrhs))
    Bp[:n] = B
    Lt = tq.to_device(Fp)
    Bt = tq.to_device(Bp)
    rc = tc.solve(n, nrhs, Lt.data_ptr(), ldl, Bt.data_ptr(), ldb, nb, tq.opts(**opt))
    torch.cuda.synchronize()
    Xp = tq.to_host(Bt)
    assert np.array_equal(Xp[n:], Bp[n:])          # rows beyond n untouched
    return rc, Xp[:n]


@pytest.mark.parametrize("n,nrhs,nb,kappa", [(64, 1, 64, 1e2), (100, 3, 64, 1e3), (333, 40, 64, 1e4),
                                             (517, 33, 128, 1e6), (1024, 64, 128, 1e3), (2000, 5, 128, 1e6),
                                             (300, 70, 128, 1e2)])
def test_solve_vs_oracle(tq, tc, n, nrhs, nb, kappa):
    # X from tilechol_solve with the GPU factor against the oracle's forward
    # and back substitution (oracle_potrs_lower) with the same L: normwise
    # within c n u kappa (both solve the same triangles, in other orders);
    # and the backward error ||A X - B||_F / (||A||_F ||X||_F).
    A = synth.spd_matrix(n + 17, n, kappa)
    rc, F, _ = factor(tq, tc, A, nb)
    assert rc == tq.OK
    B = np.random.default_rng(n + nrhs).standard_normal((n, nrhs))
    rc, X = solve_on_device(tq, tc, F, B, nb)
    assert rc == tq.OK
    Xo = oracle.potrs(np.tril(F), B)
    err = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    bwd = np.linalg.norm(A @ X - B) / (np.linalg.norm(A) * np.linalg.norm(X))
    print(f"n={n} nrhs={nrhs} nb={nb} kappa={kappa:.0e}: |X - X_oracle|/|X| = {err:.2e}, backward {bwd:.2e}")
    assert err <= 8 * n * EPS * kappa
    assert bwd <= 1e-14


def test_solve_tile_size_and_leading_dimensions(tq, tc):
    # Any tile size with any factor; leading dimensions above n.
    n, nrhs = 450, 9
    A = synth.spd_matrix(21, n, 1e4)
    rc, F, _ = factor(tq, tc, A, 128)
    assert rc == tq.OK
    B = np.random.default_rng(5).standard_normal((n, nrhs))
    rc1, X1 = solve_on_device(tq, tc, F, B, 64)
    rc2, X2 = solve_on_device(tq, tc, F, B, 128, ldl=n + 13, ldb=n + 3)
    rc3, X3 = solve_on_device(tq, tc, F, B, 0)
    assert rc1 == rc2 == rc3 == tq.OK
    Xo = oracle.potrs(np.tril(F), B)
    for X in (X1, X2, X3):
        assert np.linalg.norm(X - Xo) <= 8 * n * EPS * 1e4 * np.linalg.norm(Xo)
    assert np.array_equal(X3, X1)                   # n <= 512 chooses nb 64


def test_solve_zero_diagonal_and_arguments(tq, tc):
    n = 200
    A = synth.spd_matrix(22, n, 10.0)
    rc, F, _ = factor(tq, tc, A, 64)
    assert rc == tq.OK
    F0 = F.copy()
    F0[130, 130] = 0.0
    rc, _ = solve_on_device(tq, tc, F0, np.ones((n, 2)), 64)
    assert rc == tq.ESINGULAR
    Lt = tq.to_device(F)
    Bt = tq.to_device(np.ones((n, 2)))
    L, B = Lt.data_ptr(), Bt.data_ptr()
    assert tc.solve(-1, 2, L, n, B, n) == -1
    assert tc.solve(n, -1, L, n, B, n) == -2
    assert tc.solve(n, 2, 0, n, B, n) == -3
    assert tc.solve(n, 2, L, n - 1, B, n) == -4
    assert tc.solve(n, 2, L, n, 0, n) == -5
    assert tc.solve(n, 2, L, n, B, n - 1) == -6
    assert tc.solve(n, 2, L, n, B, n, 96) == -7
    assert tc.solve(n, 2, L, n, B, n, 0, tq.opts(precision=9)) == -8
    assert tc.solve(n, 2, L, n, B, n, 0, tq.opts(precision=tq.BF16X3)) == tq.EUNSUPPORTED
    assert tc.solve(0, 2, 0, 1, 0, 1) == tq.OK
    assert tc.solve(n, 0, L, n, 0, n) == tq.OK
    torch.cuda.synchronize()
    assert np.array_equal(tq.to_host(Bt), np.ones((n, 2)))    # nothing touched


def test_solve_full_size(tq, tc):
    # 16384^2, 16 right-hand sides: the backward error of X, with the
    # products summed with compensation on the device.
    from gpu_probes import compensated_matmul
    n, nrhs = 16384, 16
    A = synth.spd_matrix_device(3, n, 1e6, device="cuda")      # symmetric: rows = columns
    Lt = A.clone()
    info = tc.CholInfo()
    assert tc.factor(n, Lt.data_ptr(), n, 128, tq.opts(), info) == tq.OK
    g = torch.Generator(device="cuda")
    g.manual_seed(9)
    Bt = torch.randn((nrhs, n), generator=g, device="cuda", dtype=torch.float64)   # B column-major
    Xt = Bt.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    rc = tc.solve(n, nrhs, Lt.data_ptr(), n, Xt.data_ptr(), n, 128, tq.opts())
    e1.record()
    torch.cuda.synchronize()
    assert rc == tq.OK
    AX = compensated_matmul(Xt, A)                   # (A X)^T, A symmetric
    bwd = float(torch.linalg.norm(AX - Bt) / (torch.linalg.norm(A) * torch.linalg.norm(Xt)))
    print(f"n={n} nrhs={nrhs}: solve {e0.elapsed_time(e1):.2f} ms, backward error {bwd:.2e}")
    assert bwd <= 1e-14
