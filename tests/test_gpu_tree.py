"""GPU tests of the tree reduction for tall matrices (tileqr_factor_tree,
tileqr_apply_qt_tree / tileqr_apply_q_tree, tileqr_solve_ls_tree, through the
C-ABI) against the Householder QR oracle.

R is unique up to the signs of its rows, so the tree's R is compared with
the oracle's R (row signs fixed) normwise; Q^T A = [R; 0] and Q Q^T B = B
check the tree's Q as a whole (its reflectors differ from the flat tree's);
the least-squares solution is unique and is compared with the oracle's
within c kappa u.  One leaf is Algorithm 2 itself: bitwise the flat
factorisation.
"""
import numpy as np
import pytest

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


def factor_tree(tq, A, nb, ib, leaves, **opt):
    m, n = A.shape
    At = tq.to_device(A)
    F = torch.zeros(max(tq.tree_size(m, n, nb, ib, leaves), 1), dtype=torch.float64, device="cuda")
    rc = tq.factor_tree(m, n, At.data_ptr(), m, nb, ib, leaves, F.data_ptr(), tq.opts(**opt))
    torch.cuda.synchronize()
    return rc, At, F


SHAPES = [(1024, 64, 64, 16, 2), (2048, 256, 64, 16, 4), (3000, 200, 64, 32, 3), (4096, 512, 128, 32, 5),
          (2600, 200, 128, 16, 7), (1500, 120, 64, 16, 8), (6000, 1000, 256, 32, 4)]


@pytest.mark.parametrize("m,n,nb,ib,leaves", SHAPES)
def test_tree_r_and_q(tq, m, n, nb, ib, leaves):
    A = synth.uniform(11 + m + leaves, m, n)
    rc, At, F = factor_tree(tq, A, nb, ib, leaves)
    assert rc == tq.OK, tq.status_string(rc)
    R = np.triu(tq.to_host(At, m)[:n])
    Fo, _ = oracle.geqr2(A)
    Ro = oracle.r_factor(Fo)
    err = oracle.r_diff(R, Ro)
    # Q^T A = [R; 0]: the tree's transformations applied to A itself.
    Bt = tq.to_device(A)
    rc = tq.apply_qt_tree(m, n, n, At.data_ptr(), m, nb, ib, leaves, F.data_ptr(), Bt.data_ptr(), m)
    torch.cuda.synchronize()
    assert rc == tq.OK
    QtA = tq.to_host(Bt, m)
    top = np.linalg.norm(np.triu(QtA[:n]) - R) / np.linalg.norm(R)
    low = (np.linalg.norm(np.tril(QtA[:n], -1)) + np.linalg.norm(QtA[n:])) / np.linalg.norm(A)
    # Q Q^T B = B and ||Q^T B|| = ||B||.
    B = np.random.default_rng(m).standard_normal((m, 3))
    Bt = tq.to_device(B)
    rc1 = tq.apply_qt_tree(m, n, 3, At.data_ptr(), m, nb, ib, leaves, F.data_ptr(), Bt.data_ptr(), m)
    torch.cuda.synchronize()
    QtB = tq.to_host(Bt, m)
    rc2 = tq.apply_q_tree(m, n, 3, At.data_ptr(), m, nb, ib, leaves, F.data_ptr(), Bt.data_ptr(), m)
    torch.cuda.synchronize()
    assert rc1 == tq.OK and rc2 == tq.OK
    back = np.linalg.norm(tq.to_host(Bt, m) - B) / np.linalg.norm(B)
    norm = abs(np.linalg.norm(QtB) - np.linalg.norm(B)) / np.linalg.norm(B)
    print(f"{m}x{n} nb={nb} ib={ib} leaves={leaves}: r_diff {err:.2e}, Q^T A top {top:.2e} rest {low:.2e}, "
          f"Q Q^T B {back:.2e}, norm {norm:.2e}")
    assert err <= 1e-12
    assert top <= 1e-13 and low <= 1e-14 * np.sqrt(m)
    assert back <= 1e-14 * np.sqrt(m) and norm <= 1e-14 * np.sqrt(m)


@pytest.mark.parametrize("m,n,nb,ib", [(2048, 256, 64, 16), (1000, 300, 128, 32)])
def test_one_leaf_is_algorithm_2(tq, m, n, nb, ib):
    # A single leaf is the flat factorisation, bit for bit.
    A = synth.uniform(5 + m, m, n)
    rc, At, F = factor_tree(tq, A, nb, ib, 1)
    assert rc == tq.OK
    Af = tq.to_device(A)
    T = torch.zeros(tq.t_size(m, n, nb, ib), dtype=torch.float64, device="cuda")
    assert tq.factor(m, n, Af.data_ptr(), m, nb, ib, T.data_ptr()) == tq.OK
    torch.cuda.synchronize()
    assert np.array_equal(tq.to_host(At, m), tq.to_host(Af, m))
    assert np.array_equal(F[:T.numel()].cpu().numpy(), T.cpu().numpy())


def test_leaves_do_not_change_r_beyond_rounding(tq):
    # Different trees give the same R up to rounding (R is unique).
    m, n, nb, ib = 4096, 384, 128, 32
    A = synth.uniform(21, m, n)
    Rs = []
    for leaves in (1, 2, 3, 4, 8):
        rc, At, _ = factor_tree(tq, A, nb, ib, leaves)
        assert rc == tq.OK
        Rs.append(np.triu(tq.to_host(At, m)[:n]))
    for R in Rs[1:]:
        assert oracle.r_diff(R, Rs[0]) <= 1e-12


@pytest.mark.parametrize("m,n,kappa,nb,ib,leaves,nrhs", [(3000, 300, 1e4, 64, 16, 4, 1), (4096, 256, 1e8, 128, 32, 3, 2),
                                                          (2048, 512, 1e2, 256, 32, 2, 1)])
def test_solve_ls_tree_vs_oracle(tq, m, n, kappa, nb, ib, leaves, nrhs):
    A, b, _ = synth.svd_matrix(31 + m, m, n, kappa, nrhs=nrhs)
    b2 = b.reshape(m, -1)
    At, Bt = tq.to_device(A), tq.to_device(b2)
    Xt = torch.zeros((nrhs, n), dtype=torch.float64, device="cuda")
    rc, ms = tq.solve_ls_tree(m, n, nrhs, At.data_ptr(), m, Bt.data_ptr(), m, Xt.data_ptr(), n, nb, ib, leaves)
    torch.cuda.synchronize()
    assert rc == tq.OK, tq.status_string(rc)
    assert ms > 0
    assert np.array_equal(tq.to_host(At, m), A) and np.array_equal(tq.to_host(Bt, m), b2)
    x = tq.to_host(Xt, n)
    xo, ro = oracle.lstsq(A, b2)
    for v in range(nrhs):
        rel_res = np.linalg.norm(ro[:, v]) / (np.linalg.norm(A, 2) * np.linalg.norm(xo[:, v]))
        bound = 64 * n * EPS * kappa * (1 + kappa * rel_res)
        err = np.linalg.norm(x[:, v] - xo[:, v]) / np.linalg.norm(xo[:, v])
        eta = oracle.eta_ls(A, x[:, v], b2[:, v])
        print(f"{m}x{n} kappa={kappa:.0e} leaves={leaves}: |x - x_oracle|/|x| {err:.2e} (bound {bound:.1e}), "
              f"eta_ls {eta:.2e}")
        assert err <= bound
        assert eta <= 1e-14


def test_tree_arguments(tq):
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    assert tq.factor_tree(100, 200, d.data_ptr(), 100, 64, 16, 1, d.data_ptr(), None) == -2
    assert tq.factor_tree(256, 64, d.data_ptr(), 256, 64, 16, 5, d.data_ptr(), None) == -7   # leaves of 0 rows
    assert tq.factor_tree(256, 64, d.data_ptr(), 256, 64, 16, 2, 0, None) == -8
    assert tq.factor_tree(256, 64, d.data_ptr(), 256, 64, 32, 2, d.data_ptr(),
                          tq.opts(precision=tq.BF16X3)) == tq.EUNSUPPORTED
    assert tq.tree_size(256, 64, 64, 16, 5) == 0


@pytest.mark.parametrize("leaves", [4, 8])
def test_full_size_tall_ls(tq, leaves):
    # The tall least-squares workload, 65536 x 1024, kappa 1e6: the tree
    # solution against the flat FP64 solve (both unique up to rounding).
    m, n = 65536, 1024
    At, Bt, _ = synth.svd_matrix_haar_device(2, m, n, 1e6, nrhs=1, device="cuda")
    Xt = torch.zeros((1, n), dtype=torch.float64, device="cuda")
    rc, ms = tq.solve_ls_tree(m, n, 1, At.data_ptr(), m, Bt.data_ptr(), m, Xt.data_ptr(), n, 256, 32, leaves)
    torch.cuda.synchronize()
    assert rc == tq.OK, tq.status_string(rc)
    Xf = torch.zeros((1, n), dtype=torch.float64, device="cuda")
    info = tq.Info()
    rc = tq.solve_ls(m, n, 1, At.data_ptr(), m, Bt.data_ptr(), m, Xf.data_ptr(), n, tq.opts(nb=256, ib=32), info)
    torch.cuda.synchronize()
    assert rc == tq.OK
    d = float(torch.linalg.norm(Xt - Xf) / torch.linalg.norm(Xf))
    print(f"65536x1024 leaves={leaves}: tree solve {ms:.2f} ms, flat FP64 solve {info.ms_total:.2f} ms, "
          f"|x_tree - x_flat|/|x| {d:.2e}")
    assert d <= 64 * n * EPS * 1e6
