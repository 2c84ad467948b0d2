"""GPU tests of tileqr_solve_ls_batched: many least-squares systems factored
in one batched launch, then solved and refined by one workgroup each.  Each
solution is checked against the oracle's least-squares solution (unblocked
Householder QR, back substitution) within the conditioning bound, and its
backward error is recomputed here from its definition; the split precisions
must reach the same backward-error bar after refinement.

Inputs: the batched workload's distribution (m ~ U{32..768}, n ~ U{16..m},
N(0, 1) entries) with one consistent right-hand side per matrix,
b_i = A_i x_i, x_i ~ N(0, 1)."""
import numpy as np
import pytest

import oracle
from oracle import metrics
from paper_0709_1272_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EPS = np.finfo(np.float64).eps
TOL = 1e-14


@pytest.fixture(scope="module")
def tq():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0709_1272_amd import tileqr
    return tileqr


class LsBatch:
    def __init__(self, tq, mats, bs):
        self.tq = tq
        self.mats, self.bs = mats, bs
        self.A = [tq.to_device(a) for a in mats]
        self.b = [torch.as_tensor(b, dtype=torch.float64, device="cuda").contiguous() for b in bs]
        self.x = [torch.full((max(a.shape[1], 1),), float("nan"), dtype=torch.float64, device="cuda") for a in mats]
        self.A0 = [a.clone() for a in self.A]
        self.b0 = [b.clone() for b in self.b]

    def solve(self, o=None, info=None):
        ms = [a.shape[0] for a in self.mats]
        ns = [a.shape[1] for a in self.mats]
        rc, eta, its = self.tq.solve_ls_batched(ms, ns, [a.data_ptr() for a in self.A], [max(m, 1) for m in ms],
                                               [b.data_ptr() for b in self.b], [x.data_ptr() for x in self.x],
                                               o, info)
        torch.cuda.synchronize()
        return rc, eta, its

    def xsol(self, i):
        return self.x[i].cpu().numpy()[: self.mats[i].shape[1]]


def eta_of(A, x, b):
    e = metrics.eta_ls(A, x, b)
    if A.shape[0] == A.shape[1]:
        e = max(e, metrics.eta_inf(A, x, b))
    return e


@pytest.fixture(scope="module")
def workload():
    m, n, mats, bs, xs = synth.batch_ls(3, count=240)
    # a square system and a single-column one besides the drawn shapes
    rng = np.random.default_rng(5)
    for shape in ((300, 300), (200, 1)):
        A = np.asfortranarray(rng.standard_normal(shape))
        x = rng.standard_normal(shape[1])
        mats.append(A)
        bs.append(A @ x)
    return mats, bs


@pytest.mark.parametrize("name", ["FP64", "BF16X3", "FP16X2"])
def test_batched_ls_vs_oracle(tq, workload, name):
    mats, bs = workload
    B = LsBatch(tq, mats, bs)
    info = tq.BatchInfo()
    o = tq.opts(precision=getattr(tq, name), tol=TOL)
    rc, eta, its = B.solve(o, info)
    print(f"{name}: rc {tq.status_string(rc)} converged {info.converged}/{len(mats)} max_iter {info.max_iterations} "
          f"max_eta {info.max_eta:.2e} ms_factor {info.ms_factor:.2f} ms_total {info.ms_total:.2f}")
    assert rc == tq.OK, tq.status_string(rc)
    assert info.converged == len(mats) and info.max_eta <= TOL
    if name == "FP64":
        assert info.max_iterations <= 1
    else:
        assert info.max_iterations >= 1       # the split factor really needed refinement
    # A and b are not written.
    for i in range(0, len(mats), 37):
        assert torch.equal(B.A[i], B.A0[i]) and torch.equal(B.b[i], B.b0[i])
    worst = 0.0
    for i in range(len(mats)):
        A, b = mats[i], bs[i]
        x = B.xsol(i)
        e = eta_of(A, x, b)
        assert e <= 2 * TOL, (i, A.shape, e, eta[i])
        assert abs(e - eta[i]) <= 0.5 * max(e, eta[i]) + 1e-15, (i, e, eta[i])
        if i % 2 == 0:
            xo, _ = oracle.lstsq(A, b)
            kappa = np.linalg.cond(A)
            err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
            worst = max(worst, err / (kappa * EPS))
            assert err <= 64 * A.shape[1] * kappa * EPS, (i, A.shape, err, kappa)
    print(f"  worst |x - x_oracle| / |x_oracle| / (kappa u) = {worst:.2f}")


def test_batched_ls_inconsistent_and_square_paths(tq):
    # Inconsistent systems (b has a component outside range(A)): the
    # augmented-system refinement must still meet the bar with a split factor.
    rng = np.random.default_rng(9)
    mats, bs = [], []
    for m, n in ((500, 120), (333, 333), (700, 64), (96, 95)):
        A = np.asfortranarray(rng.standard_normal((m, n)))
        mats.append(A)
        bs.append(A @ rng.standard_normal(n) + rng.standard_normal(m))
    B = LsBatch(tq, mats, bs)
    rc, eta, its = B.solve(tq.opts(precision=tq.BF16X3, tol=TOL))
    assert rc == tq.OK, tq.status_string(rc)
    for i, (A, b) in enumerate(zip(mats, bs)):
        x = B.xsol(i)
        xo, _ = oracle.lstsq(A, b)
        assert eta_of(A, x, b) <= 2 * TOL
        assert np.linalg.norm(x - xo) <= 64 * A.shape[1] * np.linalg.cond(A) * EPS * np.linalg.norm(xo)
        assert its[i] >= 1


def test_batched_ls_errors(tq):
    A = np.asfortranarray(np.random.default_rng(1).standard_normal((40, 20)))
    B = LsBatch(tq, [A, A.T.copy(order="F")], [np.ones(40), np.ones(20)])
    rc, _, _ = B.solve()
    assert rc == -3                                   # n > m
    bad = A.copy(order="F")
    bad[3, 4] = np.inf
    B = LsBatch(tq, [A, bad], [np.ones(40), np.ones(40)])
    rc, _, _ = B.solve()
    assert rc == tq.ENONFINITE
    Z = np.zeros((30, 10), order="F")
    Z[:, :9] = np.random.default_rng(2).standard_normal((30, 9))
    B = LsBatch(tq, [Z], [np.ones(30)])
    rc, _, _ = B.solve()
    assert rc == tq.ESINGULAR
    B = LsBatch(tq, [A], [np.ones(40)])
    rc, _, _ = B.solve(tq.opts(flags=tq.FLAG_ASYNC))
    assert rc == tq.EUNSUPPORTED
