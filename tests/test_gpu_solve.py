"""GPU tests of tileqr_solve_ls (through the C-ABI) against the oracle.

The least-squares solution is unique for a full-rank A, so it is compared
with the oracle's (Householder QR + back substitution) within the normwise
perturbation bound c * kappa * u (plus kappa^2 u times the relative
residual for inconsistent systems); the backward error is recomputed in
numpy from the returned x.
"""
import ctypes

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


def solve(tq, A, b, **opt):
    m, n = A.shape
    b2 = b.reshape(m, -1)
    nrhs = b2.shape[1]
    At = tq.to_device(A)
    Bt = tq.to_device(b2)
    Xt = torch.zeros((nrhs, n), dtype=torch.float64, device="cuda")
    info = tq.Info()
    o = tq.opts(**opt)
    rc = tq.solve_ls(m, n, nrhs, At.data_ptr(), m, Bt.data_ptr(), m, Xt.data_ptr(), n, o, info)
    torch.cuda.synchronize()
    # A and B are left untouched.
    assert np.array_equal(tq.to_host(At, m), A)
    assert np.array_equal(tq.to_host(Bt, m), b2)
    x = tq.to_host(Xt, n)
    return rc, (x[:, 0] if b.ndim == 1 else x), info


@pytest.mark.parametrize("m,n,kappa,nb,ib,nrhs", [(600, 200, 1e4, 64, 16, 1), (1000, 300, 1e6, 128, 32, 3),
                                                  (777, 777, 1e2, 64, 32, 2), (2048, 256, 1e8, 256, 32, 1),
                                                  (300, 65, 1e3, 64, 16, 40)])
def test_fp64_solve_vs_oracle(tq, m, n, kappa, nb, ib, nrhs):
    A, b, _ = synth.svd_matrix(3 + m, m, n, kappa, nrhs=nrhs)
    rc, x, info = solve(tq, A, b, nb=nb, ib=ib)
    assert rc == tq.OK, tq.status_string(rc)
    xo, ro = oracle.lstsq(A, b)
    xo2, x2, b2 = xo.reshape(n, -1), x.reshape(n, -1), b.reshape(m, -1)
    for v in range(x2.shape[1]):
        rel_res = np.linalg.norm(ro.reshape(m, -1)[:, v]) / (np.linalg.norm(A, 2) * np.linalg.norm(xo2[:, v]))
        bound = 64 * n * EPS * kappa * (1 + kappa * rel_res)
        err = np.linalg.norm(x2[:, v] - xo2[:, v]) / np.linalg.norm(xo2[:, v])
        eta = oracle.eta_ls(A, x2[:, v], b2[:, v])
        print(f"{m}x{n} kappa={kappa:.0e} rhs {v}: |x - x_oracle|/|x| {err:.2e} (bound {bound:.1e}) eta {eta:.2e}")
        assert err <= bound
        assert eta <= 1e-14
    assert info.converged == 1
    assert info.eta <= 1e-14


def test_square_system_backward_error(tq):
    # Square systems: the paper's normwise backward error in the inf-norm
    # (Section 3.2.4), here for the QR-based solve.
    A = synth.uniform(21, 512, 512)
    xt = np.random.default_rng(2).standard_normal(512)
    b = A @ xt
    rc, x, _ = solve(tq, A, b, nb=64, ib=16)
    assert rc == tq.OK
    assert oracle.eta_inf(A, x, b) <= 1e-15
    xo, _ = oracle.lstsq(A, b)
    assert np.linalg.norm(x - xo) <= 1e-10 * np.linalg.norm(xo)


def test_singular_reported(tq):
    A = synth.uniform(5, 300, 100)
    A[:, 17] = 0.0
    b = np.ones(300)
    rc, _, _ = solve(tq, A, b, nb=64, ib=16)
    assert rc == tq.ESINGULAR


def test_bad_arguments(tq):
    o = tq.opts()
    info = tq.Info()
    assert tq.solve_ls(5, 6, 1, 1, 5, 1, 5, 1, 6, o, info) == -2
    assert tq.solve_ls(6, 5, 1, 1, 4, 1, 6, 1, 5, o, info) == -5
    assert tq.solve_ls(6, 5, 1, 1, 6, 1, 6, 1, 4, o, info) == -9


@pytest.mark.parametrize("name", ["FP64", "BF16X2"])
def test_check_flag_estimates_beta_fact(tq, name):
    # TILEQR_FLAG_CHECK estimates ||A - Q [R; 0]||_F / ||A||_F with 8 probes;
    # compared with the exact value of the same factorisation (tileqr_factor
    # with the same blocking gives the same bits), Q rebuilt in numpy.
    from test_gpu_factor import rebuild_q
    m, n, nb, ib = 1500, 700, 128, 32
    A, b, _ = synth.svd_matrix(8, m, n, 1e3)
    rc, x, info = solve(tq, A, b, nb=nb, ib=ib, precision=getattr(tq, name), flags=tq.FLAG_CHECK)
    assert rc == tq.OK
    At = tq.to_device(A)
    T = tq.factor_tensor(At, m, nb, ib, tq.opts(precision=getattr(tq, name)))
    torch.cuda.synchronize()
    F = tq.to_host(At, m)
    Q = rebuild_q(F, T.cpu().numpy(), nb, ib)[:m, :m]
    RR = np.zeros((m, n))
    RR[:n] = np.triu(F[:n])
    exact = np.linalg.norm(A - Q @ RR) / np.linalg.norm(A)
    print(f"{name}: beta_fact exact {exact:.3e}, estimate {info.beta_fact_est:.3e} ({info.probes} probes)")
    assert info.probes == 8
    assert 0.3 * exact <= info.beta_fact_est <= 3.0 * exact


def test_info_without_check(tq):
    A, b, _ = synth.svd_matrix(2, 300, 100, 1e2)
    rc, x, info = solve(tq, A, b, nb=64, ib=16)
    assert rc == tq.OK
    assert info.beta_fact_est == -1.0 and info.probes == 0
    assert info.eta_inf == 0.0                      # m > n: not defined
    assert info.eta == info.eta_ls


def test_two_streams_async_match_sync(tq):
    # Each stream has its own workspace: two asynchronous factorisations on
    # two streams, left to overlap, give the bits of synchronous calls.
    mats = [synth.uniform(30 + s, 1536, 1024) for s in range(2)]
    tsz = tq.t_size(1536, 1024, 256, 32)
    ref = []
    for A in mats:
        At = tq.to_device(A)
        # T has entries the factorisation never writes (blocks of tiles
        # above the diagonal): start from zeros on both sides.
        T = torch.zeros(tsz, dtype=torch.float64, device="cuda")
        tq.check(tq.factor(1536, 1024, At.data_ptr(), 1536, 256, 32, T.data_ptr()), "factor")
        torch.cuda.synchronize()
        ref.append((At.clone(), T.clone()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    work = [tq.to_device(A) for A in mats]
    Ts = [torch.zeros(tsz, dtype=torch.float64, device="cuda") for _ in mats]
    torch.cuda.synchronize()
    for rep in range(3):
        for s in range(2):
            work[s].copy_(tq.to_device(mats[s]))
        torch.cuda.synchronize()
        for s in range(2):
            o = tq.opts(stream=streams[s].cuda_stream, flags=tq.FLAG_ASYNC)
            tq.check(tq.factor(1536, 1024, work[s].data_ptr(), 1536, 256, 32, Ts[s].data_ptr(), o), "factor")
        torch.cuda.synchronize()
        for s in range(2):
            assert torch.equal(work[s], ref[s][0]), (rep, s)
            assert torch.equal(Ts[s], ref[s][1]), (rep, s)


def test_cli_driver(tq, capsys):
    # The command-line driver runs the library on seeded inputs and prints
    # one JSON line; a split solve reaches the backward-error target.
    import json
    from paper_0709_1272_amd import cli
    assert cli.main(["factor", "--m", "700", "--n", "300", "--nb", "64", "--ib", "16", "--repeat", "2"]) == 0
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["m"] == 700 and out["n"] == 300 and len(out["runs"]) == 2
    assert out["copy_bytes"] == 700 * 300 * 8
    assert cli.main(["solve", "--n", "512", "--nrhs", "3", "--precision", "bf16x3", "--nb", "128"]) == 0
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["runs"][0]["eta"] <= 1e-14 and out["runs"][0]["iterations"] >= 1


@pytest.mark.parametrize("m,n,nb,ib,nrhs,groups", [(1000, 300, 64, 16, 3, (1, 2, 4)),
                                                   (777, 777, 128, 16, 40, (1, 2, 4, 8)),
                                                   (1536, 1024, 256, 32, 16, (1, 2, 4, 8))])
def test_apply_group_does_not_change_bits(tq, m, n, nb, ib, nrhs, groups):
    # The Q applications take groups of consecutive inner panels per
    # workgroup; each panel is applied with the same operands in the same
    # order whatever the grouping, so the solution is bitwise the same.
    A, b, _ = synth.svd_matrix(31, m, n, 1e4, nrhs=nrhs)
    ref = None
    for g in (0,) + tuple(groups):
        rc, x, info = solve(tq, A, b, nb=nb, ib=ib, apply_group=g, max_iter=2)
        assert rc in (tq.OK, tq.ENOCONV)
        if ref is None:
            ref = x
        else:
            assert np.array_equal(x, ref), f"apply_group {g}"
    xo, _ = oracle.lstsq(A, b)
    assert np.linalg.norm(ref - xo) <= 1e-6 * np.linalg.norm(xo)


def test_apply_group_rejected(tq):
    A = synth.uniform(3, 256, 128)
    b = A @ np.ones(128)
    for g in (3, 16, -1):
        rc, _, _ = solve(tq, A, b, nb=64, ib=16, apply_group=g)
        assert rc == -10, g
    rc, _, _ = solve(tq, A, b, nb=64, ib=32, apply_group=4)   # nb / ib = 2
    assert rc == -10
