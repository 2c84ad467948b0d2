"""GPU test of tileqr_factor_noalloc, the factorisation entry point that
allocates nothing (its workspace is a fixed device array of the library):
through the C-ABI its result must equal tileqr_factor_ex's bit for bit (same
kernels, same schedule), on two calls in a row whose second input is
smaller, in FP64 and in a split precision; a shape whose workspace exceeds
the array is refused before anything runs."""
import numpy as np
import pytest

from paper_0709_1272_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tq():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0709_1272_amd import tileqr
    return tileqr


def _factor_both(tq, A, nb, ib, o):
    m, n = A.shape
    ref = tq.to_device(A)
    out = tq.to_device(A)
    T_ref = torch.zeros(max(tq.t_size(m, n, nb, ib), 1), dtype=torch.float64, device="cuda")
    T_out = torch.zeros_like(T_ref)
    rc = tq.factor(m, n, ref.data_ptr(), m, nb, ib, T_ref.data_ptr(), o)
    assert rc == tq.OK, tq.status_string(rc)
    rc = tq.factor_noalloc(m, n, out.data_ptr(), m, nb, ib, T_out.data_ptr(), o)
    assert rc == tq.OK, tq.status_string(rc)
    torch.cuda.synchronize()
    return ref, out, T_ref, T_out


@pytest.mark.parametrize("prec,nb,ib", [("FP64", 256, 32), ("FP64", 64, 16), ("BF16X3", 128, 32)])
def test_noalloc_matches_factor_ex_twice(tq, prec, nb, ib):
    o = tq.opts(precision=getattr(tq, prec))
    for shape, seed in (((1024, 768), 11), ((600, 300), 12)):
        A = synth.uniform(seed, *shape)
        print(f"noalloc {prec} nb={nb} ib={ib} {shape[0]}x{shape[1]}", flush=True)
        ref, out, T_ref, T_out = _factor_both(tq, A, nb, ib, o)
        assert torch.equal(ref, out), "factored A differs from tileqr_factor_ex"
        used = tq.t_size(*shape, nb, ib)
        assert torch.equal(T_ref[:used], T_out[:used]), "T differs from tileqr_factor_ex"


def test_noalloc_refuses_shapes_beyond_its_array(tq):
    # 4096 x 4096 needs 128 MiB of tiles alone: refused on the host, A untouched.
    m = n = 4096
    At = torch.ones((n, m), dtype=torch.float64, device="cuda")
    T = torch.zeros(tq.t_size(m, n, 256, 32), dtype=torch.float64, device="cuda")
    rc = tq.factor_noalloc(m, n, At.data_ptr(), m, 256, 32, T.data_ptr(), None)
    torch.cuda.synchronize()
    assert rc == tq.ENOMEM
    assert bool((At == 1.0).all())


def test_noalloc_bad_arguments_and_flags(tq):
    assert tq.factor_noalloc(-1, 4, 0, 1, 64, 16, 0, None) == -1
    At = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    T = torch.zeros(tq.t_size(8, 8, 64, 16), dtype=torch.float64, device="cuda")
    assert tq.factor_noalloc(8, 8, At.data_ptr(), 4, 64, 16, T.data_ptr(), None) == -4
    o = tq.opts(flags=tq.FLAG_TRACE)
    assert tq.factor_noalloc(8, 8, At.data_ptr(), 8, 64, 16, T.data_ptr(), o) == tq.EUNSUPPORTED
    assert tq.factor_noalloc(0, 8, At.data_ptr(), 1, 64, 16, T.data_ptr(), None) == tq.OK
