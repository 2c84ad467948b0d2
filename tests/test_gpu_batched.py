"""GPU tests of the batched factorisation (tileqr_factor_batched) and the
autotuner (tileqr_tune), through the C-ABI.

Every matrix of a batch must equal, bit for bit, tileqr_factor on that
matrix alone with the same blocking (each matrix is its own DAG, the tile
kernels are deterministic); the graph replay, the direct launch and
batches with several blockings must agree with it; a seeded sample is
compared with the oracle (R up to row signs, normwise).
"""
import numpy as np
import pytest

import oracle
from paper_0709_1272_amd import synth
from test_gpu_factor import rebuild_q, r_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tq():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0709_1272_amd import tileqr
    return tileqr


class Batch:
    """Column-major matrices (lda = m) carved from one device buffer, and T
    areas sized for the largest blocking used."""

    def __init__(self, tq, mats, tsize_nb=((64, 16),)):
        self.tq = tq
        self.m = [a.shape[0] for a in mats]
        self.n = [a.shape[1] for a in mats]
        sizes = [a.size for a in mats]
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        host = np.concatenate([np.asarray(a, order="F").ravel(order="F") for a in mats]) if mats else np.zeros(0)
        self.buf = torch.from_numpy(host.copy()).to("cuda")
        ts = [max([tq.t_size(m, n, b, s) for b, s in tsize_nb] + [1]) for m, n in zip(self.m, self.n)]
        self.toff = np.concatenate([[0], np.cumsum(ts)]).astype(np.int64)
        self.T = torch.zeros(int(self.toff[-1]) + 1, dtype=torch.float64, device="cuda")

    def ptrs(self):
        a0, t0 = self.buf.data_ptr(), self.T.data_ptr()
        return [a0 + 8 * int(o) for o in self.off[:-1]], [t0 + 8 * int(o) for o in self.toff[:-1]]

    def factor(self, nbs=None, ibs=None, **opt):
        A, T = self.ptrs()
        o = self.tq.opts(**opt) if opt else None
        rc = self.tq.factor_batched(self.m, self.n, A, [max(1, m) for m in self.m], nbs, ibs, T, o)
        torch.cuda.synchronize()
        return rc

    def result(self, i):
        h = self.buf[int(self.off[i]):int(self.off[i + 1])].cpu().numpy()
        return h.reshape(self.n[i], self.m[i]).T.copy()

    def tblock(self, i, nb, ib):
        return self.T[int(self.toff[i]):int(self.toff[i]) + self.tq.t_size(self.m[i], self.n[i], nb, ib)].cpu().numpy()


def single(tq, A, nb, ib, **opt):
    m, n = A.shape
    At = tq.to_device(A)
    o = tq.opts(**opt) if opt else None
    T = tq.factor_tensor(At, m, nb, ib, o)
    torch.cuda.synchronize()
    return tq.to_host(At, m), T.cpu().numpy()


def used_t(T, m, n, nb, ib):
    """The T blocks a factorisation writes: tile (i, k) with i >= k (the
    blocks with i < k are never used)."""
    p, q = -(-m // nb), -(-n // nb)
    return np.concatenate([T[(k * p + i) * ib * nb:(k * p + i + 1) * ib * nb]
                           for k in range(min(p, q)) for i in range(k, p)])


def small_batch(seed, count, m_hi=300):
    m, n, mats = synth.batch_matrices(seed, count=count, m_hi=m_hi)
    return mats


@pytest.mark.parametrize("nb,ib", [(64, 16), (128, 32)])
def test_batched_bitwise_equals_single(tq, nb, ib):
    mats = small_batch(1, 40)
    B = Batch(tq, mats, [(nb, ib)])
    assert B.factor([nb] * 40, [ib] * 40) == tq.OK
    for i in range(0, 40, 3):
        F, T = single(tq, mats[i], nb, ib)
        assert np.array_equal(B.result(i), F), i
        m, n = mats[i].shape
        assert np.array_equal(used_t(B.tblock(i, nb, ib), m, n, nb, ib), used_t(T, m, n, nb, ib)), i


def test_graph_replay_and_direct_launch_agree(tq):
    mats = small_batch(2, 30)
    B1 = Batch(tq, mats)
    assert B1.factor([64] * 30, [16] * 30) == tq.OK          # captures
    B2 = Batch(tq, mats)
    assert B2.factor([64] * 30, [16] * 30) == tq.OK          # replays with new pointers
    B3 = Batch(tq, mats)
    assert B3.factor([64] * 30, [16] * 30, flags=tq.FLAG_NO_GRAPH) == tq.OK
    for i in range(30):
        r1 = B1.result(i)
        assert np.array_equal(r1, B2.result(i)), i
        assert np.array_equal(r1, B3.result(i)), i
    assert torch.equal(B1.T, B2.T) and torch.equal(B1.T, B3.T)
    # A replay after a single-matrix call still sees valid buffers.
    single(tq, mats[0], 128, 32)
    B4 = Batch(tq, mats)
    assert B4.factor([64] * 30, [16] * 30) == tq.OK
    assert torch.equal(B1.buf, B4.buf)


def test_batch_of_one_uses_panel_tasks(tq):
    # A batch of one matrix with few tile steps is scheduled like a single
    # call (one task per inner panel); a two-matrix batch of the same shapes
    # keeps whole tile kernels.  All give the same bits.
    A = synth.uniform(8, 1100, 700)
    F, T = single(tq, A, 128, 32)
    B1 = Batch(tq, [A], [(128, 32)])
    assert B1.factor([128], [32]) == tq.OK
    assert np.array_equal(B1.result(0), F)
    B2 = Batch(tq, [A, A], [(128, 32)])
    assert B2.factor([128] * 2, [32] * 2) == tq.OK
    assert np.array_equal(B2.result(0), F) and np.array_equal(B2.result(1), F)
    Bp = Batch(tq, [A, A], [(128, 32)])
    assert Bp.factor([128] * 2, [32] * 2, panel_tasks=4) == tq.OK
    assert np.array_equal(Bp.result(1), F)


def test_groups_of_blockings(tq):
    mats = small_batch(3, 24)
    nbs = [64, 128, 256] * 8
    ibs = [16, 32, 32] * 8
    B = Batch(tq, mats, [(64, 16), (128, 32), (256, 32)])
    assert B.factor(nbs, ibs) == tq.OK
    for i in range(24):
        F, T = single(tq, mats[i], nbs[i], ibs[i])
        assert np.array_equal(B.result(i), F), i


def test_mixed_precision_batch(tq):
    mats = small_batch(4, 20)
    B = Batch(tq, mats, [(64, 32)])
    assert B.factor([64] * 20, [32] * 20, precision=tq.BF16X3) == tq.OK
    for i in range(0, 20, 4):
        F, _ = single(tq, mats[i], 64, 32, precision=tq.BF16X3)
        assert np.array_equal(B.result(i), F), i


def test_batched_vs_oracle_sample(tq):
    mats = small_batch(5, 60, m_hi=500)
    B = Batch(tq, mats, [(64, 16)])
    assert B.factor([64] * 60, [16] * 60) == tq.OK
    for i in range(0, 60, 5):
        A = mats[i]
        F = B.result(i)
        Fo, _ = oracle.geqr2(A)
        d = oracle.r_diff(r_of(F), oracle.r_factor(Fo))
        assert d <= 1e-12, (i, A.shape, d)
        if i % 15 == 0:
            m, n = A.shape
            Q = rebuild_q(F, B.tblock(i, 64, 16), 64, 16)[:m, :m]
            RR = np.zeros((m, n))
            k = min(m, n)
            RR[:k] = r_of(F)
            assert np.linalg.norm(A - Q @ RR) <= 1e-14 * np.linalg.norm(A)


def test_empty_and_nonfinite(tq):
    mats = small_batch(6, 6)
    mats.insert(2, np.zeros((0, 5)))
    mats.insert(4, np.zeros((7, 0)))
    B = Batch(tq, mats)
    assert B.factor([64] * 8, [16] * 8) == tq.OK
    F, _ = single(tq, mats[0], 64, 16)
    assert np.array_equal(B.result(0), F)
    bad = [a.copy() for a in mats]
    bad[5][3, 1] = np.nan
    Bb = Batch(tq, bad)
    before = Bb.buf.clone()
    assert Bb.factor([64] * 8, [16] * 8) == tq.ENONFINITE
    assert torch.equal(torch.nan_to_num(before, nan=7.0), torch.nan_to_num(Bb.buf, nan=7.0))


def test_bad_arguments(tq):
    assert tq.factor_batched([5], [5], [1], [4], [64], [16], [1]) == -5
    assert tq.factor_batched([5], [5], [1], [5], [64], [48], [1]) == -7
    assert tq.factor_batched([5], [5], [0], [5], [64], [16], [1]) == -4
    assert tq.factor_batched([5], [5], [1], [5], [64], [16], [1], tq.opts(flags=tq.FLAG_SERIAL)) == tq.EUNSUPPORTED


def test_default_blocking_when_nothing_is_tuned(tq):
    # nb = ib = NULL for shapes the tuner has not seen: the library's own
    # blocking for the batch (the path takes the library lock only once).
    mats = small_batch(13, 10, m_hi=200)
    B = Batch(tq, mats, [(64, 16), (64, 32), (128, 16), (128, 32), (256, 16), (256, 32)])
    assert B.factor() == tq.OK
    for i in range(0, 10, 3):
        Fo, _ = oracle.geqr2(mats[i])
        assert oracle.r_diff(r_of(B.result(i)), oracle.r_factor(Fo)) <= 1e-12, i


def test_tuner_picks_a_supported_blocking_and_is_used(tq):
    mats = small_batch(7, 50)
    ms = [a.shape[0] for a in mats]
    ns = [a.shape[1] for a in mats]
    t = tq.tune(ms, ns, tq.FP64, trials=1)
    print(f"tuned: nb={t.nb} ib={t.ib} panel_workers={t.panel_workers} {t.ms:.3f} ms")
    assert tq.blocking_supported(t.nb, t.ib) and t.ms > 0
    B = Batch(tq, mats, [(64, 16), (64, 32), (128, 16), (128, 32), (256, 16), (256, 32)])
    assert B.factor() == tq.OK                               # nb = ib = NULL: the tuned choice
    for i in range(0, 50, 7):
        F, _ = single(tq, mats[i], t.nb, t.ib)
        assert np.array_equal(B.result(i), F), i
    # one matrix: tileqr_choose_blocking returns the tuned blocking
    t1 = tq.tune([1500], [700], tq.FP64, trials=1)
    assert tq.choose_blocking(1500, 700) == (t1.nb, t1.ib)


def test_tuned_entry_serves_its_size_class_and_persists(tq, tmp_path):
    # A tuned single shape also sets the blocking of shapes in its size class;
    # the table goes to a file and back, keyed by the device's kind.
    import torch
    t1 = tq.tune([1500], [700], tq.FP64, trials=1)
    assert tq.choose_blocking(1500, 700) == (t1.nb, t1.ib)
    assert tq.choose_blocking(1600, 600) == (t1.nb, t1.ib)       # same size class
    f = tmp_path / "tune.txt"
    assert tq.tune_save(str(f)) >= 1
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    assert arch in f.read_text()
    tq.tune_clear()
    try:
        assert tq.choose_blocking(1500, 700) == (128, 16)        # the untuned default
        assert tq.tune_load(str(f)) >= 1
        assert tq.choose_blocking(1500, 700) == (t1.nb, t1.ib)
        t = tq.tune_lookup(arch, props.multi_processor_count, [1500], [700])
        assert t is not None and (t.nb, t.ib) == (t1.nb, t1.ib)
    finally:
        tq.tune_clear()


def test_full_batched_config_sampled(tq):
    # 4000 matrices, m ~ U{32..768}, n ~ U{16..m}, N(0, 1), seed 0; one call.
    mats = synth.batch_matrices(0)[2]
    B = Batch(tq, mats, [(64, 16)])
    assert B.factor([64] * len(mats), [16] * len(mats)) == tq.OK
    sample = np.random.default_rng(11).choice(len(mats), size=25, replace=False)
    for i in sample:
        Fo, _ = oracle.geqr2(mats[i])
        assert oracle.r_diff(r_of(B.result(i)), oracle.r_factor(Fo)) <= 1e-12, i
    for i in sample[:5]:
        F, _ = single(tq, mats[i], 64, 16)
        assert np.array_equal(B.result(i), F), i
