"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every entry point the header declares, and its host-only DAG utilities agree
with Algorithm 2 (task counts, dependency rules) and with the cost model of
Section 3.2.3."""
import os
import re

import pytest

from conftest import ROOT


def _tq():
    lib = os.path.join(ROOT, "paper_0709_1272_amd", "libtileqr.so")
    if not os.path.exists(lib):
        pytest.skip("libtileqr.so not built")
    from paper_0709_1272_amd import tileqr
    return tileqr


def header_functions():
    text = open(os.path.join(ROOT, "include", "tileqr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tileqr_[a-z_0-9]+)\s*\(", text)))


def test_exports_match_header():
    tq = _tq()
    declared = header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(tq._L, name), f"{name} declared in include/tileqr.h but not exported"
    assert sorted(tq.EXPORTS) == declared


def test_dag_counts_p3q3():
    # Algorithm 2 on a 3 x 3 tile grid: 3 GEQRT, 3 TSQRT, 3 LARFB, 5 SSRFB.
    tq = _tq()
    total, c = tq.dag_counts(3, 3, 1)
    assert total == 14
    assert c == [3, 3, 3, 5, 0]


@pytest.mark.parametrize("p,q", [(1, 1), (4, 4), (8, 8), (32, 32), (256, 4), (3, 7), (7, 3)])
def test_dag_counts_closed_form(p, q):
    tq = _tq()
    kmax = min(p, q)
    geqrt = kmax
    tsqrt = sum(p - k - 1 for k in range(kmax))
    larfb = sum(q - k - 1 for k in range(kmax))
    ssrfb = sum((p - k - 1) * (q - k - 1) for k in range(kmax))
    for strips in (1, 8):
        for panels in (1, 4, 8):
            total, c = tq.dag_counts(p, q, strips, panels)
            # One panel per strip: every tile of column k gets, for each
            # panel l, one PUPD task per later strip.
            pupd = (sum(p - k for k in range(kmax)) * panels * (panels - 1) // 2
                    if panels == strips and panels > 1 else 0)
            assert c == [geqrt * panels, tsqrt * panels, larfb * strips, ssrfb * strips, pupd]
            assert total == sum(c)


@pytest.mark.parametrize("p,q,strips,trials", [(1, 1, 1, 3), (3, 3, 1, 50), (3, 3, 4, 50), (5, 2, 2, 50),
                                               (2, 6, 2, 50), (6, 6, 8, 20), (12, 4, 2, 10), (1, 5, 2, 10),
                                               (5, 1, 2, 10)])
@pytest.mark.parametrize("panels", [1, 2, 8])
def test_dag_rules_random_orders(p, q, strips, trials, panels):
    # Random topological orders of the scheduler's DAG must show every task
    # the tile versions that Algorithm 2's loop order shows it.
    tq = _tq()
    assert tq.dag_selfcheck(p, q, strips, trials, 1234 + p * 100 + q, panels) == 0


def test_flop_model():
    tq = _tq()
    # Per-kernel sum with s << b approaches 2n^2(m - n/3)(1 + s/(4b)) (Section 3.2.3).
    for (m, n, b, s) in ((8192, 8192, 256, 32), (65536, 1024, 256, 32), (32768, 32768, 256, 32)):
        tiled = tq.flops_tiled(m, n, b, s)
        model = 2.0 * n * n * (m - n / 3.0) * (1 + s / (4.0 * b))
        assert abs(tiled / model - 1) < 0.05, (m, n, tiled / model)
    # s = b costs 25 % more than the LAPACK count (Section 3.2.3).
    r = tq.flops_tiled(16384, 16384, 64, 64) / tq.flops_lapack(16384, 16384)
    assert abs(r - 1.25) < 0.02
    assert tq.flops_lapack(8192, 8192) == pytest.approx(2 * 8192**3 - 2 * 8192**3 / 3)


def test_blocking_rules():
    tq = _tq()
    for nb in (64, 128, 256):
        for ib in (16, 32):
            assert tq.blocking_supported(nb, ib)
    assert not tq.blocking_supported(96, 32)
    assert not tq.blocking_supported(64, 8)
    assert tq.t_size(512, 512, 64, 16) == 8 * 8 * 16 * 64
    assert tq.t_size(0, 5, 64, 16) == 0
    assert tq.t_size(100, 300, 64, 16) == 2 * 2 * 16 * 64   # p = 2, q = 5, min = 2


def test_automatic_blocking():
    # The untuned choice (the tuner's entries override it; none exist in a
    # fresh process): tiny -> 64/16, near-square up to 2048 -> 128/16, tall
    # and larger -> 256/32; the split modes always take ib = 32.
    tq = _tq()
    assert tq.choose_blocking(200, 100) == (64, 16)
    assert tq.choose_blocking(2048, 2048) == (128, 16)
    assert tq.choose_blocking(1024, 1500) == (128, 16)
    assert tq.choose_blocking(65536, 1024) == (256, 32)
    assert tq.choose_blocking(16384, 2048) == (256, 32)
    assert tq.choose_blocking(32768, 4096) == (256, 32)
    assert tq.choose_blocking(4096, 4096) == (256, 32)
    assert tq.choose_blocking(8192, 8192) == (256, 32)
    assert tq.choose_blocking(2048, 2048, tq.FP16X2) == (128, 32)
    assert tq.choose_blocking(65536, 1024, tq.BF16X3) == (256, 32)
    assert tq.choose_blocking(200, 100, tq.FP16X2) == (64, 32)
    for m, n in ((1, 1), (300, 7000), (100000, 64)):
        nb, ib = tq.choose_blocking(m, n)
        assert tq.blocking_supported(nb, ib)


def test_cli_arguments():
    # The driver's argument checks run before it touches a device.
    from paper_0709_1272_amd import cli
    with pytest.raises(SystemExit):
        cli.main(["qr", "--n", "8"])
    with pytest.raises(SystemExit):
        cli.main(["solve", "--n", "8", "--precision", "fp8"])
    with pytest.raises(SystemExit):
        cli.main(["solve"])


def _tune_line(arch, cu, nb, ib, pw, prec, shapes):
    key = [prec, len(shapes)] + [v for mn in sorted(shapes) for v in mn]
    return f"tileqr-tune-1 {arch} {cu} {nb} {ib} {pw} 0 1.5 {len(key)} " + " ".join(map(str, key))


def test_tune_table_file_exact_and_size_class(tmp_path):
    # The tuner's table survives the process through a text file and serves
    # shapes of the same size class (ceil log2 of the batch, of the typical
    # min(m, n) and of the largest m and n) when no entry has exactly theirs.
    tq = _tq()
    tq.tune_clear()
    try:
        f = tmp_path / "tune.txt"
        f.write_text("\n".join([
            _tune_line("gfx950", 256, 256, 32, 0, tq.FP64, [(8192, 8192)]),
            _tune_line("gfx950", 256, 128, 16, 32, tq.FP64, [(700, 300), (500, 500), (64, 40)]),
            _tune_line("gfx942", 304, 64, 16, 0, tq.FP64, [(8192, 8192)]),
            _tune_line("gfx950", 256, 128, 32, 0, tq.BF16X3, [(8192, 8192)]),
        ]) + "\n")
        assert tq.tune_load(str(f)) == 4
        t = tq.tune_lookup("gfx950", 256, [8192], [8192])
        assert (t.nb, t.ib, t.panel_workers) == (256, 32, 0)
        t = tq.tune_lookup("gfx950", 256, [8000], [7000])        # same class as 8192^2
        assert (t.nb, t.ib) == (256, 32)
        assert tq.tune_lookup("gfx950", 256, [4000], [4000]) is None   # next class down
        t = tq.tune_lookup("gfx942", 304, [8192], [8192])
        assert (t.nb, t.ib) == (64, 16)
        assert tq.tune_lookup("gfx950", 128, [8192], [8192]) is None   # other CU count
        t = tq.tune_lookup("gfx950", 256, [8192], [8192], tq.BF16X3)
        assert (t.nb, t.ib) == (128, 32)
        assert tq.tune_lookup("gfx950", 256, [8192], [8192], tq.FP16X2) is None
        t = tq.tune_lookup("gfx950", 256, [64, 500, 700], [40, 500, 300])   # the batch, any order
        assert (t.nb, t.ib, t.panel_workers) == (128, 16, 32)
        t = tq.tune_lookup("gfx950", 256, [60, 480, 690], [40, 490, 300])   # same class
        assert (t.nb, t.ib) == (128, 16)
        assert tq.tune_lookup("gfx950", 256, [700] * 9, [300] * 9) is None  # batch of 9: 4 > 2
        # Save, clear, load back: the same answers.
        g = tmp_path / "saved.txt"
        assert tq.tune_save(str(g)) == 4
        tq.tune_clear()
        assert tq.tune_lookup("gfx950", 256, [8192], [8192]) is None
        assert tq.tune_load(str(g)) == 4
        t = tq.tune_lookup("gfx950", 256, [8000], [7000])
        assert (t.nb, t.ib) == (256, 32)
        # Loading an entry with the same device kind and shapes replaces it.
        h = tmp_path / "newer.txt"
        h.write_text(_tune_line("gfx950", 256, 128, 32, 0, tq.FP64, [(8192, 8192)]) + "\n")
        assert tq.tune_load(str(h)) == 1
        assert tq.tune_save(str(g)) == 4
        t = tq.tune_lookup("gfx950", 256, [8192], [8192])
        assert (t.nb, t.ib) == (128, 32)
    finally:
        tq.tune_clear()


@pytest.mark.parametrize("line", [
    "tileqr-tune-2 gfx950 256 256 32 0 0 1.0 4 0 1 64 64",          # unknown version
    "tileqr-tune-1 gfx950 256 96 32 0 0 1.0 4 0 1 64 64",           # unsupported nb
    "tileqr-tune-1 gfx950 256 256 16 0 0 1.0 4 3 1 64 64",          # split precision with ib 16
    "tileqr-tune-1 gfx950 256 256 32 0 0 1.0 6 0 1 64 64 64 64",    # key longer than its batch
    "tileqr-tune-1 gfx950 256 256 32 0 0 1.0 4 0 1 64",             # key cut short
    "tileqr-tune-1 gfx950 256 256 32 0 0 1.0 4 0 1 64 64 7",        # trailing token
    "tileqr-tune-1 gfx950 0 256 32 0 0 1.0 4 0 1 64 64",            # no compute units
    "tileqr-tune-1 gfx950 256 256 32 0 0 1.0 4 0 1 -64 64",         # negative size
])
def test_tune_table_file_rejects_malformed_lines(tmp_path, line):
    tq = _tq()
    tq.tune_clear()
    try:
        f = tmp_path / "bad.txt"
        f.write_text(_tune_line("gfx950", 256, 256, 32, 0, tq.FP64, [(8192, 8192)]) + "\n" + line + "\n")
        with pytest.raises(OSError):
            tq.tune_load(str(f))
        assert tq.tune_lookup("gfx950", 256, [8192], [8192]) is None   # nothing loaded
        with pytest.raises(OSError):
            tq.tune_load(str(tmp_path / "missing.txt"))
    finally:
        tq.tune_clear()


def test_trace_export_format(tmp_path):
    # Chrome trace-event JSON from trace tuples (type, k, i, j, strip,
    # worker, t_pop, t_start, t_body_end, t_end): per task a body slice and,
    # when they take time, the acquire and the release slices.
    import json
    from paper_0709_1272_amd import trace
    ev = [(0, 0, 0, 0, 1, 0, 100, 110, 200, 210),
          (3, 0, 2, 1, 3, (1 << 16) | 5, 150, 150, 400, 420),
          (4, 0, 1, 2, 6, (1 << 16) | 7, 300, 305, 350, 350)]
    n = trace.write_chrome_json(str(tmp_path / "t.json"), ev, 1e8)   # 10 ns per tick
    data = json.loads((tmp_path / "t.json").read_text())["traceEvents"]
    assert n == len(data)
    bodies = [d for d in data if d["ph"] == "X" and d.get("cat") != "fence"]
    assert [d["name"] for d in bodies] == ["GEQRT(0,0) panel 1", "SSRFB(0,2,1) strip 3", "PUPD(0,1) panel 2 strip 6"]
    assert bodies[0]["ts"] == pytest.approx(0.1) and bodies[0]["dur"] == pytest.approx(0.9)
    assert bodies[1]["ts"] == pytest.approx(0.5) and bodies[1]["dur"] == pytest.approx(2.5)
    fences = [d for d in data if d.get("cat") == "fence"]
    assert len(fences) == 4   # acquire + release of the first, release of the second, acquire of the third
    names = {d["args"]["name"] for d in data if d["ph"] == "M" and d["name"] == "thread_name"}
    assert names == {"panel wg 0", "update wg 5", "update wg 7"}
    assert trace.chrome_events([], 1e8) == []


def test_tilechol_exports_match_header():
    _tq()
    from paper_0709_1272_amd import tilechol
    text = open(os.path.join(ROOT, "include", "tilechol.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(tilechol_[a-z_0-9]+)\s*\(", text)))
    assert declared and sorted(tilechol.EXPORTS) == declared
    for name in declared:
        assert hasattr(tilechol._L, name), name


def test_tilechol_dag_counts_and_selfcheck():
    # Algorithm 1 on a p x p tile grid: p POTF2, p(p-1)/2 TRSM and
    # (p-1)p(p+1)/6 GSMM (k < j <= i); the scheduler's in-degrees match its
    # successor lists and random topological orders respect every tile's
    # order of writes in Algorithm 1.
    _tq()
    from paper_0709_1272_amd import tilechol
    for p in (1, 2, 3, 4, 7, 16):
        total, c = tilechol.dag_counts(p)
        brute = [p, sum(1 for k in range(p) for i in range(k + 1, p)),
                 sum(1 for k in range(p) for i in range(k + 1, p) for j in range(k + 1, i + 1))]
        assert c == brute and total == sum(brute), p
        assert tilechol.dag_selfcheck(p, trials=4, seed=p) == 0, p
    assert tilechol.dag_selfcheck(0) == -1 and tilechol.dag_selfcheck(65) == -1


def test_tilechol_argument_checks_need_no_device():
    tq = _tq()
    from paper_0709_1272_amd import tilechol
    info = tilechol.CholInfo()
    assert tilechol.factor(-1, 0, 1) == -1
    assert tilechol.factor(4, 0, 4) == -2
    assert tilechol.factor(4, 1 << 20, 3) == -3
    assert tilechol.factor(4, 1 << 20, 4, 256) == -4
    assert tilechol.factor(4, 1 << 20, 4, 32) == -4
    assert tilechol.factor(4, 1 << 20, 4, 64, tq.opts(precision=7)) == -5
    assert tilechol.factor(4, 1 << 20, 4, 64, tq.opts(precision=tq.BF16X3), info) == tq.EUNSUPPORTED
    assert tilechol.factor(0, 0, 1, 0, None, info) == tq.OK and info.nb == 64
    assert tq.status_string(tq.ENOTSPD) == "matrix not positive definite"


def test_tilelu_exports_counts_selfcheck():
    # Algorithm 3 on a p x p grid: p GETRF, p(p-1)/2 GESSM and TSTRF, and
    # sum (p-k-1)^2 SSSSM; the scheduler's graph passes its self-check.
    _tq()
    from paper_0709_1272_amd import tilelu
    text = open(os.path.join(ROOT, "include", "tilelu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = sorted(set(re.findall(r"\b(tilelu_[a-z_0-9]+)\s*\(", text)))
    assert declared and sorted(tilelu.EXPORTS) == declared
    for p in (1, 2, 3, 6, 13):
        total, c = tilelu.dag_counts(p)
        brute = [p, p * (p - 1) // 2, p * (p - 1) // 2, sum((p - k - 1) ** 2 for k in range(p))]
        assert c == brute and total == sum(brute), p
        assert tilelu.dag_selfcheck(p, trials=4, seed=p) == 0, p
    assert tilelu.lup_size(0, 64, 16) == 0 and tilelu.lup_size(64, 32, 16) == 0


def test_tree_size_and_arguments():
    # The tree's storage: every leaf's T (leaves of h rows, h the largest
    # multiple of nb with leaves * h <= m, the last leaf the rest), then per
    # merge (up to four children) a stacked kn x n matrix and its T; argument
    # checks before any device work.
    tq = _tq()
    m, n, nb, ib, L = 5000, 300, 64, 16, 3
    h = (m // L) // nb * nb
    rows = [h, h, m - 2 * h]
    want = sum(tq.t_size(r, n, nb, ib) for r in rows) + 3 * n * n + tq.t_size(3 * n, n, nb, ib)
    assert tq.tree_size(m, n, nb, ib, L) == want
    # Six leaves: a merge of four and one of two, then a merge of those two.
    m, n, L = 6000, 100, 6
    h = (m // L) // nb * nb
    rows = [h] * 5 + [m - 5 * h]
    want = (sum(tq.t_size(r, n, nb, ib) for r in rows) + 4 * n * n + tq.t_size(4 * n, n, nb, ib)
            + 2 * (2 * n * n + tq.t_size(2 * n, n, nb, ib)))
    assert tq.tree_size(m, n, nb, ib, L) == want
    assert tq.tree_size(m, n, nb, ib, 1) == tq.t_size(m, n, nb, ib)
    assert tq.tree_size(1000, 300, 64, 16, 4) == 0           # leaves of 192 rows < n
    assert tq.tree_size(1000, 2000, 64, 16, 1) == 0          # not tall
    assert tq.factor_tree(-1, 1, 8, 1, 64, 16, 1, 8, None) == -1
    assert tq.factor_tree(10, 20, 8, 10, 64, 16, 1, 8, None) == -2
    assert tq.factor_tree(1000, 300, 8, 1000, 64, 16, 4, 8, None) == -7
    assert tq.factor_tree(1000, 300, 8, 1000, 64, 16, 2, 0, None) == -8
    assert tq.apply_qt_tree(1000, 300, 1, 8, 1000, 64, 16, 4, 8, 8, 1000) == -8
