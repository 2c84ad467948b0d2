"""ctypes binding of ``libtileqr.so`` (declared in ``include/tileqr.h``).

Argument marshalling only: every step of the factorisation and of the
solvers runs in the library's HIP kernels.  Functions take device pointers
(ints) exactly like the C entry points; the ``*_tensor`` helpers accept torch
CUDA tensors holding column-major FP64 matrices (a column-major m x n matrix
is a contiguous torch tensor of shape (n, m)).

Importing this module fails loudly when the library has not been built:
there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtileqr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                      f"g.build()'` (hipcc, gfx950)")

_L = ctypes.CDLL(LIB_PATH)

OK, EHIP, ENONFINITE, ENOCONV, ETIMEOUT, ENOMEM, EUNSUPPORTED, ESINGULAR, ENOTSPD = range(9)
FP64, BF16X2, FP16X2, BF16X3 = range(4)
FLAG_ASYNC, FLAG_SERIAL, FLAG_TRACE, FLAG_SHUFFLE, FLAG_TIMING, FLAG_NO_GRAPH, FLAG_CHECK = 1, 2, 4, 8, 16, 32, 64


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("nb", ctypes.c_int64), ("ib", ctypes.c_int64),
                ("max_iter", ctypes.c_int), ("tol", ctypes.c_double), ("stream", ctypes.c_void_p),
                ("flags", ctypes.c_uint), ("seed", ctypes.c_uint64), ("spin_limit", ctypes.c_int64),
                ("workers", ctypes.c_int64), ("drop_edge", ctypes.c_int64),
                ("panel_workers", ctypes.c_int64), ("panel_tasks", ctypes.c_int64),
                ("apply_group", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int64), ("ib", ctypes.c_int64), ("panel_workers", ctypes.c_int64),
                ("workers", ctypes.c_int64), ("ms", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int64), ("not_converged", ctypes.c_int64), ("max_iterations", ctypes.c_int),
                ("max_eta", ctypes.c_double), ("ms_factor", ctypes.c_double), ("ms_total", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("eta", ctypes.c_double),
                ("eta_hist", ctypes.c_double * 65), ("nb", ctypes.c_int64), ("ib", ctypes.c_int64),
                ("ms_factor", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("eta_ls", ctypes.c_double), ("eta_inf", ctypes.c_double),
                ("beta_fact_est", ctypes.c_double), ("probes", ctypes.c_int), ("ms_worker", ctypes.c_double)]


_i64, _int, _vp, _dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
_I64P = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "tileqr_opts_default": (None, [ctypes.POINTER(Opts)]),
    "tileqr_blocking_supported": (_int, [_i64, _i64]),
    "tileqr_choose_blocking": (_int, [_i64, _i64, _int, _I64P, _I64P]),
    "tileqr_t_size": (ctypes.c_size_t, [_i64, _i64, _i64, _i64]),
    "tileqr_factor": (_int, [_i64, _i64, _vp, _i64, _i64, _i64, _vp]),
    "tileqr_factor_ex": (_int, [_i64, _i64, _vp, _i64, _i64, _i64, _vp, ctypes.POINTER(Opts)]),
    "tileqr_factor_noalloc": (_int, [_i64, _i64, _vp, _i64, _i64, _i64, _vp, ctypes.POINTER(Opts)]),
    "tileqr_apply_qt": (_int, [_i64, _i64, _i64, _vp, _i64, _i64, _i64, _vp, _vp, _i64]),
    "tileqr_apply_q": (_int, [_i64, _i64, _i64, _vp, _i64, _i64, _i64, _vp, _vp, _i64]),
    "tileqr_solve_ls": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                               ctypes.POINTER(Opts), ctypes.POINTER(Info)]),
    "tileqr_tree_size": (ctypes.c_size_t, [_i64, _i64, _i64, _i64, _i64]),
    "tileqr_factor_tree": (_int, [_i64, _i64, _vp, _i64, _i64, _i64, _i64, _vp, ctypes.POINTER(Opts)]),
    "tileqr_apply_qt_tree": (_int, [_i64, _i64, _i64, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _i64]),
    "tileqr_apply_q_tree": (_int, [_i64, _i64, _i64, _vp, _i64, _i64, _i64, _i64, _vp, _vp, _i64]),
    "tileqr_solve_ls_tree": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64,
                                    ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_double)]),
    "tileqr_factor_batched": (_int, [_i64, _I64P, _I64P, ctypes.POINTER(_vp), _I64P, _I64P, _I64P,
                                     ctypes.POINTER(_vp), ctypes.POINTER(Opts)]),
    "tileqr_solve_ls_batched": (_int, [_i64, _I64P, _I64P, ctypes.POINTER(_vp), _I64P, ctypes.POINTER(_vp),
                                       ctypes.POINTER(_vp), ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(BatchInfo)]),
    "tileqr_tune": (_int, [_i64, _I64P, _I64P, _int, _int, ctypes.POINTER(Tuning)]),
    "tileqr_tune_save": (_i64, [ctypes.c_char_p]),
    "tileqr_tune_load": (_i64, [ctypes.c_char_p]),
    "tileqr_tune_lookup": (_int, [ctypes.c_char_p, _int, _i64, _I64P, _I64P, _int, ctypes.POINTER(Tuning)]),
    "tileqr_tune_clear": (None, []),
    "tileqr_flops_lapack": (_dbl, [_i64, _i64]),
    "tileqr_flops_tiled": (_dbl, [_i64, _i64, _i64, _i64]),
    "tileqr_dag_counts": (_i64, [_i64, _i64, _i64, _i64, _I64P]),
    "tileqr_dag_selfcheck": (_int, [_i64, _i64, _i64, _i64, _i64, ctypes.c_uint64]),
    "tileqr_trace": (_i64, [_I64P, _i64]),
    "tileqr_trace_clock_hz": (_dbl, []),
    "tileqr_last_timing": (_int, [ctypes.POINTER(ctypes.c_double)]),
    "tileqr_mfma_peak": (_int, [_int, ctypes.POINTER(ctypes.c_double)]),
    "tileqr_status_string": (ctypes.c_char_p, [_int]),
    "tileqr_last_hip_error": (ctypes.c_char_p, []),
    "tileqr_finalize": (_int, []),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = sorted(_SIGS)


class TileQRError(RuntimeError):
    def __init__(self, status, where):
        msg = _L.tileqr_status_string(status).decode()
        if status == EHIP:
            msg += ": " + _L.tileqr_last_hip_error().decode()
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


def opts(**kw):
    o = Opts()
    _L.tileqr_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr_opts(o):
    return ctypes.byref(o) if o is not None else None


# ------------------------------------------------------------ raw entry points

def blocking_supported(nb, ib):
    return bool(_L.tileqr_blocking_supported(nb, ib))


def choose_blocking(m, n, precision=FP64):
    nb, ib = ctypes.c_int64(), ctypes.c_int64()
    _L.tileqr_choose_blocking(m, n, precision, ctypes.byref(nb), ctypes.byref(ib))
    return nb.value, ib.value


def t_size(m, n, nb, ib):
    return int(_L.tileqr_t_size(m, n, nb, ib))


def factor(m, n, A, lda, nb, ib, T, o=None):
    if o is None:
        return _L.tileqr_factor(m, n, A, lda, nb, ib, T)
    return _L.tileqr_factor_ex(m, n, A, lda, nb, ib, T, _ptr_opts(o))


def factor_noalloc(m, n, A, lda, nb, ib, T, o=None):
    return _L.tileqr_factor_noalloc(m, n, A, lda, nb, ib, T, _ptr_opts(o))


def apply_qt(m, n, nrhs, A, lda, nb, ib, T, B, ldb):
    return _L.tileqr_apply_qt(m, n, nrhs, A, lda, nb, ib, T, B, ldb)


def apply_q(m, n, nrhs, A, lda, nb, ib, T, B, ldb):
    return _L.tileqr_apply_q(m, n, nrhs, A, lda, nb, ib, T, B, ldb)


def solve_ls(m, n, nrhs, A, lda, B, ldb, X, ldx, o=None, info=None):
    return _L.tileqr_solve_ls(m, n, nrhs, A, lda, B, ldb, X, ldx, _ptr_opts(o),
                              ctypes.byref(info) if info is not None else None)


def tree_size(m, n, nb, ib, leaves):
    return int(_L.tileqr_tree_size(m, n, nb, ib, leaves))


def factor_tree(m, n, A, lda, nb, ib, leaves, F, o=None):
    return _L.tileqr_factor_tree(m, n, A, lda, nb, ib, leaves, F, _ptr_opts(o))


def apply_qt_tree(m, n, nrhs, A, lda, nb, ib, leaves, F, B, ldb):
    return _L.tileqr_apply_qt_tree(m, n, nrhs, A, lda, nb, ib, leaves, F, B, ldb)


def apply_q_tree(m, n, nrhs, A, lda, nb, ib, leaves, F, B, ldb):
    return _L.tileqr_apply_q_tree(m, n, nrhs, A, lda, nb, ib, leaves, F, B, ldb)


def solve_ls_tree(m, n, nrhs, A, lda, B, ldb, X, ldx, nb, ib, leaves, o=None):
    """Returns (status, device milliseconds of the call)."""
    ms = ctypes.c_double(0.0)
    rc = _L.tileqr_solve_ls_tree(m, n, nrhs, A, lda, B, ldb, X, ldx, nb, ib, leaves, _ptr_opts(o), ctypes.byref(ms))
    return rc, ms.value


def solve_ls_batched(ms, ns, A_ptrs, ldas, b_ptrs, x_ptrs, o=None, info=None):
    """Returns (status, eta list, iterations list)."""
    b = len(ms)
    arr = lambda vals: (ctypes.c_int64 * b)(*[int(v) for v in vals])
    ptrs = lambda vals: (ctypes.c_void_p * b)(*[int(v) for v in vals])
    eta = (ctypes.c_double * b)()
    its = (ctypes.c_int32 * b)()
    rc = _L.tileqr_solve_ls_batched(b, arr(ms), arr(ns), ptrs(A_ptrs), arr(ldas), ptrs(b_ptrs), ptrs(x_ptrs),
                                    _ptr_opts(o), eta, its, ctypes.byref(info) if info is not None else None)
    return rc, list(eta), list(its)


def factor_batched(ms, ns, A_ptrs, ldas, nbs, ibs, T_ptrs, o=None):
    b = len(ms)
    arr = lambda vals: (ctypes.c_int64 * b)(*[int(v) for v in vals])
    ptrs = lambda vals: (ctypes.c_void_p * b)(*[int(v) for v in vals])
    return _L.tileqr_factor_batched(b, arr(ms), arr(ns), ptrs(A_ptrs), arr(ldas),
                                    arr(nbs) if nbs is not None else None,
                                    arr(ibs) if ibs is not None else None, ptrs(T_ptrs), _ptr_opts(o))


def tune(ms, ns, precision=FP64, trials=2):
    """Autotune (tileqr_tune) for matrices of these shapes; returns a Tuning
    (nb, ib, panel_workers, workers, ms) and raises on an error status."""
    b = len(ms)
    arr = lambda vals: (ctypes.c_int64 * b)(*[int(v) for v in vals])
    t = Tuning()
    check(_L.tileqr_tune(b, arr(ms), arr(ns), precision, trials, ctypes.byref(t)), "tileqr_tune")
    return t


def tune_save(path):
    """Write the tuner's table to a text file; returns the entry count."""
    r = _L.tileqr_tune_save(os.fsencode(path))
    if r < 0:
        raise OSError(f"tileqr_tune_save({path!r}) returned {r}")
    return r


def tune_load(path):
    """Add the entries of a file written by tune_save; returns their count."""
    r = _L.tileqr_tune_load(os.fsencode(path))
    if r < 0:
        raise OSError(f"tileqr_tune_load({path!r}) returned {r}")
    return r


def tune_lookup(arch, cu, ms, ns, precision=FP64):
    """The tuned entry the automatic blocking would use on a device of this
    architecture and CU count (exact shapes, else the size class), or None."""
    b = len(ms)
    arr = lambda vals: (ctypes.c_int64 * b)(*[int(v) for v in vals])
    t = Tuning()
    r = _L.tileqr_tune_lookup(arch.encode(), cu, b, arr(ms), arr(ns), precision, ctypes.byref(t))
    if r < 0:
        raise ValueError(f"tileqr_tune_lookup: argument {-r}")
    return t if r == 1 else None


def tune_clear():
    _L.tileqr_tune_clear()


def flops_lapack(m, n):
    return _L.tileqr_flops_lapack(m, n)


def flops_tiled(m, n, nb, ib):
    return _L.tileqr_flops_tiled(m, n, nb, ib)


def dag_counts(p, q, strips=1, panels=1):
    c = (ctypes.c_int64 * 5)()
    total = _L.tileqr_dag_counts(p, q, strips, panels, c)
    return total, list(c)


def dag_selfcheck(p, q, strips, trials, seed, panels=1):
    return _L.tileqr_dag_selfcheck(p, q, strips, panels, trials, seed)


TRACE_WORDS = 10


def trace():
    """(events, clock_hz): events are tuples (type, k, i, j, strip, worker,
    t_pop, t_start, t_body_end, t_end) in device clock ticks."""
    n = _L.tileqr_trace(None, 0)
    buf = (ctypes.c_int64 * (TRACE_WORDS * max(n, 1)))()
    n = _L.tileqr_trace(buf, n)
    return [tuple(buf[TRACE_WORDS * e: TRACE_WORDS * (e + 1)]) for e in range(n)], _L.tileqr_trace_clock_hz()


def last_timing():
    """[layout in, scheduler set-up, factorisation kernel(s), layout out] in ms."""
    ms = (ctypes.c_double * 4)()
    check(_L.tileqr_last_timing(ms), "tileqr_last_timing")
    return list(ms)


def mfma_peak(kind):
    """Measured MFMA rate in TFLOP/s: kind 0 FP64 16x16x4, 1 BF16 16x16x32,
    2 FP16 16x16x32."""
    t = ctypes.c_double()
    check(_L.tileqr_mfma_peak(kind, ctypes.byref(t)), "tileqr_mfma_peak")
    return t.value


def status_string(s):
    return _L.tileqr_status_string(s).decode()


def finalize():
    return _L.tileqr_finalize()


def check(status, where):
    if status != OK:
        raise TileQRError(status, where)


# ------------------------------------------------------- torch conveniences

def _torch():
    import torch
    return torch


def to_device(M, device="cuda"):
    """Column-major device copy of a host matrix (numpy or torch): returns a
    contiguous (n, m) float64 tensor whose storage is M column-major."""
    torch = _torch()
    t = torch.as_tensor(M, dtype=torch.float64)
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    return t.t().contiguous().to(device)


def to_host(t, m=None):
    """Inverse of to_device: numpy (m, n) array from a (n, ld) column-major tensor."""
    a = t.detach().cpu().numpy().T
    return a[:m] if m is not None else a


def factor_tensor(At, m, nb, ib, o=None):
    """Factor the column-major matrix in tensor At (shape (n, lda)) in place;
    returns the T tensor."""
    torch = _torch()
    n, lda = At.shape
    T = torch.empty(max(t_size(m, n, nb, ib), 1), dtype=torch.float64, device=At.device)
    check(factor(m, n, At.data_ptr(), lda, nb, ib, T.data_ptr(), o), "tileqr_factor")
    return T
