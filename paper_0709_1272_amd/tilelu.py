"""ctypes binding of the tiled LU entry points (``include/tilelu.h``) in
``libtileqr.so``.  Argument marshalling only: every step of the
factorisation runs in the library's HIP kernels; importing fails loudly when
the library has not been built (through ``tileqr``)."""
import ctypes

from . import tileqr as _tq

_L = _tq._L


class LUInfo(ctypes.Structure):
    _fields_ = [("minor", ctypes.c_int64), ("ms_factor", ctypes.c_double), ("ms_worker", ctypes.c_double)]


class LUSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("eta", ctypes.c_double),
                ("minor", ctypes.c_int64)]


_i64 = ctypes.c_int64
_SIGS = {
    "tilelu_lup_size": (ctypes.c_size_t, [_i64, _i64, _i64]),
    "tilelu_piv_size": (ctypes.c_size_t, [_i64, _i64]),
    "tilelu_factor": (ctypes.c_int, [_i64, ctypes.c_void_p, _i64, _i64, _i64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(_tq.Opts), ctypes.POINTER(LUInfo)]),
    "tilelu_solve": (ctypes.c_int, [_i64, _i64, ctypes.c_void_p, _i64, ctypes.c_void_p, _i64, ctypes.c_void_p, _i64,
                                    _i64, ctypes.POINTER(_tq.Opts), ctypes.POINTER(LUSolveInfo)]),
    "tilelu_dag_counts": (_i64, [_i64, ctypes.POINTER(_i64)]),
    "tilelu_dag_selfcheck": (ctypes.c_int, [_i64, _i64, ctypes.c_uint64]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = sorted(_SIGS)


def solve(n, nrhs, A, lda, B, ldb, X, ldx, ib=0, o=None, info=None):
    """tilelu_solve on device pointers; returns the status."""
    return _L.tilelu_solve(n, nrhs, A, lda, B, ldb, X, ldx, ib, ctypes.byref(o) if o is not None else None,
                           ctypes.byref(info) if info is not None else None)


def lup_size(n, nb, ib):
    return int(_L.tilelu_lup_size(n, nb, ib))


def piv_size(n, nb):
    return int(_L.tilelu_piv_size(n, nb))


def factor(n, A, lda, nb, ib, Lup, piv, o=None, info=None):
    """tilelu_factor on device pointers; returns the status."""
    return _L.tilelu_factor(n, A, lda, nb, ib, Lup, piv, ctypes.byref(o) if o is not None else None,
                            ctypes.byref(info) if info is not None else None)


def dag_counts(p):
    c = (_i64 * 4)()
    total = _L.tilelu_dag_counts(p, c)
    return total, list(c)


def dag_selfcheck(p, trials=3, seed=1):
    return _L.tilelu_dag_selfcheck(p, trials, seed)


def flops(n):
    """2 n^3 / 3: the leading-order operation count of the LU factorisation."""
    return 2.0 * n ** 3 / 3.0


def factor_tensor(At, n, nb=64, ib=16, o=None):
    """Factor the column-major n x n matrix in tensor At (shape (n, lda)) in
    place; returns (status, Lup tensor, piv tensor, LUInfo)."""
    import torch
    Lup = torch.zeros(max(lup_size(n, nb, ib), 1), dtype=torch.float64, device=At.device)
    piv = torch.zeros(max(piv_size(n, nb), 1), dtype=torch.int32, device=At.device)
    info = LUInfo()
    rc = factor(n, At.data_ptr(), At.shape[1], nb, ib, Lup.data_ptr(), piv.data_ptr(), o, info)
    return rc, Lup, piv, info
