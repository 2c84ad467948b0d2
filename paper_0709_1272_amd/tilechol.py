"""ctypes binding of the tiled Cholesky entry points (``include/tilechol.h``)
in ``libtileqr.so``.  Argument marshalling only: every step of the
factorisation runs in the library's HIP kernels; importing fails loudly when
the library has not been built (through ``tileqr``)."""
import ctypes

from . import tileqr as _tq

_L = _tq._L


class CholInfo(ctypes.Structure):
    _fields_ = [("minor", ctypes.c_int64), ("nb", ctypes.c_int64), ("ms_factor", ctypes.c_double),
                ("ms_worker", ctypes.c_double)]


_i64 = ctypes.c_int64
_SIGS = {
    "tilechol_factor": (ctypes.c_int, [_i64, ctypes.c_void_p, _i64, _i64, ctypes.POINTER(_tq.Opts),
                                       ctypes.POINTER(CholInfo)]),
    "tilechol_solve": (ctypes.c_int, [_i64, _i64, ctypes.c_void_p, _i64, ctypes.c_void_p, _i64, _i64,
                                      ctypes.POINTER(_tq.Opts)]),
    "tilechol_dag_counts": (_i64, [_i64, ctypes.POINTER(_i64)]),
    "tilechol_dag_selfcheck": (ctypes.c_int, [_i64, _i64, ctypes.c_uint64]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = sorted(_SIGS)


def factor(n, A, lda, nb=0, o=None, info=None):
    """tilechol_factor on a device pointer; returns the status."""
    return _L.tilechol_factor(n, A, lda, nb, ctypes.byref(o) if o is not None else None,
                              ctypes.byref(info) if info is not None else None)


def solve(n, nrhs, L, ldl, B, ldb, nb=0, o=None):
    """tilechol_solve on device pointers (B overwritten with X); returns the status."""
    return _L.tilechol_solve(n, nrhs, L, ldl, B, ldb, nb, ctypes.byref(o) if o is not None else None)


def dag_counts(p):
    c = (_i64 * 3)()
    total = _L.tilechol_dag_counts(p, c)
    return total, list(c)


def dag_selfcheck(p, trials=3, seed=1):
    return _L.tilechol_dag_selfcheck(p, trials, seed)


def flops(n):
    """n^3 / 3: the leading-order operation count of the Cholesky factorisation."""
    return n ** 3 / 3.0


def factor_tensor(At, n, nb=0, o=None):
    """Factor the lower triangle of the column-major n x n matrix in tensor At
    (shape (n, lda)) in place; returns (status, CholInfo)."""
    info = CholInfo()
    lda = At.shape[1]
    return factor(n, At.data_ptr(), lda, nb, o, info), info
