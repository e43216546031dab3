"""FP64 CPU oracle for the RLT2 dual ascent (arXiv 1510.02065).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
library (`paper_1510_02065_amd`) and neither imports the other; both are fed
the same seeded instances from `qapgen`.

The heavy lifting is plain C (`rlt2_oracle.c`) loaded with ctypes; the
pure-Python helpers for tiny cases live in `oracle.brute`.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _build.needs_build():
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    vp = ctypes.c_void_p
    lib.oracle_lap_solve.argtypes = [ctypes.c_int, dp, ip]
    lib.oracle_lap_solve.restype = ctypes.c_double
    lib.oracle_lap_canonical_dual.argtypes = [ctypes.c_int, dp, ip, dp, dp, dp, dp]
    lib.oracle_lap_canonical_dual.restype = None
    lib.oracle_lap_concentrate.argtypes = [ctypes.c_int, dp, dp, dp, ip]
    lib.oracle_lap_concentrate.restype = ctypes.c_double
    lib.oracle_rlt2_new.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double]
    lib.oracle_rlt2_new.restype = vp
    lib.oracle_rlt2_free.argtypes = [vp]
    lib.oracle_rlt2_free.restype = None
    for name in ("oracle_rlt2_iteration0",):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = None
    lib.oracle_rlt2_step.argtypes = [vp, ctypes.c_int]
    lib.oracle_rlt2_step.restype = None
    lib.oracle_rlt2_iterate.argtypes = [vp, ctypes.c_int]
    lib.oracle_rlt2_iterate.restype = None
    lib.oracle_rlt2_N.argtypes = [vp]
    lib.oracle_rlt2_N.restype = ctypes.c_int
    for name in ("oracle_rlt2_lb", "oracle_rlt2_last_lbprime"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = ctypes.c_double
    for name in ("oracle_rlt2_B", "oracle_rlt2_C", "oracle_rlt2_D",
                 "oracle_rlt2_SD", "oracle_rlt2_SC"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = dp
    lib.oracle_rlt2_set_lb.argtypes = [vp, ctypes.c_double]
    lib.oracle_rlt2_set_lb.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n threads (results do not change)."""
    _load().oracle_set_threads(int(n))


def lap_solve(M):
    """Optimal assignment of square M: returns (value, row2col)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = M.shape[0]
    r2c = np.empty(n, dtype=np.int32)
    val = _load().oracle_lap_solve(n, _dptr(M), _iptr(r2c))
    return float(val), r2c


def lap_canonical_dual(M, row2col):
    """Canonical dual points (uc, vc, ur, vr) of M for an optimal row2col."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = M.shape[0]
    r2c = np.ascontiguousarray(row2col, dtype=np.int32)
    out = [np.empty(n) for _ in range(4)]
    _load().oracle_lap_canonical_dual(n, _dptr(M), _iptr(r2c), *[_dptr(o) for o in out])
    return tuple(out)


def lap_concentrate(M):
    """Cost concentration of one block: returns (S, R, duals[4,n], row2col)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = M.shape[0]
    R = np.empty_like(M)
    duals = np.empty((4, n))
    r2c = np.empty(n, dtype=np.int32)
    S = _load().oracle_lap_concentrate(n, _dptr(M), _dptr(R), _dptr(duals), _iptr(r2c))
    return float(S), R, duals, r2c


class Rlt2Oracle:
    """Dense-state FP64 RLT2 dual ascent (Algorithm 1 of the paper).

    State arrays are exposed as numpy views: B[i,j], C[i,j,k,n],
    D[i,j,k,n,p,q]; entries with repeated facility or location indices are
    unused (zero).  SD[i,j,k,n] and SC[i,j] hold the values moved by the most
    recent D->C and C->B concentrations.
    """

    def __init__(self, F, D, B0=None, constant=0.0):
        lib = _load()
        self._F = np.ascontiguousarray(F, dtype=np.float64)
        self._D = np.ascontiguousarray(D, dtype=np.float64)
        N = self._F.shape[0]
        self._B0 = None if B0 is None else np.ascontiguousarray(B0, dtype=np.float64)
        h = lib.oracle_rlt2_new(N, _dptr(self._F), _dptr(self._D),
                                None if self._B0 is None else _dptr(self._B0),
                                float(constant))
        if not h:
            raise ValueError("oracle_rlt2_new failed (N < 3 or out of memory)")
        self._h = ctypes.c_void_p(h)
        self.N = N

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_rlt2_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iteration0(self):
        _load().oracle_rlt2_iteration0(self._h)

    def step(self, k: int):
        _load().oracle_rlt2_step(self._h, int(k))

    def iterate(self, T: int = 1):
        _load().oracle_rlt2_iterate(self._h, int(T))

    @property
    def lb(self) -> float:
        return float(_load().oracle_rlt2_lb(self._h))

    @lb.setter
    def lb(self, value: float):
        _load().oracle_rlt2_set_lb(self._h, float(value))

    @property
    def lbprime(self) -> float:
        return float(_load().oracle_rlt2_last_lbprime(self._h))

    def _view(self, fn, shape):
        p = getattr(_load(), fn)(self._h)
        size = int(np.prod(shape))
        return np.ctypeslib.as_array(p, shape=(size,)).reshape(shape)

    @property
    def B(self):
        return self._view("oracle_rlt2_B", (self.N,) * 2)

    @property
    def C(self):
        return self._view("oracle_rlt2_C", (self.N,) * 4)

    @property
    def D(self):
        return self._view("oracle_rlt2_D", (self.N,) * 6)

    @property
    def SD(self):
        return self._view("oracle_rlt2_SD", (self.N,) * 4)

    @property
    def SC(self):
        return self._view("oracle_rlt2_SC", (self.N,) * 2)
