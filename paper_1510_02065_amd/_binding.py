"""ctypes binding of libqap_rlt2.so (include/qap_rlt2.h).

Argument marshalling only: every step of the dual ascent runs in the HIP
library.  Importing this module does not touch the GPU; the first call loads
the library and raises if it has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqap_rlt2.so")

QAP_OK, QAP_EINVAL, QAP_ENOMEM, QAP_EDEVICE, QAP_ESTATE = 0, -1, -2, -3, -4
QAP_FP64, QAP_FP32_CERTIFIED, QAP_FP32_NEAREST = 0, 1, 2
# Precision names of the Python API: "fp32" is the certified mode (every
# write rounded toward -inf), "fp32n" the round-to-nearest mode.
PRECISIONS = {"fp64": QAP_FP64, "fp32": QAP_FP32_CERTIFIED, "fp32n": QAP_FP32_NEAREST}
QAP_LAP_DEVICE, QAP_LAP_RESIDUAL, QAP_LAP_AUCTION = 1, 2, 4
SOLVERS = {"canonical": 0, "auction": 1}
MAX_N = 64

# Every function the header declares, with (restype, argtypes).
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("trace_level", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("tune_cache", ctypes.c_char_p), ("complementary", ctypes.c_int), ("K", ctypes.c_double),
                ("UB", ctypes.c_double), ("level", ctypes.c_int), ("lap_solver", ctypes.c_int),
                ("overlap", ctypes.c_int)]


class BnbParams(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("root_iters", ctypes.c_int), ("iters", ctypes.c_int), ("K", ctypes.c_double),
                ("UB", ctypes.c_double), ("strong_iters", ctypes.c_int), ("leaf_size", ctypes.c_int),
                ("max_nodes", ctypes.c_int64), ("checkpoint", ctypes.c_char_p),
                ("checkpoint_every", ctypes.c_int64), ("resume", ctypes.c_int)]


class BnbResult(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("perm", ctypes.c_int32 * MAX_N), ("root_bound", ctypes.c_double),
                ("nodes", ctypes.c_int64), ("pruned", ctypes.c_int64), ("leaves", ctypes.c_int64),
                ("complete", ctypes.c_int)]


SIGNATURES = {
    "qap_rlt2_default_opts": (ctypes.c_int, [ctypes.POINTER(Opts)]),
    "qap_rlt2_create": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.POINTER(_vp)]),
    "qap_rlt2_create_ex": (ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                          ctypes.POINTER(Opts), ctypes.POINTER(_vp)]),
    "qap_rlt2_ascend": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "qap_rlt2_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "qap_rlt2_certify": (ctypes.c_int, [_vp, _dp]),
    "qap_rlt2_bound": (ctypes.c_int, [_vp, _dp, _i64p]),
    "qap_rlt2_trace": (ctypes.c_int, [_vp, ctypes.c_int64, _i64p, _dp, _dp]),
    "qap_rlt2_lap_values": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "qap_rlt2_read_state": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "qap_rlt2_destroy": (None, [_vp]),
    "qap_lap_solve": (ctypes.c_int, [ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp,
                                     ctypes.c_int, _vp]),
    "qap_lap_solve_noalloc": (ctypes.c_int, [ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp,
                                             ctypes.c_int, _vp]),
    "qap_last_error": (ctypes.c_char_p, []),
    "qap_rlt2_batch_create": (ctypes.c_int, [ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts),
                                             ctypes.POINTER(_vp)]),
    "qap_rlt2_count": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "qap_rlt2_batch_bounds": (ctypes.c_int, [_vp, _dp, _dp]),
    "qap_rlt2_instance_trace": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int64, _i64p, _dp, _dp]),
    "qap_rlt2_instance_lap_values": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp, _dp]),
    "qap_rlt2_instance_state": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp, _dp, _dp]),
    "qap_subproblem": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.c_int, _vp, _vp, _dp, _dp, _dp, _dp]),
    "qap_rlt2_set_stop": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
    "qap_rlt2_batch_status": (ctypes.c_int, [_vp, _vp, _vp]),
    "qap_rlt2_instance_assignment": (ctypes.c_int, [_vp, ctypes.c_int, _vp]),
    "qap_rlt2_load_state": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp, _dp, _dp]),
    "qap_rlt2_snapshot": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]),
    "qap_rlt2_restore": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64]),
    "qap_rlt2_children": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int,
                                         ctypes.POINTER(_vp)]),
    "qap_rlt2_strong_branch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]),
    "qap_objective": (ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _vp, _dp]),
    "qap_ub_local_search": (ctypes.c_int, [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _vp, _dp]),
    "qap_bnb_default_params": (ctypes.c_int, [ctypes.POINTER(BnbParams)]),
    "qap_bnb_solve": (ctypes.c_int, [ctypes.c_int, _dp, _dp, ctypes.POINTER(BnbParams),
                                     ctypes.POINTER(BnbResult)]),
}

_lib = None


class QapError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where} failed with status {status}: {message}")
        self.status = status


def lib():
    """Load libqap_rlt2.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python paper_1510_02065_amd/build.py")
        # One HIP runtime per process: torch ships its own copy of
        # libamdhip64.so.7 and loads it by file name, so if this library loaded
        # the system copy first the process would hold two runtimes and torch
        # would see no GPU.  Importing torch first makes the dynamic loader
        # resolve this library's libamdhip64.so.7 to torch's already-loaded one.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, where):
    if status != QAP_OK:
        raise QapError(status, where, lib().qap_last_error().decode(errors="replace"))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _opts(precision, trace_level, use_graph, device, stream, autotune=True, tune_cache=None,
          complementary=True, K=0.0, UB=0.0, level=2, lap_solver="canonical",
          overlap=True):
    opts = Opts()
    _check(lib().qap_rlt2_default_opts(ctypes.byref(opts)), "qap_rlt2_default_opts")
    opts.precision = PRECISIONS[precision]
    opts.K = float(K)
    opts.UB = float(UB)
    opts.level = int(level)
    opts.lap_solver = SOLVERS[lap_solver]
    opts.overlap = 1 if overlap else 0
    opts.device = device
    opts.stream = stream
    opts.trace_level = trace_level
    opts.use_graph = 1 if use_graph else 0
    opts.autotune = 1 if autotune else 0
    opts.tune_cache = None if tune_cache is None else str(tune_cache).encode()
    opts.complementary = 1 if complementary else 0
    return opts


class Rlt2:
    """One RLT2 dual-ascent state on the GPU (qap_rlt2_* calls).  A handle
    made by Rlt2.batch holds several instances; the plain accessors then
    refer to instance 0 and the *_k accessors to instance k."""

    def __init__(self, F, D, B0=None, constant=0.0, precision="fp64", trace_level=1,
                 use_graph=True, device=-1, stream=None, autotune=True, tune_cache=None,
                 complementary=True, K=0.0, UB=0.0, level=2, lap_solver="canonical",
          overlap=True):
        L = lib()
        F = _f64(F)
        D = _f64(D)
        N = F.shape[0]
        if F.shape != (N, N) or D.shape != (N, N):
            raise ValueError("F and D must be square and of the same size")
        B0 = None if B0 is None else _f64(B0)
        opts = _opts(precision, trace_level, use_graph, device, stream, autotune, tune_cache, complementary,
                     K, UB, level, lap_solver, overlap)
        h = _vp()
        _check(L.qap_rlt2_create_ex(N, _dptr(F), _dptr(D), _dptr(B0), float(constant),
                                    ctypes.byref(opts), ctypes.byref(h)), "qap_rlt2_create_ex")
        self._h = h
        self.N = N
        self.Ns = [N]
        self.precision = precision

    @classmethod
    def batch(cls, Fs, Ds, B0s=None, constants=None, precision="fp64", trace_level=1,
              use_graph=True, device=-1, stream=None, autotune=True, tune_cache=None,
              complementary=True, K=0.0, UB=0.0, level=2, lap_solver="canonical",
          overlap=True):
        """Many instances (e.g. branch-and-bound nodes) in one handle."""
        count = len(Fs)
        Fs = [_f64(F) for F in Fs]
        Ds = [_f64(D) for D in Ds]
        Ns = np.array([F.shape[0] for F in Fs], dtype=np.int32)
        B0s = [None if B is None else _f64(B) for B in (B0s or [None] * count)]
        consts = np.array(constants if constants is not None else [0.0] * count, dtype=np.float64)
        fp = (ctypes.c_void_p * count)(*[F.ctypes.data for F in Fs])
        dp = (ctypes.c_void_p * count)(*[D.ctypes.data for D in Ds])
        bp = (ctypes.c_void_p * count)(*[None if B is None else B.ctypes.data for B in B0s])
        opts = _opts(precision, trace_level, use_graph, device, stream, autotune, tune_cache, complementary,
                     K, UB, level, lap_solver, overlap)
        h = _vp()
        _check(lib().qap_rlt2_batch_create(count, Ns.ctypes.data, ctypes.cast(fp, _vp), ctypes.cast(dp, _vp),
                                           ctypes.cast(bp, _vp), consts.ctypes.data, ctypes.byref(opts),
                                           ctypes.byref(h)), "qap_rlt2_batch_create")
        self = cls.__new__(cls)
        self._h = h
        self.N = int(Ns[0])
        self.Ns = [int(n) for n in Ns]
        self.precision = precision
        self._keep = (Fs, Ds, B0s)
        return self

    @classmethod
    def _wrap(cls, h, Ns, precision):
        self = cls.__new__(cls)
        self._h = h
        self.N = int(Ns[0])
        self.Ns = [int(n) for n in Ns]
        self.precision = precision
        return self

    def children(self, k, fac, loc, level=2):
        """Children of instance k (qap_rlt2_children): child c fixes facility
        fac[c] at location loc[c] (instance k's indices), inheriting its
        reduced costs."""
        fac = np.ascontiguousarray(fac, dtype=np.int32)
        loc = np.ascontiguousarray(loc, dtype=np.int32)
        h = _vp()
        _check(lib().qap_rlt2_children(self._h, int(k), len(fac), fac.ctypes.data, loc.ctypes.data, int(level),
                                       ctypes.byref(h)), "qap_rlt2_children")
        return Rlt2._wrap(h, [self.Ns[k] - 1] * len(fac), self.precision)

    def strong_branch(self, k=0, iters=2):
        """Strong branching at instance k: (kind, index, bounds N x N)."""
        N = self.Ns[k]
        bounds = np.empty(N * N)
        kind = ctypes.c_int()
        index = ctypes.c_int()
        _check(lib().qap_rlt2_strong_branch(self._h, int(k), int(iters), _dptr(bounds), ctypes.byref(kind),
                                            ctypes.byref(index)), "qap_rlt2_strong_branch")
        return kind.value, index.value, bounds.reshape(N, N)

    def set_stop(self, K, UB):
        _check(lib().qap_rlt2_set_stop(self._h, float(K), float(UB)), "qap_rlt2_set_stop")

    def status(self):
        """(active flags, loop iterations run) per instance."""
        K = len(self.Ns)
        act = np.empty(K, dtype=np.int32)
        its = np.empty(K, dtype=np.int64)
        _check(lib().qap_rlt2_batch_status(self._h, act.ctypes.data, its.ctypes.data), "qap_rlt2_batch_status")
        return act, its

    def assignment(self, k=0):
        perm = np.empty(self.Ns[k], dtype=np.int32)
        _check(lib().qap_rlt2_instance_assignment(self._h, int(k), perm.ctypes.data),
               "qap_rlt2_instance_assignment")
        return perm

    def load_state(self, k=0, lb=None, B=None, C=None, D=None):
        lbv = None if lb is None else np.array([float(lb)])
        args = [None if a is None else _f64(a).ravel() for a in (B, C, D)]
        _check(lib().qap_rlt2_load_state(self._h, int(k), _dptr(lbv), *[_dptr(a) for a in args]),
               "qap_rlt2_load_state")

    def snapshot(self):
        """The handle's snapshot as bytes (qap_rlt2_snapshot)."""
        size = ctypes.c_uint64()
        _check(lib().qap_rlt2_snapshot(self._h, None, 0, ctypes.byref(size)), "qap_rlt2_snapshot")
        buf = ctypes.create_string_buffer(size.value)
        _check(lib().qap_rlt2_snapshot(self._h, buf, size.value, ctypes.byref(size)), "qap_rlt2_snapshot")
        return buf.raw[: size.value]

    def restore(self, data):
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        _check(lib().qap_rlt2_restore(self._h, buf, len(data)), "qap_rlt2_restore")

    def count(self):
        c = ctypes.c_int()
        _check(lib().qap_rlt2_count(self._h, ctypes.byref(c)), "qap_rlt2_count")
        return c.value

    def bounds(self, certified=False):
        """Per-instance LB (and certified bounds when certified=True)."""
        K = len(self.Ns)
        lb = np.empty(K)
        cert = np.empty(K) if certified else None
        _check(lib().qap_rlt2_batch_bounds(self._h, _dptr(lb), _dptr(cert)), "qap_rlt2_batch_bounds")
        return (lb, cert) if certified else lb

    def trace_k(self, k):
        cnt = ctypes.c_int64()
        _check(lib().qap_rlt2_instance_trace(self._h, k, 0, ctypes.byref(cnt), None, None), "qap_rlt2_instance_trace")
        lb = np.empty(cnt.value)
        lbp = np.empty(cnt.value)
        _check(lib().qap_rlt2_instance_trace(self._h, k, cnt.value, ctypes.byref(cnt), _dptr(lb), _dptr(lbp)),
               "qap_rlt2_instance_trace")
        return lb, lbp

    def lap_values_k(self, k):
        N = self.Ns[k]
        sD = np.empty(N * N * (N - 1) * (N - 1))
        sC = np.empty(N * N)
        sB = np.empty(1)
        _check(lib().qap_rlt2_instance_lap_values(self._h, k, _dptr(sD), _dptr(sC), _dptr(sB)),
               "qap_rlt2_instance_lap_values")
        return sD, sC, float(sB[0])

    def read_state_k(self, k, want_D=True):
        N = self.Ns[k]
        B = np.empty(N * N)
        C = np.empty(N * N * (N - 1) ** 2)
        D = np.empty(N * N * (N - 1) ** 2 * (N - 2) ** 2) if want_D else None
        lb = np.empty(1)
        _check(lib().qap_rlt2_instance_state(self._h, k, _dptr(lb), _dptr(B), _dptr(C), _dptr(D)),
               "qap_rlt2_instance_state")
        return float(lb[0]), B, C, D

    def close(self):
        if getattr(self, "_h", None):
            lib().qap_rlt2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def ascend(self, iters=1):
        out = ctypes.c_double()
        _check(lib().qap_rlt2_ascend(self._h, int(iters), ctypes.byref(out)), "qap_rlt2_ascend")
        return out.value

    def step(self, step):
        _check(lib().qap_rlt2_step(self._h, int(step)), "qap_rlt2_step")

    def certify(self):
        out = ctypes.c_double()
        _check(lib().qap_rlt2_certify(self._h, ctypes.byref(out)), "qap_rlt2_certify")
        return out.value

    def bound(self):
        lb = ctypes.c_double()
        it = ctypes.c_int64()
        _check(lib().qap_rlt2_bound(self._h, ctypes.byref(lb), ctypes.byref(it)), "qap_rlt2_bound")
        return lb.value, it.value

    def trace(self):
        cnt = ctypes.c_int64()
        _check(lib().qap_rlt2_trace(self._h, 0, ctypes.byref(cnt), None, None), "qap_rlt2_trace")
        lb = np.empty(cnt.value)
        lbp = np.empty(cnt.value)
        _check(lib().qap_rlt2_trace(self._h, cnt.value, ctypes.byref(cnt), _dptr(lb), _dptr(lbp)),
               "qap_rlt2_trace")
        return lb, lbp

    def lap_values(self):
        N = self.N
        sD = np.empty(N * N * (N - 1) * (N - 1))
        sC = np.empty(N * N)
        sB = np.empty(1)
        _check(lib().qap_rlt2_lap_values(self._h, _dptr(sD), _dptr(sC), _dptr(sB)), "qap_rlt2_lap_values")
        return sD, sC, float(sB[0])

    def read_state(self, want_D=True):
        N = self.N
        B = np.empty(N * N)
        C = np.empty(N * N * (N - 1) ** 2)
        D = np.empty(N * N * (N - 1) ** 2 * (N - 2) ** 2) if want_D else None
        lb = np.empty(1)
        _check(lib().qap_rlt2_read_state(self._h, _dptr(lb), _dptr(B), _dptr(C), _dptr(D)),
               "qap_rlt2_read_state")
        return float(lb[0]), B, C, D


def objective(F, D, perm, B0=None, constant=0.0):
    """QAP objective of perm (qap_objective)."""
    F = _f64(F)
    D = _f64(D)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    B0 = None if B0 is None else _f64(B0)
    out = ctypes.c_double()
    _check(lib().qap_objective(F.shape[0], _dptr(F), _dptr(D), _dptr(B0), float(constant), perm.ctypes.data,
                               ctypes.byref(out)), "qap_objective")
    return out.value


def local_search(F, D, perm, B0=None, constant=0.0):
    """Pairwise-exchange descent from perm (qap_ub_local_search): (perm, value)."""
    F = _f64(F)
    D = _f64(D)
    p = np.array(perm, dtype=np.int32)
    B0 = None if B0 is None else _f64(B0)
    out = ctypes.c_double()
    _check(lib().qap_ub_local_search(F.shape[0], _dptr(F), _dptr(D), _dptr(B0), float(constant), p.ctypes.data,
                                     ctypes.byref(out)), "qap_ub_local_search")
    return p, out.value


def bnb_solve(F, D, **kw):
    """Branch and bound (qap_bnb_solve).  Keyword arguments set the fields of
    qap_bnb_params (precision as a name); returns a dict of the result."""
    F = _f64(F)
    D = _f64(D)
    N = F.shape[0]
    prm = BnbParams()
    _check(lib().qap_bnb_default_params(ctypes.byref(prm)), "qap_bnb_default_params")
    for key, val in kw.items():
        if key == "precision":
            val = PRECISIONS[val]
        elif key == "checkpoint":
            val = None if val is None else str(val).encode()
        elif key == "stream":
            val = None if val is None else int(val)
        setattr(prm, key, val)
    res = BnbResult()
    _check(lib().qap_bnb_solve(N, _dptr(F), _dptr(D), ctypes.byref(prm), ctypes.byref(res)), "qap_bnb_solve")
    return {"value": res.value, "perm": np.array(res.perm[:N], dtype=np.int32), "root_bound": res.root_bound,
            "nodes": res.nodes, "pruned": res.pruned, "leaves": res.leaves, "complete": bool(res.complete)}


def subproblem(F, D, fac, loc):
    """Branch-and-bound node: fix facility fac[t] at location loc[t].
    Returns (Fsub, Dsub, B0sub, constant) (qap_subproblem)."""
    F = _f64(F)
    D = _f64(D)
    N = F.shape[0]
    fac = np.ascontiguousarray(fac, dtype=np.int32)
    loc = np.ascontiguousarray(loc, dtype=np.int32)
    m = len(fac)
    M = N - m
    Fs = np.empty((M, M))
    Ds = np.empty((M, M))
    Bs = np.empty((M, M))
    c = ctypes.c_double()
    _check(lib().qap_subproblem(N, _dptr(F), _dptr(D), m, fac.ctypes.data, loc.ctypes.data, _dptr(Fs),
                                _dptr(Ds), _dptr(Bs), ctypes.byref(c)), "qap_subproblem")
    return Fs, Ds, Bs, c.value


def lap_solve(mats, residual=False, want_duals=True, want_assign=True, auction=False):
    """Solve a batch of square host matrices (list of 2-D arrays, FP64);
    auction=True: by the auction algorithm instead of the canonical dual.

    Returns dict with 'value' (S per problem), 'duals' (list of (4, n)
    arrays: uc, vc, ur, vr), 'assign' (list of row->column arrays) and, with
    residual=True, 'residual' (list of n x n arrays)."""
    mats = [_f64(m) for m in mats]
    batch = len(mats)
    n = np.array([m.shape[0] for m in mats], dtype=np.int32)
    mat_off = np.zeros(batch, dtype=np.int64)
    vec_off = np.zeros(batch, dtype=np.int64)
    if batch:
        mat_off[1:] = np.cumsum(n.astype(np.int64) ** 2)[:-1]
        vec_off[1:] = np.cumsum(n.astype(np.int64))[:-1]
    total_m = int((n.astype(np.int64) ** 2).sum())
    total_v = int(n.sum())
    cost = np.concatenate([m.ravel() for m in mats]) if batch else np.zeros(0)
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    value = np.empty(batch)
    duals = np.empty(4 * total_v) if want_duals else None
    assign = np.empty(total_v, dtype=np.int32) if want_assign else None
    flags = (QAP_LAP_RESIDUAL if residual else 0) | (QAP_LAP_AUCTION if auction else 0)
    _check(lib().qap_lap_solve(batch, n.ctypes.data, mat_off.ctypes.data, vec_off.ctypes.data,
                               cost.ctypes.data if total_m else None, QAP_FP64, value.ctypes.data,
                               None if duals is None else duals.ctypes.data,
                               None if assign is None else assign.ctypes.data, flags, None),
           "qap_lap_solve")
    out = {"value": value}
    if want_duals:
        out["duals"] = [duals[4 * vec_off[b]: 4 * vec_off[b] + 4 * n[b]].reshape(4, n[b]) for b in range(batch)]
    if want_assign:
        out["assign"] = [assign[vec_off[b]: vec_off[b] + n[b]] for b in range(batch)]
    if residual:
        out["residual"] = [cost[mat_off[b]: mat_off[b] + n[b] ** 2].reshape(n[b], n[b]) for b in range(batch)]
    return out


def lap_solve_device(n, mat_off, vec_off, cost, value, duals=None, assign=None, residual=False,
                     stream=None, fp32=False, nearest=False, auction=False):
    """Device-pointer batch: every argument is a torch CUDA tensor (or None);
    the call is asynchronous on `stream` (a torch.cuda.Stream or None)."""
    ptr = (lambda t: None if t is None else t.data_ptr())
    flags = QAP_LAP_DEVICE | (QAP_LAP_RESIDUAL if residual else 0) | (QAP_LAP_AUCTION if auction else 0)
    sp = None if stream is None else stream.cuda_stream
    _check(lib().qap_lap_solve(int(n.numel()), ptr(n), ptr(mat_off), ptr(vec_off), ptr(cost),
                               (QAP_FP32_NEAREST if nearest else QAP_FP32_CERTIFIED) if fp32 else QAP_FP64,
                               ptr(value), ptr(duals),
                               ptr(assign), flags, sp), "qap_lap_solve")
