"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Mirrors the oracle's C entry points one to one; no arithmetic happens here.
"""
from __future__ import annotations

import ctypes as C
import numpy as np

from . import build as _build

NSCALARS = 16
STATUS = {0: "NOT_SOLVED", 1: "OPTIMAL", 2: "ITERATION_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL",
          5: "PRIMAL_INFEASIBLE", 6: "DUAL_INFEASIBLE"}
SCALAR_NAMES = ["eta_hat", "omega", "W", "KKT0", "KKT_prev", "k", "t", "attempts", "restarts",
                "status", "eta_last"]


class _Opts(C.Structure):
    _fields_ = [("ruiz_iters", C.c_int), ("pc_alpha", C.c_double), ("check_every", C.c_int),
                ("kkt_p", C.c_double), ("fixed_step", C.c_int), ("fixed_eta", C.c_double),
                ("infeas_tol", C.c_double)]


_lib = None
_libs = {}


def lib(path=None):
    """The oracle library (the built one, or a planted-mistake build at `path`)."""
    global _lib
    if path is not None:
        if path not in _libs:
            _libs[path] = _bind(C.CDLL(path))
        return _libs[path]
    if _lib is None:
        _lib = _bind(C.CDLL(_build.build(force=False)))
    return _lib


def _bind(L):
    """Declare the argument and result types of the oracle's entry points."""
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    L.orc_load.argtypes = [C.POINTER(C.c_void_p), C.c_int64, C.c_int64, C.c_int64, ip, ip, dp,
                           dp, dp, dp, dp, C.c_int64, C.POINTER(_Opts)]
    L.orc_load.restype = C.c_int
    L.orc_set_start.argtypes = [C.c_void_p, dp, dp]
    L.orc_set_start_weight.argtypes = [C.c_void_p, C.c_double]
    L.orc_solve.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_double]
    L.orc_result.argtypes = [C.c_void_p, dp, dp, dp, dp]
    L.orc_state_len.argtypes = [C.c_void_p]
    L.orc_state_len.restype = C.c_int64
    L.orc_get_state.argtypes = [C.c_void_p, dp]
    L.orc_set_state.argtypes = [C.c_void_p, dp]
    L.orc_get_scaling.argtypes = [C.c_void_p, dp, dp, dp]
    L.orc_spmv.argtypes = [C.c_void_p, C.c_int, dp, dp]
    L.orc_eval_unscaled.argtypes = [C.c_void_p, dp, dp, dp]
    L.orc_free.argtypes = [C.c_void_p]
    L.orc_step_next.argtypes = [C.c_double, C.c_double, C.c_int64]
    L.orc_step_next.restype = C.c_double
    L.orc_restart_decision.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int64]
    L.orc_restart_decision.restype = C.c_int
    L.orc_omega_update.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_omega_update.restype = C.c_double
    L.orc_kkt_omega.argtypes = [C.c_void_p, dp, dp, C.c_double]
    L.orc_kkt_omega.restype = C.c_double
    return L


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


class Oracle:
    """One LP loaded into the oracle."""

    def __init__(self, lp, ruiz_iters=10, pc_alpha=1.0, check_every=64, kkt_p=2.0,
                 fixed_step=False, fixed_eta=0.0, infeas_tol=1e-8, libpath=None):
        L = lib(libpath)
        self.L = L
        self.m, self.n, self.m1 = int(lp.m), int(lp.n), int(lp.m1)
        o = _Opts(ruiz_iters, pc_alpha, check_every, kkt_p, int(bool(fixed_step)), fixed_eta, infeas_tol)
        self._keep = [np.ascontiguousarray(lp.row_ptr, np.int32), np.ascontiguousarray(lp.col, np.int32),
                      _f64(lp.val), _f64(lp.c), _f64(lp.q), _f64(lp.l), _f64(lp.u)]
        rp, ci, v, c, q, l, u = self._keep
        h = C.c_void_p()
        rc = L.orc_load(C.byref(h), self.m, self.n, int(rp[-1]) if rp.size else 0, _ip(rp), _ip(ci),
                        _dp(v), _dp(c), _dp(q), _dp(l), _dp(u), self.m1, C.byref(o))
        if rc != 0:
            raise OracleError(rc)
        self.h = h
        self.nnz = int(rp[-1])

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and getattr(self, "L", None) is not None:
            self.L.orc_free(h)
            self.h = None

    def set_start(self, x=None, y=None):
        xs = None if x is None else _f64(x)
        ys = None if y is None else _f64(y)
        self.L.orc_set_start(self.h, _dp(xs), _dp(ys))

    def set_start_weight(self, omega):
        self.L.orc_set_start_weight(self.h, float(omega))

    def solve(self, tol=1e-4, max_iters=10**6, time_limit=0.0):
        rc = self.L.orc_solve(self.h, tol, int(max_iters), float(time_limit))
        if rc != 0:
            raise OracleError(rc)
        return self.result()

    def result(self):
        x = np.empty(self.n); y = np.empty(self.m); lam = np.empty(self.n); info = np.zeros(16)
        rc = self.L.orc_result(self.h, _dp(x), _dp(y), _dp(lam), _dp(info))
        if rc != 0:
            raise OracleError(rc)
        d = dict(status=STATUS[int(info[0])], pobj=info[1], dobj=info[2], rel_p=info[3],
                 rel_d=info[4], rel_g=info[5], iterations=int(info[6]), attempts=int(info[7]),
                 restarts=int(info[8]), omega=info[9], eta=info[10], seconds=info[11])
        d["rel_kkt"] = max(d["rel_p"], d["rel_d"], d["rel_g"])
        return x, y, lam, d

    def get_state(self):
        buf = np.empty(self.L.orc_state_len(self.h))
        self.L.orc_get_state(self.h, _dp(buf))
        return unpack_state(buf, self.n, self.m)

    def get_state_raw(self):
        buf = np.empty(self.L.orc_state_len(self.h))
        self.L.orc_get_state(self.h, _dp(buf))
        return buf

    def set_state_raw(self, buf):
        buf = _f64(buf)
        self.L.orc_set_state(self.h, _dp(buf))

    def scaling(self):
        Dr = np.empty(self.m); Dc = np.empty(self.n); kv = np.empty(self.nnz)
        self.L.orc_get_scaling(self.h, _dp(Dr), _dp(Dc), _dp(kv))
        return Dr, Dc, kv

    def spmv(self, v, transpose=False):
        v = _f64(v)
        out = np.empty(self.n if transpose else self.m)
        self.L.orc_spmv(self.h, int(bool(transpose)), _dp(v), _dp(out))
        return out

    def kkt_omega(self, x_scaled, y_scaled, omega):
        x = _f64(x_scaled); y = _f64(y_scaled)
        return self.L.orc_kkt_omega(self.h, _dp(x), _dp(y), float(omega))

    def eval_unscaled(self, x, y):
        out = np.empty(7)
        x = _f64(x); y = _f64(y)
        self.L.orc_eval_unscaled(self.h, _dp(x), _dp(y), _dp(out))
        return dict(rel_p=out[0], rel_d=out[1], rel_g=out[2], pobj=out[3], dobj=out[4],
                    bound_viol=out[5], sign_viol=out[6], rel_kkt=max(out[0], out[1], out[2]))


STATE_VECTORS = [("x", "n"), ("y", "m"), ("Kx", "m"), ("KTy", "n"), ("xbar", "n"), ("ybar", "m"),
                 ("Kxbar", "m"), ("KTybar", "n"), ("x0", "n"), ("y0", "m")]


def unpack_state(buf, n, m):
    """Split a flat state (16 scalars then 10 vectors) into a dict."""
    d = {name: buf[i] for i, name in enumerate(SCALAR_NAMES)}
    p = NSCALARS
    for name, dim in STATE_VECTORS:
        ln = n if dim == "n" else m
        d[name] = buf[p:p + ln].copy()
        p += ln
    return d


def step_next(eta, eta_bar, k):
    return lib().orc_step_next(eta, eta_bar, k)


def restart_decision(kkt_c, kkt0, kkt_prev, t, k):
    return lib().orc_restart_decision(kkt_c, kkt0, kkt_prev, t, k)


def omega_update(omega, dx, dy):
    return lib().orc_omega_update(omega, dx, dy)
