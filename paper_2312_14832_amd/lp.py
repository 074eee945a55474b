"""Thin ctypes binding of libpdlp_amd.so (include/lp.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  The library must have been built (``paper_2312_14832_amd.build``);
importing this module on a machine without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdlp_amd.so")

LP_FP64, LP_MIXED = 0, 1
LP_HOST, LP_DEVICE = 0, 1
STATUS = {0: "NOT_SOLVED", 1: "OPTIMAL", 2: "ITERATION_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL",
          5: "PRIMAL_INFEASIBLE", 6: "DUAL_INFEASIBLE"}
ERRORS = {-1: "LP_ERR_ARG", -2: "LP_ERR_DIM", -3: "LP_ERR_NAN", -4: "LP_ERR_BOUNDS",
          -5: "LP_ERR_TOO_LARGE", -6: "LP_ERR_STATE", -7: "LP_ERR_HIP", -8: "LP_ERR_NOMEM"}
NSCALARS = 16

# every symbol include/lp.h declares
EXPORTS = ["lp_default_options", "lp_workspace_size", "lp_load", "lp_set_start", "lp_set_start_weight", "lp_solve", "lp_result", "lp_get_state",
           "lp_set_state", "lp_get_scaling", "lp_spmv", "lp_spmv_noalloc", "lp_gather_probe", "lp_kernel_time", "lp_device_bytes", "lp_layout",
           "lp_layout_blocks", "lp_layout_split", "lp_presolved_size", "lp_free",
           "lp_strerror", "lp_last_error", "lp_batch_load", "lp_batch_solve", "lp_batch_result",
           "lp_batch_get_state", "lp_batch_set_state", "lp_batch_device_bytes", "lp_batch_layout_blocks", "lp_batch_loop_form",
           "lp_batch_free",
           "lp_batch_last_error", "lp_shared_load", "lp_shared_set_start", "lp_shared_solve", "lp_shared_result",
           "lp_shared_get_state", "lp_shared_set_state", "lp_shared_device_bytes", "lp_shared_free",
           "lp_shared_last_error"]


class LPCsr(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class LPOptions(C.Structure):
    _fields_ = [("precision", C.c_int), ("stream", C.c_void_p), ("ruiz_iters", C.c_int),
                ("pc_alpha", C.c_double), ("check_every", C.c_int), ("kkt_omega_power", C.c_double),
                ("fixed_step", C.c_int), ("fixed_eta", C.c_double), ("use_graph", C.c_int),
                ("window", C.c_int), ("kernel_timing", C.c_int), ("slice_kib", C.c_int),
                ("autotune", C.c_int), ("verbose", C.c_int), ("ptr_kind", C.c_int),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("infeas_tol", C.c_double),
                ("presolve", C.c_int), ("persistent", C.c_int), ("split_sums", C.c_int)]


class LPInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("pobj", C.c_double), ("dobj", C.c_double),
                ("rel_primal", C.c_double), ("rel_dual", C.c_double), ("rel_gap", C.c_double),
                ("iterations", C.c_int64), ("attempts", C.c_int64), ("restarts", C.c_int64),
                ("omega", C.c_double), ("eta", C.c_double), ("seconds", C.c_double)]


_lib = None


def library():
    """Load libpdlp_amd.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_14832_amd.build`")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.lp_default_options.argtypes = [C.POINTER(LPOptions)]
        L.lp_default_options.restype = None
        L.lp_workspace_size.argtypes = [C.POINTER(LPCsr), C.POINTER(LPOptions), C.POINTER(C.c_size_t)]
        L.lp_load.argtypes = [C.POINTER(C.c_void_p), C.POINTER(LPCsr), dp, dp, dp, dp, C.c_int64,
                              C.POINTER(LPOptions)]
        L.lp_set_start.argtypes = [C.c_void_p, dp, dp]
        L.lp_set_start_weight.argtypes = [C.c_void_p, C.c_double]
        L.lp_solve.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_double]
        L.lp_result.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(LPInfo)]
        L.lp_get_state.argtypes = [C.c_void_p, dp, C.POINTER(C.c_int64)]
        L.lp_set_state.argtypes = [C.c_void_p, dp, C.c_int64]
        L.lp_get_scaling.argtypes = [C.c_void_p, dp, dp]
        L.lp_spmv.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.lp_spmv_noalloc.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.lp_gather_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_int, C.c_int64, C.c_void_p,
                                      C.c_int, C.c_void_p, C.POINTER(C.c_double)]
        L.lp_kernel_time.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.lp_device_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.lp_layout.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.lp_layout_blocks.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int)]
        L.lp_layout_split.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int)]
        L.lp_presolved_size.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lp_free.argtypes = [C.c_void_p]
        L.lp_free.restype = None
        L.lp_strerror.argtypes = [C.c_int]
        L.lp_strerror.restype = C.c_char_p
        L.lp_last_error.argtypes = [C.c_void_p]
        L.lp_last_error.restype = C.c_char_p
        PP = C.POINTER(C.POINTER(C.c_double))
        L.lp_batch_load.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(LPCsr), PP, PP, PP, PP,
                                    C.POINTER(C.c_int64), C.POINTER(LPOptions)]
        L.lp_batch_solve.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_double]
        L.lp_batch_result.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp, C.POINTER(LPInfo)]
        L.lp_batch_get_state.argtypes = [C.c_void_p, C.c_int32, dp, C.POINTER(C.c_int64)]
        L.lp_batch_set_state.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64]
        L.lp_batch_device_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.lp_batch_layout_blocks.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.lp_batch_loop_form.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.lp_batch_free.argtypes = [C.c_void_p]
        L.lp_batch_free.restype = None
        L.lp_batch_last_error.argtypes = [C.c_void_p]
        L.lp_batch_last_error.restype = C.c_char_p
        L.lp_shared_load.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(LPCsr), PP, PP, PP, PP, C.c_int64,
                                     C.POINTER(LPOptions)]
        L.lp_shared_set_start.argtypes = [C.c_void_p, C.c_int32, dp, dp, C.c_double]
        L.lp_shared_solve.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_double]
        L.lp_shared_result.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp, C.POINTER(LPInfo)]
        L.lp_shared_get_state.argtypes = [C.c_void_p, C.c_int32, dp, C.POINTER(C.c_int64)]
        L.lp_shared_set_state.argtypes = [C.c_void_p, C.c_int32, dp, C.c_int64]
        L.lp_shared_device_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.lp_shared_free.argtypes = [C.c_void_p]
        L.lp_shared_free.restype = None
        L.lp_shared_last_error.argtypes = [C.c_void_p]
        L.lp_shared_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class LPError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_options(**kw) -> LPOptions:
    """lp_options with the library defaults and the given fields.  precision
    and ptr_kind accept "fp64"/"mixed" and "host"/"device"; stream a
    torch.cuda.Stream; workspace a contiguous torch uint8 CUDA tensor."""
    o = LPOptions()
    library().lp_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": LP_FP64, "mixed": LP_MIXED}[v]
        if k == "ptr_kind" and isinstance(v, str):
            v = {"host": LP_HOST, "device": LP_DEVICE}[v]
        if k == "stream" and v is not None and not isinstance(v, int):
            v = int(v.cuda_stream)  # a torch.cuda.Stream
        if k == "workspace" and v is not None and not isinstance(v, int):
            assert v.is_cuda and v.is_contiguous()
            o.workspace_bytes = v.numel() * v.element_size()
            v = v.data_ptr()
        setattr(o, k, v)
    return o


def _ptr(a, ctype):
    """Host numpy array or device torch tensor -> typed pointer."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        assert a.is_cuda and a.is_contiguous()
        return C.cast(C.c_void_p(a.data_ptr()), C.POINTER(ctype))
    return a.ctypes.data_as(C.POINTER(ctype))


def _csr(lp, device):
    """LPCsr of lp.row_ptr / col / val (numpy, or torch CUDA tensors when device)."""
    if device:
        rp, ci, v = lp.row_ptr, lp.col, lp.val
        nnz = int(rp[-1].item())
    else:
        rp = np.ascontiguousarray(lp.row_ptr, np.int32)
        ci = np.ascontiguousarray(lp.col, np.int32)
        v = None if getattr(lp, "val", None) is None else _f64(lp.val)
        nnz = int(rp[-1])
    return LPCsr(int(lp.m), int(lp.n), nnz, _ptr(rp, C.c_int32), _ptr(ci, C.c_int32), _ptr(v, C.c_double)), (rp, ci, v)


def workspace_size(lp, **options):
    """Device bytes lp_load needs from a caller workspace (lp_workspace_size);
    runs on the host only."""
    o = default_options(**options)
    K, keep = _csr(lp, o.ptr_kind == LP_DEVICE)
    b = C.c_size_t()
    rc = library().lp_workspace_size(C.byref(K), C.byref(o), C.byref(b))
    if rc != 0:
        raise LPError(rc, library().lp_strerror(rc).decode())
    return b.value


class Problem:
    """One LP loaded on the GPU (lp_load); see include/lp.h for semantics."""

    def __init__(self, lp, **options):
        """options as default_options.  With ptr_kind="device" the arrays of lp
        (row_ptr, col int32; val, c, q, l, u float64) are torch CUDA tensors,
        and set_start / result take and fill torch CUDA tensors."""
        L = library()
        self.m, self.n, self.m1 = int(lp.m), int(lp.n), int(lp.m1)
        self.workspace = options.get("workspace")   # kept alive as long as the handle
        self.opt = default_options(**options)
        self.device = self.opt.ptr_kind == LP_DEVICE
        K, keep = _csr(lp, self.device)
        vecs = [lp.c, lp.q, lp.l, lp.u] if self.device else [_f64(a) for a in (lp.c, lp.q, lp.l, lp.u)]
        c, q, l, u = (_ptr(a, C.c_double) for a in vecs)
        h = C.c_void_p()
        rc = L.lp_load(C.byref(h), C.byref(K), c, q, l, u, self.m1, C.byref(self.opt))
        if rc != 0:
            raise LPError(rc, L.lp_strerror(rc).decode())
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise LPError(rc, library().lp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.lp_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_start(self, x=None, y=None):
        if self.device:
            self._check(library().lp_set_start(self.h, _ptr(x, C.c_double), _ptr(y, C.c_double)))
            return
        xs = None if x is None else _f64(x)
        ys = None if y is None else _f64(y)
        self._check(library().lp_set_start(self.h, _dp(xs), _dp(ys)))

    def set_start_weight(self, omega):
        self._check(library().lp_set_start_weight(self.h, float(omega)))

    def solve(self, tol=1e-4, max_iters=10**7, time_limit=0.0):
        self._check(library().lp_solve(self.h, float(tol), int(max_iters), float(time_limit)))
        return self.info()

    def info(self):
        inf = LPInfo()
        self._check(library().lp_result(self.h, None, None, None, C.byref(inf)))
        d = {k: getattr(inf, k) for k, _ in LPInfo._fields_}
        d["status"] = STATUS[inf.status]
        d["rel_kkt"] = max(inf.rel_primal, inf.rel_dual, inf.rel_gap)
        return d

    def result(self):
        if self.device:
            import torch
            x = torch.empty(self.n, dtype=torch.float64, device="cuda")
            y = torch.empty(self.m, dtype=torch.float64, device="cuda")
            lam = torch.empty(self.n, dtype=torch.float64, device="cuda")
            self._check(library().lp_result(self.h, _ptr(x, C.c_double), _ptr(y, C.c_double),
                                            _ptr(lam, C.c_double), None))
            return x, y, lam, self.info()
        x = np.empty(self.n); y = np.empty(self.m); lam = np.empty(self.n)
        inf = LPInfo()
        self._check(library().lp_result(self.h, _dp(x), _dp(y), _dp(lam), C.byref(inf)))
        return x, y, lam, self.info()

    def get_state(self):
        ln = C.c_int64()
        self._check(library().lp_get_state(self.h, None, C.byref(ln)))
        buf = np.empty(ln.value)
        self._check(library().lp_get_state(self.h, _dp(buf), C.byref(ln)))
        return buf

    def set_state(self, buf):
        buf = _f64(buf)
        self._check(library().lp_set_state(self.h, _dp(buf), buf.size))

    def presolved_size(self):
        """(rows, columns) of the problem on the GPU: the reduced one after presolve."""
        m, n = C.c_int64(), C.c_int64()
        self._check(library().lp_presolved_size(self.h, C.byref(m), C.byref(n)))
        return m.value, n.value

    def scaling(self):
        m, n = self.presolved_size()
        Dr = np.empty(m); Dc = np.empty(n)
        self._check(library().lp_get_scaling(self.h, _dp(Dr), _dp(Dc)))
        return Dr, Dc

    def spmv(self, v, transpose=False):
        v = _f64(v)
        m, n = self.presolved_size()
        out = np.empty(n if transpose else m)
        self._check(library().lp_spmv(self.h, int(bool(transpose)), _dp(v), _dp(out)))
        return out

    def spmv_noalloc(self, d_in, d_out, transpose=False):
        """lp_spmv_noalloc on device buffers (torch float64 tensors or raw
        device addresses); enqueues only, the caller synchronises the stream."""
        pin = d_in if isinstance(d_in, int) else d_in.data_ptr()
        pout = d_out if isinstance(d_out, int) else d_out.data_ptr()
        self._check(library().lp_spmv_noalloc(self.h, int(bool(transpose)), C.c_void_p(pin), C.c_void_p(pout)))

    def kernel_time(self, which):
        cnt = C.c_int64(); ms = C.c_double()
        self._check(library().lp_kernel_time(self.h, int(which), C.byref(cnt), C.byref(ms)))
        return cnt.value, ms.value

    def layout(self):
        a = C.c_int(); b = C.c_int()
        self._check(library().lp_layout(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def layout_blocks(self, which):
        """(slices, most nonzeros, most rows) of one row block of K (0) or K' (1)."""
        s, nb, rb = C.c_int(), C.c_int(), C.c_int()
        self._check(library().lp_layout_blocks(self.h, which, C.byref(s), C.byref(nb), C.byref(rb)))
        return s.value, nb.value, rb.value

    def layout_split(self, which):
        """1 if the partial passes of K (0) or K' (1) sum short rows split by entries, else 0."""
        v = C.c_int()
        self._check(library().lp_layout_split(self.h, which, C.byref(v)))
        return v.value

    def device_bytes(self):
        b = C.c_int64()
        self._check(library().lp_device_bytes(self.h, C.byref(b)))
        return b.value


STATE_VECTORS = [("x", "n"), ("y", "m"), ("Kx", "m"), ("KTy", "n"), ("xbar", "n"), ("ybar", "m"),
                 ("Kxbar", "m"), ("KTybar", "n"), ("x0", "n"), ("y0", "m")]
SCALAR_NAMES = ["eta_hat", "omega", "W", "KKT0", "KKT_prev", "k", "t", "attempts", "restarts",
                "status", "eta_last"]


def unpack_state(buf, n, m):
    d = {name: buf[i] for i, name in enumerate(SCALAR_NAMES)}
    p = NSCALARS
    for name, dim in STATE_VECTORS:
        ln = n if dim == "n" else m
        d[name] = buf[p:p + ln].copy()
        p += ln
    return d


def _info_dict(inf):
    d = {k: getattr(inf, k) for k, _ in LPInfo._fields_}
    d["status"] = STATUS[inf.status]
    d["rel_kkt"] = max(inf.rel_primal, inf.rel_dual, inf.rel_gap)
    return d


class Batch:
    """Many LPs solved together (lp_batch_*); see include/lp.h."""

    def __init__(self, lps, **options):
        L = library()
        self.count = len(lps)
        self.dims = [(int(p.n), int(p.m)) for p in lps]
        self.opt = default_options(**options)
        keep = []
        Ks = (LPCsr * self.count)()
        arr = {k: (C.POINTER(C.c_double) * self.count)() for k in "cqlu"}
        m1 = (C.c_int64 * self.count)()
        for i, p in enumerate(lps):
            rp = np.ascontiguousarray(p.row_ptr, np.int32)
            ci = np.ascontiguousarray(p.col, np.int32)
            v = _f64(p.val)
            keep += [rp, ci, v]
            Ks[i] = LPCsr(int(p.m), int(p.n), int(rp[-1]), rp.ctypes.data_as(C.POINTER(C.c_int32)),
                          ci.ctypes.data_as(C.POINTER(C.c_int32)), _dp(v))
            for k in "cqlu":
                a = _f64(getattr(p, k))
                keep.append(a)
                arr[k][i] = _dp(a)
            m1[i] = int(p.m1)
        h = C.c_void_p()
        rc = L.lp_batch_load(C.byref(h), self.count, Ks, arr["c"], arr["q"], arr["l"], arr["u"], m1,
                             C.byref(self.opt))
        if rc != 0:
            raise LPError(rc, L.lp_strerror(rc).decode())
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise LPError(rc, library().lp_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.lp_batch_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def solve(self, tol=1e-4, max_iters=10**7, time_limit=0.0):
        self._check(library().lp_batch_solve(self.h, float(tol), int(max_iters), float(time_limit)))

    def info(self, i):
        inf = LPInfo()
        self._check(library().lp_batch_result(self.h, int(i), None, None, None, C.byref(inf)))
        return _info_dict(inf)

    def result(self, i):
        n, m = self.dims[i]
        x = np.empty(n); y = np.empty(m); lam = np.empty(n)
        inf = LPInfo()
        self._check(library().lp_batch_result(self.h, int(i), _dp(x), _dp(y), _dp(lam), C.byref(inf)))
        return x, y, lam, _info_dict(inf)

    def get_state(self, i):
        ln = C.c_int64()
        self._check(library().lp_batch_get_state(self.h, int(i), None, C.byref(ln)))
        buf = np.empty(ln.value)
        self._check(library().lp_batch_get_state(self.h, int(i), _dp(buf), C.byref(ln)))
        return buf

    def set_state(self, i, buf):
        buf = _f64(buf)
        self._check(library().lp_batch_set_state(self.h, int(i), _dp(buf), buf.size))

    def layout_blocks(self, which):
        """(most nonzeros, most rows) of one row block of K (0) or K' (1)."""
        nb, rb = C.c_int(), C.c_int()
        self._check(library().lp_batch_layout_blocks(self.h, which, C.byref(nb), C.byref(rb)))
        return nb.value, rb.value

    def device_bytes(self):
        b = C.c_int64()
        self._check(library().lp_batch_device_bytes(self.h, C.byref(b)))
        return b.value

    def loop_form(self):
        """0: batched kernel launches; 1: one workgroup per instance."""
        f = C.c_int()
        self._check(library().lp_batch_loop_form(self.h, C.byref(f)))
        return f.value


class Shared:
    """A batch of one family: instances that share K (lp_shared_*).  `lps`
    are LPData with the same row_ptr / col / val and m1; their c, q, l, u
    are each instance's own."""

    def __init__(self, lps, **options):
        L = library()
        self.h = None
        self.count = len(lps)
        p0 = lps[0]
        self.n, self.m = int(p0.n), int(p0.m)
        self.opt = default_options(**options)
        rp = np.ascontiguousarray(p0.row_ptr, np.int32)
        ci = np.ascontiguousarray(p0.col, np.int32)
        v = _f64(p0.val)
        self._keep = [rp, ci, v]
        K = LPCsr(self.m, self.n, int(rp[-1]), rp.ctypes.data_as(C.POINTER(C.c_int32)),
                  ci.ctypes.data_as(C.POINTER(C.c_int32)), _dp(v))
        arr = {k: (C.POINTER(C.c_double) * self.count)() for k in "cqlu"}
        for i, p in enumerate(lps):
            for k in "cqlu":
                a = _f64(getattr(p, k))
                self._keep.append(a)
                arr[k][i] = _dp(a)
        h = C.c_void_p()
        rc = L.lp_shared_load(C.byref(h), self.count, C.byref(K), arr["c"], arr["q"], arr["l"], arr["u"],
                              int(p0.m1), C.byref(self.opt))
        self._keep = None
        if rc != 0:
            raise LPError(rc, L.lp_strerror(rc).decode())
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise LPError(rc, library().lp_shared_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.lp_shared_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_start(self, i, x=None, y=None, omega=0.0):
        xs = None if x is None else _f64(x)
        ys = None if y is None else _f64(y)
        self._check(library().lp_shared_set_start(self.h, int(i), _dp(xs), _dp(ys), float(omega)))

    def solve(self, tol=1e-4, max_iters=10**7, time_limit=0.0):
        self._check(library().lp_shared_solve(self.h, float(tol), int(max_iters), float(time_limit)))

    def info(self, i):
        inf = LPInfo()
        self._check(library().lp_shared_result(self.h, int(i), None, None, None, C.byref(inf)))
        return _info_dict(inf)

    def result(self, i):
        x = np.empty(self.n); y = np.empty(self.m); lam = np.empty(self.n)
        inf = LPInfo()
        self._check(library().lp_shared_result(self.h, int(i), _dp(x), _dp(y), _dp(lam), C.byref(inf)))
        return x, y, lam, _info_dict(inf)

    def get_state(self, i):
        ln = C.c_int64()
        self._check(library().lp_shared_get_state(self.h, int(i), None, C.byref(ln)))
        buf = np.empty(ln.value)
        self._check(library().lp_shared_get_state(self.h, int(i), _dp(buf), C.byref(ln)))
        return buf

    def set_state(self, i, buf):
        buf = _f64(buf)
        self._check(library().lp_shared_set_state(self.h, int(i), _dp(buf), buf.size))

    def device_bytes(self):
        b = C.c_int64()
        self._check(library().lp_shared_device_bytes(self.h, C.byref(b)))
        return b.value


def gather_probe(idx, x, slices, slice_len, reps=20, stream=None):
    """lp_gather_probe on torch device tensors (idx int32, x float64 or
    float32); returns milliseconds per pass."""
    import torch
    out = torch.empty(4096 * 256, dtype=x.dtype, device=x.device)
    prec = LP_FP64 if x.dtype == torch.float64 else LP_MIXED
    st = stream if stream is not None else torch.cuda.current_stream()
    ms = C.c_double()
    rc = library().lp_gather_probe(C.c_void_p(idx.data_ptr()), C.c_void_p(x.data_ptr()), prec, idx.numel(),
                                   int(slices), int(slice_len), C.c_void_p(out.data_ptr()), int(reps),
                                   C.c_void_p(st.cuda_stream), C.byref(ms))
    if rc != 0:
        raise LPError(rc, "lp_gather_probe")
    return ms.value
