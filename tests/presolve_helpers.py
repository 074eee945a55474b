"""The library's host presolve and postsolve behind a small C shim
(tests/presolve_shim.cpp, built with g++; host code only, no GPU), for the
tests that need the reduced LP or the mapping back."""
import ctypes as C
import os
import subprocess

import numpy as np

from paper_2312_14832_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def build_shim(outdir):
    out = os.path.join(outdir, "libpresolve_shim.so")
    csrc = os.path.join(ROOT, "paper_2312_14832_amd", "csrc")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(csrc, "presolve.cpp"), os.path.join(ROOT, "tests", "presolve_shim.cpp"), "-o", out],
                   check=True)
    L = C.CDLL(out)
    L.ps_presolve.restype = C.c_int
    return L


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def run_presolve(L, lp):
    rp, ci = np.ascontiguousarray(lp.row_ptr, np.int32), np.ascontiguousarray(lp.col, np.int32)
    v, c, q, l, u = (np.ascontiguousarray(a, np.float64) for a in (lp.val, lp.c, lp.q, lp.l, lp.u))
    dims = np.zeros(4, np.int64)
    ok = L.ps_presolve(C.c_int64(lp.m), C.c_int64(lp.n), C.c_int64(lp.nnz), _p(rp, C.c_int32), _p(ci, C.c_int32),
                       _p(v), _p(c), _p(q), _p(l), _p(u), C.c_int64(lp.m1), _p(dims, C.c_int64))
    if not ok:
        return None
    m, n, m1, nnz = (int(t) for t in dims)
    R = dict(rp=np.zeros(m + 1, np.int32), ci=np.zeros(max(nnz, 1), np.int32), v=np.zeros(max(nnz, 1)),
             c=np.zeros(n), q=np.zeros(m), l=np.zeros(n), u=np.zeros(n), row_new=np.zeros(lp.m, np.int32),
             col_new=np.zeros(lp.n, np.int32))
    L.ps_reduced(*(_p(R[k], C.c_int32 if R[k].dtype == np.int32 else C.c_double)
                   for k in ("rp", "ci", "v", "c", "q", "l", "u", "row_new", "col_new")))
    red = gen.LPData(m=m, n=n, m1=m1, row_ptr=R["rp"], col=R["ci"][:nnz], val=R["v"][:nnz], c=R["c"], q=R["q"],
                     l=R["l"], u=R["u"])
    return red, R["row_new"], R["col_new"]


def run_postsolve(L, lp, xr, yr):
    x, y, lam, out = np.zeros(lp.n), np.zeros(lp.m), np.zeros(lp.n), np.zeros(5)
    L.ps_postsolve(_p(np.ascontiguousarray(xr)), _p(np.ascontiguousarray(yr)), _p(x), _p(y), _p(lam), _p(out))
    return x, y, lam, dict(zip(("pobj", "dobj", "rel_p", "rel_d", "rel_g"), out))
