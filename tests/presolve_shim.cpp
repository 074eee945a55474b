// Test shim: the library's presolve and postsolve (host code, no GPU) behind
// a C interface for ctypes.  Built by tests/test_presolve_cpu.py.
#include <algorithm>
#include <cstdint>

#include "presolve.h"

static pdlp::Presolved g;

extern "C" int ps_presolve(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                           const double *c, const double *q, const double *l, const double *u, int64_t m1,
                           int64_t *dims)
{
    lp_csr K{m, n, nnz, rp, ci, v};
    const bool ok = pdlp::presolve(&K, c, q, l, u, m1, g);
    dims[0] = g.m; dims[1] = g.n; dims[2] = g.m1; dims[3] = g.K.nnz;
    return ok ? 1 : 0;
}

extern "C" void ps_reduced(int32_t *rp, int32_t *ci, double *v, double *c, double *q, double *l, double *u,
                           int32_t *row_new, int32_t *col_new)
{
    std::copy(g.rp.begin(), g.rp.end(), rp);
    std::copy(g.ci.begin(), g.ci.end(), ci);
    std::copy(g.v.begin(), g.v.end(), v);
    std::copy(g.c.begin(), g.c.end(), c);
    std::copy(g.q.begin(), g.q.end(), q);
    std::copy(g.l.begin(), g.l.end(), l);
    std::copy(g.u.begin(), g.u.end(), u);
    std::copy(g.row_new.begin(), g.row_new.end(), row_new);
    std::copy(g.col_new.begin(), g.col_new.end(), col_new);
}

extern "C" void ps_postsolve(const double *xr, const double *yr, double *x, double *y, double *lam, double *out5)
{
    pdlp::postsolve(g, xr, yr, x, y, lam, out5[0], out5[1], out5[2], out5[3], out5[4]);
}
