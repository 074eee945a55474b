// Host-side presolve and postsolve (see presolve.h).
#include "presolve.h"

#include <algorithm>
#include <cmath>

namespace pdlp {

namespace {

// slack accepted when a reduction checks a right-hand side or a bound
double slack(double a) { return 1e-9 * (1.0 + std::fabs(a)); }

// column view (CSC) of a CSR
void to_columns(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci, const double *v, std::vector<int64_t> &cp,
                std::vector<int> &cr, std::vector<double> &cv)
{
    const int64_t nnz = rp[m];
    cp.assign((size_t)n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) ++cp[(size_t)ci[p] + 1];
    for (int64_t j = 0; j < n; ++j) cp[(size_t)j + 1] += cp[(size_t)j];
    cr.resize((size_t)std::max<int64_t>(nnz, 1));
    cv.resize((size_t)std::max<int64_t>(nnz, 1));
    std::vector<int64_t> at(cp.begin(), cp.end() - 1);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t k = at[(size_t)ci[p]]++;
            cr[(size_t)k] = (int)i;
            cv[(size_t)k] = v ? v[p] : 0.0;
        }
}

double proj_cone(double g, bool lf, bool uf)
{
    if (lf && uf) return g;
    if (lf) return g > 0.0 ? g : 0.0;
    if (uf) return g < 0.0 ? g : 0.0;
    return 0.0;
}

}  // namespace

bool presolve(const lp_csr *K, const double *c, const double *q, const double *l, const double *u, int64_t m1,
              Presolved &R)
{
    const int64_t m = K->m, n = K->n, nnz = K->nnz;
    R = Presolved{};
    R.m0 = m; R.n0 = n; R.m10 = m1;
    R.rp0.assign(K->row_ptr, K->row_ptr + m + 1);
    R.ci0.assign(K->col, K->col + nnz);
    R.v0.assign((size_t)nnz, 0.0);
    if (K->val) std::copy(K->val, K->val + nnz, R.v0.begin());
    R.c0.assign(c, c + n);
    R.q0.assign(q, q + m);
    R.l0.assign(l, l + n);
    R.u0.assign(u, u + n);
    const int32_t *rp = R.rp0.data(), *ci = R.ci0.data();
    const double *v = R.v0.data();
    std::vector<int64_t> cp;
    std::vector<int> cr;
    std::vector<double> cv;
    to_columns(m, n, rp, ci, v, cp, cr, cv);

    std::vector<char> row_on((size_t)m, 1), col_on((size_t)n, 1);
    std::vector<int> rlen((size_t)m), clen((size_t)n);
    for (int64_t i = 0; i < m; ++i) rlen[(size_t)i] = rp[i + 1] - rp[i];
    for (int64_t j = 0; j < n; ++j) clen[(size_t)j] = (int)(cp[(size_t)j + 1] - cp[(size_t)j]);
    std::vector<double> qw(R.q0), lw(R.l0), uw(R.u0);
    R.xfix.assign((size_t)n, 0.0);

    auto drop_row = [&](int64_t i) {
        row_on[(size_t)i] = 0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (col_on[(size_t)ci[p]]) --clen[(size_t)ci[p]];
    };
    auto fix_col = [&](int64_t j, double val, PresolveOp::Kind kind) {
        col_on[(size_t)j] = 0;
        R.xfix[(size_t)j] = val;
        R.offset += c[j] * val;
        for (int64_t p = cp[(size_t)j]; p < cp[(size_t)j + 1]; ++p) {
            const int i = cr[(size_t)p];
            if (row_on[(size_t)i]) {
                qw[(size_t)i] -= cv[(size_t)p] * val;
                --rlen[(size_t)i];
            }
        }
        R.ops.push_back({kind, -1, (int)j, 0.0, 0});
    };

    bool changed = true;
    while (changed) {
        changed = false;
        for (int64_t j = 0; j < n; ++j) {
            if (!col_on[(size_t)j]) continue;
            if (lw[(size_t)j] == uw[(size_t)j]) {
                fix_col(j, lw[(size_t)j], PresolveOp::FIX_COL);
                changed = true;
            } else if (clen[(size_t)j] == 0) {
                // the column meets no remaining row: its best value is a bound
                double val;
                if (c[j] > 0.0) {
                    if (!std::isfinite(lw[(size_t)j])) continue;   // unbounded: left to the solver
                    val = lw[(size_t)j];
                } else if (c[j] < 0.0) {
                    if (!std::isfinite(uw[(size_t)j])) continue;
                    val = uw[(size_t)j];
                } else {
                    val = std::min(std::max(0.0, lw[(size_t)j]), uw[(size_t)j]);
                }
                fix_col(j, val, PresolveOp::EMPTY_COL);
                changed = true;
            }
        }
        for (int64_t i = 0; i < m; ++i) {
            if (!row_on[(size_t)i]) continue;
            const bool eq = i < m1;
            if (rlen[(size_t)i] == 0) {
                const double r = qw[(size_t)i], tol = slack(R.q0[(size_t)i]);
                if (eq ? std::fabs(r) > tol : r > tol) continue;   // infeasible: left to the solver
                drop_row(i);
                R.ops.push_back({PresolveOp::EMPTY_ROW, (int)i, -1, 0.0, 0});
                changed = true;
            } else if (rlen[(size_t)i] == 1) {
                int64_t j = -1;
                double a = 0.0;
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                    if (col_on[(size_t)ci[p]]) {
                        j = ci[p];
                        a = v[p];
                    }
                if (j < 0 || a == 0.0) continue;
                const double b = qw[(size_t)i] / a, lo = lw[(size_t)j], hi = uw[(size_t)j];
                if (eq) {
                    // a x_j = q_i fixes x_j
                    if (b < lo - slack(lo) || b > hi + slack(hi)) continue;   // infeasible: left to the solver
                    drop_row(i);
                    R.ops.push_back({PresolveOp::SING_EQ, (int)i, (int)j, a, 0});
                    lw[(size_t)j] = uw[(size_t)j] = std::min(std::max(b, lo), hi);
                } else {
                    // a x_j >= q_i is a bound on x_j
                    int t = 0;
                    if (a > 0.0 && b > lo) t = 1;
                    if (a < 0.0 && b < hi) t = -1;
                    if ((t == 1 && b > hi + slack(hi)) || (t == -1 && b < lo - slack(lo))) continue;
                    drop_row(i);
                    R.ops.push_back({PresolveOp::SING_INEQ, (int)i, (int)j, a, t});
                    if (t == 1) lw[(size_t)j] = std::min(b, hi);
                    if (t == -1) uw[(size_t)j] = std::max(b, lo);
                }
                changed = true;
            }
        }
    }

    // the reduced problem: kept rows (equalities still first) and columns
    R.row_new.assign((size_t)m, -1);
    R.col_new.assign((size_t)n, -1);
    for (int64_t j = 0; j < n; ++j)
        if (col_on[(size_t)j]) R.col_new[(size_t)j] = (int)R.n++;
    if (R.n == 0 || R.ops.empty()) {
        R = Presolved{};
        return false;
    }
    for (int64_t i = 0; i < m; ++i)
        if (row_on[(size_t)i]) {
            R.row_new[(size_t)i] = (int)R.m++;
            if (i < m1) ++R.m1;
        }
    R.rp.assign(1, 0);
    for (int64_t i = 0; i < m; ++i) {
        if (!row_on[(size_t)i]) continue;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (col_on[(size_t)ci[p]]) {
                R.ci.push_back(R.col_new[(size_t)ci[p]]);
                R.v.push_back(v[p]);
            }
        R.rp.push_back((int32_t)R.ci.size());
        R.q.push_back(qw[(size_t)i]);
    }
    for (int64_t j = 0; j < n; ++j)
        if (col_on[(size_t)j]) {
            R.c.push_back(c[j]);
            R.l.push_back(lw[(size_t)j]);
            R.u.push_back(uw[(size_t)j]);
        }
    R.K.m = R.m;
    R.K.n = R.n;
    R.K.nnz = (int64_t)R.ci.size();
    R.K.row_ptr = R.rp.data();
    R.K.col = R.ci.data();
    R.K.val = R.v.data();
    return true;
}

void postsolve(const Presolved &R, const double *xr, const double *yr, double *x, double *y, double *lam,
               double &pobj, double &dobj, double &rel_p, double &rel_d, double &rel_g)
{
    const int64_t m = R.m0, n = R.n0;
    const int32_t *rp = R.rp0.data(), *ci = R.ci0.data();
    const double *v = R.v0.data();
    std::vector<double> X((size_t)n), Y((size_t)m, 0.0);
    for (int64_t j = 0; j < n; ++j) {
        const int k = R.col_new[(size_t)j];
        X[(size_t)j] = k >= 0 ? xr[k] : R.xfix[(size_t)j];
    }
    for (int64_t i = 0; i < m; ++i) {
        const int k = R.row_new[(size_t)i];
        if (k >= 0) Y[(size_t)i] = yr[k];
    }
    std::vector<int64_t> cp;
    std::vector<int> cr;
    std::vector<double> cv;
    to_columns(m, n, rp, ci, v, cp, cr, cv);
    auto reduced_cost = [&](int j) {
        double r = R.c0[(size_t)j];
        for (int64_t p = cp[(size_t)j]; p < cp[(size_t)j + 1]; ++p) r -= cv[(size_t)p] * Y[(size_t)cr[(size_t)p]];
        return r;
    };
    // Duals of removed rows, last reduction first.  A singleton inequality
    // that tightened a bound takes over that bound's multiplier when it has
    // the bound's sign (y_i = r_j / a >= 0); a singleton equality takes the
    // whole reduced cost (y_i = r_j / a, lam_j = 0 is in every cone); empty
    // and redundant rows get 0.
    for (auto it = R.ops.rbegin(); it != R.ops.rend(); ++it) {
        const PresolveOp &op = *it;
        if (op.kind == PresolveOp::SING_EQ) {
            Y[(size_t)op.row] = reduced_cost(op.col) / op.a;
        } else if (op.kind == PresolveOp::SING_INEQ) {
            const double r = reduced_cost(op.col);
            if ((op.tightened == 1 && r > 0.0) || (op.tightened == -1 && r < 0.0)) Y[(size_t)op.row] = r / op.a;
        }
    }
    // the termination quantities on the original problem (the paper's three
    // relative criteria, 2-norms)
    std::vector<double> Kx((size_t)m, 0.0), KTy((size_t)n, 0.0);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) Kx[(size_t)i] += v[p] * X[(size_t)ci[p]];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) KTy[(size_t)ci[p]] += v[p] * Y[(size_t)i];
    double rp2 = 0.0, qy = 0.0, nq = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double r = Kx[(size_t)i] - R.q0[(size_t)i];
        if (i >= R.m10) r = -r > 0.0 ? -r : 0.0;
        rp2 += r * r;
        qy += R.q0[(size_t)i] * Y[(size_t)i];
        nq += R.q0[(size_t)i] * R.q0[(size_t)i];
    }
    double rd2 = 0.0, cx = 0.0, bnd = 0.0, nc = 0.0;
    std::vector<double> L((size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        const bool lf = std::isfinite(R.l0[(size_t)j]), uf = std::isfinite(R.u0[(size_t)j]);
        const double g = R.c0[(size_t)j] - KTy[(size_t)j];
        const double lm = proj_cone(g, lf, uf);
        L[(size_t)j] = lm;
        rd2 += (g - lm) * (g - lm);
        cx += R.c0[(size_t)j] * X[(size_t)j];
        if (lf && lm > 0.0) bnd += R.l0[(size_t)j] * lm;
        if (uf && lm < 0.0) bnd += R.u0[(size_t)j] * lm;
        nc += R.c0[(size_t)j] * R.c0[(size_t)j];
    }
    pobj = cx;
    dobj = qy + bnd;
    rel_p = std::sqrt(rp2) / (1.0 + std::sqrt(nq));
    rel_d = std::sqrt(rd2) / (1.0 + std::sqrt(nc));
    rel_g = std::fabs(dobj - pobj) / (1.0 + std::fabs(dobj) + std::fabs(pobj));
    if (x) std::copy(X.begin(), X.end(), x);
    if (y) std::copy(Y.begin(), Y.end(), y);
    if (lam) std::copy(L.begin(), L.end(), lam);
}

}  // namespace pdlp
