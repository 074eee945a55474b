// Simple host-side presolve of an LP in the library's form (K = [A; G] in
// CSR, equality rows first; l <= x <= u) and the matching postsolve.
//
// The paper runs its solver after third-party presolvers (COPT's, CLP's) and
// reports them as a large speed-up on MIPLIB relaxations (Table 1).  Those are
// not available here; this is a native stand-in with the classic reductions
// that need no factorisation: fixed columns, empty columns, empty rows and
// singleton rows (an equality fixes its variable, an inequality tightens a
// bound).  A reduction that would itself prove the LP infeasible or
// unbounded is not made: the solver's ray test reports those.
#pragma once

#include <cstdint>
#include <vector>

#include "lp.h"

namespace pdlp {

struct PresolveOp {
    enum Kind : int { FIX_COL, EMPTY_COL, EMPTY_ROW, SING_EQ, SING_INEQ } kind;
    int row, col;
    double a;        // the singleton's coefficient
    int tightened;   // SING_INEQ: +1 it raised l_col, -1 it lowered u_col, 0 it was redundant
};

struct Presolved {
    // the original problem (host copies)
    int64_t m0 = 0, n0 = 0, m10 = 0;
    std::vector<int32_t> rp0, ci0;
    std::vector<double> v0, c0, q0, l0, u0;
    // the reduced problem
    int64_t m = 0, n = 0, m1 = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v, c, q, l, u;
    lp_csr K{};
    std::vector<int> row_new, col_new;   // original index -> reduced index, or -1 if removed
    std::vector<double> xfix;            // value of each removed column (original index)
    std::vector<PresolveOp> ops;         // reductions in the order they were made
    double offset = 0.0;                 // c'x of the removed columns
};

// Reduce (K, c, q, l, u, m1).  Returns false (and leaves R empty) when no
// reduction applies or every column would go; the caller then loads the
// original problem.
bool presolve(const lp_csr *K, const double *c, const double *q, const double *l, const double *u, int64_t m1,
              Presolved &R);

// Map a point of the reduced problem (xr[n], yr[m]) back to the original:
// x[n0], y[m0], lam[n0] = proj_Lambda(c - K'y), and the termination
// quantities of that point on the original problem.
void postsolve(const Presolved &R, const double *xr, const double *yr, double *x, double *y, double *lam,
               double &pobj, double &dobj, double &rel_p, double &rel_d, double &rel_g);

}  // namespace pdlp
