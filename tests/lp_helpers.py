"""Helpers shared by the tests: independent solvers and hand-derivable checks.

Nothing here calls the oracle or the GPU library."""
from __future__ import annotations

import itertools
import json
import os

import numpy as np
import scipy.optimize as so

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def fnum(v):
    if isinstance(v, str):
        return float(v)
    return float(v)


def highs(lp):
    """Solve with scipy's HiGHS: returns (objective, x, y) with y = duals of K rows
    in the paper's sign convention (y_G >= 0 for Gx >= h)."""
    K = lp.csr()
    m1 = lp.m1
    bounds = [(None if np.isinf(a) else a, None if np.isinf(b) else b) for a, b in zip(lp.l, lp.u)]
    kw = {}
    if m1 > 0:
        kw["A_eq"] = K[:m1]
        kw["b_eq"] = lp.q[:m1]
    if lp.m - m1 > 0:
        kw["A_ub"] = -K[m1:]
        kw["b_ub"] = -lp.q[m1:]
    res = so.linprog(lp.c, bounds=bounds, method="highs", **kw)
    assert res.status == 0, res.message
    y = np.zeros(lp.m)
    if m1 > 0:
        y[:m1] = res.eqlin.marginals
    if lp.m - m1 > 0:
        y[m1:] = -res.ineqlin.marginals
    return res.fun, res.x, y


def highs_status(lp):
    """scipy linprog (HiGHS) status of the LP: 0 optimal, 2 infeasible, 3 unbounded."""
    K = lp.csr()
    m1 = lp.m1
    bounds = [(None if np.isinf(a) else a, None if np.isinf(b) else b) for a, b in zip(lp.l, lp.u)]
    kw = {}
    if m1 > 0:
        kw["A_eq"], kw["b_eq"] = K[:m1], lp.q[:m1]
    if lp.m - m1 > 0:
        kw["A_ub"], kw["b_ub"] = -K[m1:], -lp.q[m1:]
    return so.linprog(lp.c, bounds=bounds, method="highs", **kw).status


def farkas_ratios(lp, x_ray, y_ray):
    """The two Farkas certificates of an LP without a solution, computed from
    the unscaled data.  Dual ray w: objective q'w + sum(l lam+ - u lam-) with
    lam = proj_Lambda(-K'w), residual |(-K'w - lam, min(w_G, 0))|.  Primal ray
    d: objective c'd, residual |(A d, max(-G d, 0), recession-cone violation)|.
    Returns (dual_obj, dual_res, primal_obj, primal_res)."""
    K = lp.csr()
    m1 = lp.m1
    lf, uf = np.isfinite(lp.l), np.isfinite(lp.u)
    w, d = y_ray, x_ray
    g = -(K.T @ w)
    lam = np.where(lf & uf, g, np.where(lf, np.maximum(g, 0), np.where(uf, np.minimum(g, 0), 0.0)))
    lo, hi = np.where(lf, lp.l, 0.0), np.where(uf, lp.u, 0.0)
    dobj = lp.q @ w + np.sum(np.where(lf & (lam > 0), lo * lam, 0.0)) \
        + np.sum(np.where(uf & (lam < 0), hi * lam, 0.0))
    dres = np.linalg.norm(np.concatenate([g - lam, np.minimum(w[m1:], 0.0)]))
    Kd = K @ d
    cone = np.where(lf, np.minimum(d, 0.0), 0.0) + np.where(uf, np.maximum(d, 0.0), 0.0)
    pres = np.linalg.norm(np.concatenate([Kd[:m1], np.maximum(-Kd[m1:], 0.0), cone]))
    return dobj, dres, lp.c @ d, pres


def brute_force_vertices(Kd, q, m1, l, u, c):
    """Minimum of c'x over the vertices of {Ax=b, Gx>=h, l<=x<=u} (all bounds finite).

    Every vertex makes n linearly independent constraints active, and the
    equalities are always active: try every choice of n - m1 more from the G
    rows and the 2n bounds, solve, keep the feasible points."""
    Kd = np.asarray(Kd, float)
    m, n = Kd.shape
    rows = [(Kd[i], q[i]) for i in range(m1, m)]
    for j in range(n):
        e = np.zeros(n); e[j] = 1.0
        rows.append((e, l[j]))
        rows.append((e, u[j]))
    best = np.inf
    best_x = None
    for pick in itertools.combinations(range(len(rows)), n - m1):
        M = np.vstack([Kd[:m1]] + [rows[p][0][None, :] for p in pick]) if m1 else \
            np.vstack([rows[p][0][None, :] for p in pick])
        rhs = np.concatenate([q[:m1], [rows[p][1] for p in pick]])
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, rhs)
        ok = np.all(x >= l - 1e-9) and np.all(x <= u + 1e-9)
        ok = ok and np.allclose(Kd[:m1] @ x, q[:m1], atol=1e-9)
        ok = ok and np.all(Kd[m1:] @ x >= q[m1:] - 1e-9)
        if ok:
            v = float(c @ x)
            if v < best:
                best, best_x = v, x
    return best, best_x


def objective_band(eps, data, x_ref, y_ref, pobj, dobj):
    """How far the objectives of two points that both meet the termination
    criteria at eps can be apart, to first order.  With primal residual r_p
    and dual residual r_d, convexity of the LP value function in q and c
    gives opt - |y*||r_p| <= c'x <= opt + |x*||r_d| + |gap|; the criteria bound
    |r_p| <= eps(1+|q|), |r_d| <= eps(1+|c|), |gap| <= eps(1+|p|+|d|).  The
    band is twice that sum, with (x*, y*) taken from a reference point."""
    per = (eps * (1 + abs(pobj) + abs(dobj))
           + np.linalg.norm(y_ref) * eps * (1 + np.linalg.norm(data.q))
           + np.linalg.norm(x_ref) * eps * (1 + np.linalg.norm(data.c)))
    return 2.0 * per


def restart_golden_lp(g):
    """The LP of restart_candidate_1var.json (no rows)."""
    from paper_2312_14832_amd import gen
    n = int(g["n"])
    return gen.from_dense(np.zeros((0, n)), g["c"], g["q"], [fnum(a) for a in g["l"]],
                          [fnum(a) for a in g["u"]], g["m1"])


RESTART_SCALARS = ["eta_hat", "omega", "W", "KKT0", "KKT_prev", "k", "t", "attempts", "restarts",
                   "status", "eta_last"]


def restart_golden_state(g, case):
    """Flat solver state (16 scalars, then x, K'y, xbar, K'ybar, x0 for one
    column and no rows) of one case of restart_candidate_1var.json."""
    st = g["start"]
    sc = dict(eta_hat=g["eta"], omega=g["omega"], W=case["W"], KKT0=case["KKT0"],
              KKT_prev=fnum(st["KKT_prev"]), k=st["k"], t=st["t"], attempts=st["attempts"],
              restarts=st["restarts"], status=0, eta_last=g["eta"])
    buf = np.zeros(16 + 5)
    for i, name in enumerate(RESTART_SCALARS):
        buf[i] = sc[name]
    buf[16:] = [case["x"], 0.0, case["xbar"], 0.0, st["x0"]]
    return buf


def check_restart_golden_state(st, want, label):
    """Compare an unpacked state with one 'after' entry of the golden."""
    for key in ("x", "xbar", "x0"):
        assert st[key][0] == pytest_approx(fnum(want[key])), (label, key, st[key][0], want[key])
    for key in ("W", "KKT0", "KKT_prev", "omega"):
        w = fnum(want[key])
        assert (st[key] == w) if np.isinf(w) else st[key] == pytest_approx(w), (label, key, st[key], w)
    for key in ("t", "k", "restarts"):
        assert int(st[key]) == int(want[key]), (label, key, st[key], want[key])


def pytest_approx(v):
    import pytest
    return pytest.approx(v, rel=1e-15, abs=1e-300)
