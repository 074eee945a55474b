"""The library's presolve and postsolve (host code) checked exactly, without
PDHG: the reduced LP is solved by HiGHS, its vertex solution mapped back, and
the result must be an optimal primal-dual pair of the original LP."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2312_14832_amd import gen
from lp_helpers import highs
from presolve_helpers import build_shim, run_postsolve, run_presolve


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    return build_shim(str(tmp_path_factory.mktemp("presolve")))


def optimality(lp, x, y, lam):
    """Primal and dual residuals and the gap of (x, y, lam) on lp, computed
    here from the definitions (A3 of the paper's termination criteria)."""
    K = lp.csr()
    r = K @ x - lp.q
    rp = np.concatenate([r[:lp.m1], np.maximum(-r[lp.m1:], 0.0)])
    lf, uf = np.isfinite(lp.l), np.isfinite(lp.u)
    g = lp.c - K.T @ y
    dual_sign = np.minimum(y[lp.m1:], 0.0)
    cone = np.where(lf & uf, 0.0, np.where(lf, np.minimum(lam, 0), np.where(uf, np.maximum(lam, 0), lam)))
    bviol = np.maximum(lp.l - x, 0) + np.maximum(x - lp.u, 0)
    pobj = lp.c @ x
    dobj = lp.q @ y + np.sum(np.where(lf & (lam > 0), np.where(lf, lp.l, 0) * lam, 0)) \
        + np.sum(np.where(uf & (lam < 0), np.where(uf, lp.u, 0) * lam, 0))
    return (np.linalg.norm(rp), np.linalg.norm(g - lam), np.linalg.norm(dual_sign), np.linalg.norm(cone),
            np.abs(bviol).max(), pobj, dobj)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_postsolve_of_exact_reduced_solution_is_optimal(shim, seed):
    lp = gen.presolve_lp(seed)
    red, row_new, col_new = run_presolve(shim, lp)
    # at least the planted reductions: 13 singleton rows, 2 empty rows;
    # 5 fixed, 5 fixed by singleton equalities, 3 empty columns
    assert lp.m - red.m >= 15 and lp.n - red.n >= 13
    assert red.m1 <= lp.m1 - 6 and np.all(red.l <= red.u)
    opt, xr, yr = highs(red)
    x, y, lam, info = run_postsolve(shim, lp, xr, yr)
    ref, _, _ = highs(lp)
    rp, rd, ysign, cone, bviol, pobj, dobj = optimality(lp, x, y, lam)
    scale = 1 + np.abs(lp.q).max() + np.abs(lp.c).max()
    assert rp <= 1e-8 * scale and rd <= 1e-8 * scale and ysign == 0 and cone == 0 and bviol <= 1e-12
    assert pobj == pytest.approx(ref, rel=1e-9) and dobj == pytest.approx(ref, rel=1e-9)
    # the postsolve's own report agrees with the definitions
    assert info["pobj"] == pytest.approx(pobj, rel=1e-12) and info["dobj"] == pytest.approx(dobj, rel=1e-12)
    assert max(info["rel_p"], info["rel_d"], info["rel_g"]) <= 1e-9
    # kept entries come straight from the reduced solution
    kc, kr = col_new >= 0, row_new >= 0
    assert np.array_equal(x[kc], xr[col_new[kc]]) and np.array_equal(y[kr], yr[row_new[kr]])


def test_nothing_to_reduce(shim):
    """A dense LP (every row and column full, no fixed bounds) has no
    reduction; tiny_lp(0) has one singleton inequality row (row 405), which
    becomes a bound, and loses exactly that row."""
    rng = np.random.default_rng(3)
    K = sp.csr_matrix(rng.uniform(0.5, 1.5, (6, 9)))
    lp = gen.LPData(m=6, n=9, m1=2, row_ptr=K.indptr.astype(np.int32), col=K.indices.astype(np.int32),
                    val=K.data, c=rng.standard_normal(9), q=np.ones(6), l=np.zeros(9), u=np.full(9, 10.0))
    assert run_presolve(shim, lp) is None
    t = gen.tiny_lp(0)
    red, row_new, col_new = run_presolve(shim, t)
    single = np.flatnonzero(np.diff(t.row_ptr) == 1)
    assert list(single) == [405] and (red.m, red.n) == (t.m - 1, t.n) and row_new[405] == -1


def test_reductions_that_prove_infeasibility_are_left_alone(shim):
    """A singleton equality outside its variable's box and an empty equality
    row with a nonzero right-hand side stay in the reduced problem."""
    Kd = np.array([[2.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    K = sp.csr_matrix(Kd)
    K.eliminate_zeros()
    lp = gen.LPData(m=3, n=3, m1=2, row_ptr=K.indptr.astype(np.int32), col=K.indices.astype(np.int32),
                    val=K.data, c=np.ones(3), q=np.array([50.0, 1.0, 0.0]), l=np.zeros(3), u=np.full(3, 10.0))
    out = run_presolve(shim, lp)
    assert out is None


# ------------------------------------------------------------ random instances

from hypothesis import HealthCheck, assume, given, settings, strategies as st  # noqa: E402


def _planted(seed, m1, m2, n, kmax, nfix, nsing):
    """A small certificate LP (feasible and bounded by construction) with
    planted reductions: some boxed variables fixed at the certificate point,
    singleton equality rows through it and singleton inequality rows it
    satisfies; the column counts 0..kmax leave empty columns and rows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = m1 + m2
    counts = rng.integers(0, min(kmax, m) + 1, size=n).astype(np.int64) if m else np.zeros(n, np.int64)
    base = gen.certificate_lp(rng, m1, m2, counts)
    l, u, x0 = base.l.copy(), base.u.copy(), base.x0
    boxed = np.flatnonzero(np.isfinite(l) & np.isfinite(u))
    for j in rng.choice(boxed, min(nfix, boxed.size), replace=False):
        l[j] = u[j] = x0[j]
    K = base.csr()

    def single(j, a):
        return sp.csr_matrix(([a], ([0], [j])), shape=(1, n))

    eq_rows, eq_q, ge_rows, ge_q = [], [], [], []
    for _ in range(nsing):
        j = int(rng.integers(n))
        a = float(rng.uniform(0.5, 2.0) * rng.choice([-1.0, 1.0]))
        if rng.random() < 0.5:
            eq_rows.append(single(j, a)); eq_q.append(a * x0[j])
        else:
            ge_rows.append(single(j, a)); ge_q.append(a * x0[j] - float(rng.uniform(0.0, 1.0)))
    A = sp.vstack([K[:m1]] + eq_rows) if (m1 or eq_rows) else sp.csr_matrix((0, n))
    G = sp.vstack([K[m1:]] + ge_rows) if (m2 or ge_rows) else sp.csr_matrix((0, n))
    q = np.concatenate([base.q[:m1], eq_q, base.q[m1:], ge_q])
    M = sp.vstack([A, G]).tocsr()
    M.sort_indices()
    return gen.LPData(m=M.shape[0], n=n, m1=A.shape[0], row_ptr=M.indptr.astype(np.int32),
                      col=M.indices.astype(np.int32), val=M.data.astype(float), c=base.c, q=q, l=l, u=u)


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.too_slow,
                                                                  HealthCheck.function_scoped_fixture])
@given(seed=st.integers(0, 2**32 - 1), m1=st.integers(0, 10), m2=st.integers(0, 10), n=st.integers(1, 20),
       kmax=st.integers(0, 4), nfix=st.integers(0, 3), nsing=st.integers(0, 5))
def test_presolve_postsolve_random(shim, seed, m1, m2, n, kmax, nfix, nsing):
    """On random LPs with planted reductions: the reduced LP's HiGHS optimum,
    mapped back, is an optimal primal-dual pair of the original with
    HiGHS's objective."""
    lp = _planted(seed, m1, m2, n, kmax, nfix, nsing)
    from lp_helpers import highs_status
    assume(highs_status(lp) == 0)
    out = run_presolve(shim, lp)
    assume(out is not None)
    red = out[0]
    assert highs_status(red) == 0
    _, xr, yr = highs(red)
    x, y, lam, info = run_postsolve(shim, lp, xr, yr)
    ref, _, _ = highs(lp)
    rp, rd, ysign, cone, bviol, pobj, dobj = optimality(lp, x, y, lam)
    scale = 1 + np.abs(lp.q).max(initial=0) + np.abs(lp.c).max() + np.abs(x).max()
    assert rp <= 1e-7 * scale and rd <= 1e-7 * scale and ysign == 0 and cone == 0 and bviol <= 1e-9 * scale
    assert abs(pobj - ref) <= 1e-7 * (1 + abs(ref)) and abs(dobj - ref) <= 1e-7 * (1 + abs(ref))


def test_everything_removable_keeps_the_original(shim):
    """Only singleton rows: once they are gone every column is empty and
    would be fixed at its best bound, so nothing would remain to solve;
    the presolve then declines and the original LP is loaded as it is."""
    Kd = np.array([[2.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, 3.0]])
    K = sp.csr_matrix(Kd)
    # 2 x0 = 4 (fixes x0 = 2), -x1 >= -5 (x1 <= 5), 3 x2 >= 3 (x2 >= 1)
    lp = gen.LPData(m=3, n=3, m1=1, row_ptr=K.indptr.astype(np.int32), col=K.indices.astype(np.int32),
                    val=K.data, c=np.array([1.0, -1.0, 2.0]), q=np.array([4.0, -5.0, 3.0]),
                    l=np.array([0.0, 0.0, 0.0]), u=np.array([10.0, np.inf, np.inf]))
    assert run_presolve(shim, lp) is None
