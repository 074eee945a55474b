"""Property tests (hypothesis) of the seeded generators and of the oracle.

Generators: every instance carries a valid primal/dual certificate, its CSR
is well formed, and the same seed gives the same bytes.  Oracle: on randomly
drawn small bounded LPs its optimum at rel KKT 1e-9 equals the minimum over
the vertices (brute force), and weak duality holds at the certificate."""
import numpy as np
from hypothesis import HealthCheck, given, settings, strategies as st

from paper_2312_14832_amd import gen
from lp_helpers import brute_force_vertices

SETTINGS = dict(deadline=None, suppress_health_check=[HealthCheck.too_slow])


@settings(max_examples=40, **SETTINGS)
@given(seed=st.integers(0, 2**32 - 1), m1=st.integers(0, 30), m2=st.integers(0, 30), n=st.integers(1, 60),
       kmax=st.integers(1, 6))
def test_certificate_lp_is_feasible_and_dual_feasible(seed, m1, m2, n, kmax):
    m = m1 + m2
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.integers(0, min(kmax, m) + 1, size=n).astype(np.int64) if m else np.zeros(n, np.int64)
    lp = gen.certificate_lp(rng, m1, m2, counts)
    # well-formed CSR: sorted, distinct columns per row, counts per column as asked
    rp, ci = lp.row_ptr, lp.col
    assert rp[0] == 0 and rp[-1] == counts.sum() and np.all(np.diff(rp) >= 0)
    for i in range(m):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0) and (row.size == 0 or (row[0] >= 0 and row[-1] < n))
    assert np.array_equal(np.bincount(ci, minlength=n), counts)
    K = lp.csr()
    # primal certificate: Ax0 = b, Gx0 - h = s >= 0, l <= x0 <= u
    Kx0 = K @ lp.x0
    assert np.allclose(Kx0[:m1], lp.q[:m1], rtol=1e-12, atol=1e-12)
    assert np.allclose(Kx0[m1:] - lp.q[m1:], lp.s, rtol=1e-12, atol=1e-12) and np.all(lp.s >= 0)
    assert np.all(lp.l <= lp.x0) and np.all(lp.x0 <= lp.u)
    # dual certificate: y0_G >= 0, c - K'y0 = lam0 in Lambda of each variable
    assert np.all(lp.y0[m1:] >= 0)
    lam = lp.c - K.T @ lp.y0
    assert np.allclose(lam, lp.lam0, rtol=1e-12, atol=1e-12)
    lf, uf = np.isfinite(lp.l), np.isfinite(lp.u)
    assert np.all(lp.lam0[~lf & ~uf] == 0) and np.all(lp.lam0[lf & ~uf] >= 0)
    # bound kinds: boxed [0,10], lower-only [0,inf), free
    assert np.all((lp.l == 0) | (lp.l == -np.inf)) and np.all((lp.u == 10) | (lp.u == np.inf))
    assert not np.any(~lf & uf)


@settings(max_examples=10, **SETTINGS)
@given(seed=st.integers(0, 2**31 - 1))
def test_generators_are_reproducible(seed):
    a, b = gen.tiny_lp(seed % 1000), gen.tiny_lp(seed % 1000)
    for f in ("row_ptr", "col", "val", "c", "q", "l", "u"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


@settings(max_examples=25, **SETTINGS)
@given(seed=st.integers(0, 10**6), n=st.integers(2, 5), m1=st.integers(0, 2), m2=st.integers(1, 3))
def test_oracle_matches_vertex_enumeration(oracle_mod, seed, n, m1, m2):
    if m1 >= n:
        m1 = n - 1
    lp = gen.dense_small_lp(seed, n, m1, m2)
    best, _ = brute_force_vertices(lp.csr().toarray(), lp.q, m1, lp.l, lp.u, lp.c)
    o = oracle_mod.Oracle(lp)
    _, _, _, info = o.solve(1e-9, 2_000_000)
    assert info["status"] == "OPTIMAL"
    assert abs(info["pobj"] - best) <= 1e-6 * max(1.0, abs(best))
    # weak duality with the generator's certificate: dobj(y0, lam0) <= opt <= c'x0
    dcert = lp.q @ lp.y0 + np.sum(np.where(lp.lam0 > 0, lp.l * lp.lam0, 0.0)) \
        + np.sum(np.where(lp.lam0 < 0, lp.u * lp.lam0, 0.0))
    assert dcert <= best + 1e-9 * max(1.0, abs(best)) and best <= lp.c @ lp.x0 + 1e-9 * max(1.0, abs(best))
