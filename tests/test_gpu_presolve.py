"""The presolved solve path on the GPU: the LP is reduced on the host, the
reduced LP solved by the HIP path, and the point mapped back; checked on
the original LP by the FP64 oracle's evaluation and against HiGHS."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from lp_helpers import highs
from gpu_helpers import objective_spread, say
from presolve_helpers import build_shim, run_postsolve, run_presolve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    return build_shim(str(tmp_path_factory.mktemp("presolve")))


@pytest.mark.parametrize("seed", [0, 1])
def test_presolved_solve_meets_criteria_on_original(lpmod, oracle_mod, shim, seed):
    """The mapped-back point meets the three relative criteria of the
    original LP near the tolerance, the reported quantities are the
    oracle's evaluation of that point, and the objective is held to the
    measured bar of the oracle solving the same reduced LP: its solution,
    mapped back by the same postsolve, gives the reference objective, and 24
    runs perturbed by 1e-15 give the spread (the postsolve adds a constant
    to the objective, so the spread carries over)."""
    say(f"case presolve seed={seed}")
    lp = gen.presolve_lp(seed)
    p = lpmod.Problem(lp, presolve=1)
    mr, nr = p.presolved_size()
    assert mr <= lp.m - 15 and nr <= lp.n - 13
    info = p.solve(1e-6, 400_000)
    assert info["status"] == "OPTIMAL"
    x, y, lam, _ = p.result()
    o = oracle_mod.Oracle(lp)
    ev = o.eval_unscaled(x, y)
    say(f"  reduced {mr}x{nr} of {lp.m}x{lp.n}: {info['iterations']} it, rel_kkt on original {ev['rel_kkt']:.2e}")
    assert ev["rel_kkt"] <= 1e-5
    for k in ("rel_primal", "rel_dual", "rel_gap"):
        kk = {"rel_primal": "rel_p", "rel_dual": "rel_d", "rel_gap": "rel_g"}[k]
        assert info[k] == pytest.approx(ev[kk], rel=1e-9, abs=1e-15)
    assert info["pobj"] == pytest.approx(ev["pobj"], rel=1e-12)
    red, _, _ = run_presolve(shim, lp)
    assert (red.m, red.n) == (mr, nr)
    io, dev, bar = objective_spread(oracle_mod, red, 1e-6, max_iters=400_000)
    xr, yr, _, _ = oracle_mod.Oracle(red).solve(1e-6, 400_000)
    _, _, _, post = run_postsolve(shim, lp, xr, yr)
    say(f"  gpu pobj {info['pobj']:.12g}, oracle on the reduced LP mapped back {post['pobj']:.12g}, spread {dev:.2e}")
    assert abs(info["pobj"] - post["pobj"]) <= bar, (info["pobj"], post["pobj"], dev)
    assert ev["bound_viol"] <= 1e-12 * (1 + np.abs(x).max())


def test_presolved_warm_start_in_original_space(lpmod):
    """lp_set_start takes original-space vectors: started at HiGHS's optimum
    of the original LP, the presolved solve stops within two checks."""
    say("case presolve warm start")
    lp = gen.presolve_lp(2)
    _, xh, yh = highs(lp)
    p = lpmod.Problem(lp, presolve=1)
    p.set_start(xh, yh)
    info = p.solve(1e-6, 400_000)
    assert info["status"] == "OPTIMAL" and info["iterations"] <= 128


def test_no_reduction_keeps_the_problem(lpmod, oracle_mod):
    """With nothing to remove the presolve flag changes nothing: same size,
    same iterates, bit-identical result."""
    say("case presolve no-op")
    rng = np.random.default_rng(3)
    import scipy.sparse as sp
    K = sp.csr_matrix(rng.uniform(0.5, 1.5, (6, 9)))
    lp = gen.LPData(m=6, n=9, m1=2, row_ptr=K.indptr.astype(np.int32), col=K.indices.astype(np.int32),
                    val=K.data, c=rng.standard_normal(9), q=np.ones(6), l=np.zeros(9), u=np.full(9, 10.0))
    a, b = lpmod.Problem(lp, presolve=1), lpmod.Problem(lp)
    assert a.presolved_size() == (6, 9)
    ia, ib = a.solve(1e-6, 100_000), b.solve(1e-6, 100_000)
    assert ia["iterations"] == ib["iterations"]
    assert all(np.array_equal(u, v) for u, v in zip(a.result()[:3], b.result()[:3]))


def test_everything_removable_solves_the_original(lpmod):
    """Every row is a singleton and every column would then be fixed: the
    presolve declines, the original LP is solved, and the answer is the
    closed-form optimum x = (2, 5, 1), y = (1/2, 1, 2/3)."""
    say("case presolve declines")
    import scipy.sparse as sp
    K = sp.csr_matrix(np.array([[2.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, 3.0]]))
    lp = gen.LPData(m=3, n=3, m1=1, row_ptr=K.indptr.astype(np.int32), col=K.indices.astype(np.int32),
                    val=K.data, c=np.array([1.0, -1.0, 2.0]), q=np.array([4.0, -5.0, 3.0]),
                    l=np.array([0.0, 0.0, 0.0]), u=np.array([10.0, np.inf, np.inf]))
    p = lpmod.Problem(lp, presolve=1)
    assert p.presolved_size() == (3, 3)
    info = p.solve(1e-8, 100_000)
    assert info["status"] == "OPTIMAL"
    x, y, lam, info = p.result()
    assert np.allclose(x, [2.0, 5.0, 1.0], atol=1e-6)
    assert np.allclose(y, [0.5, 1.0, 2.0 / 3.0], atol=1e-6)
    assert info["pobj"] == pytest.approx(-1.0, abs=1e-6)
