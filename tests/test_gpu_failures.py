"""Failure handling through the C ABI on the GPU, each case forced from the
host with kernels that still exit normally: a NaN warm start (NaN-propagating
projections -> NUMERICAL, then the cold-start fallback), a time limit, an
infeasible LP (a Farkas certificate: PRIMAL_INFEASIBLE, or ITERATION_LIMIT
with the ray test off), and the per-window trace of verbose mode."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def test_nan_start_is_numerical_then_cold_fallback(lpmod, oracle_mod):
    say("case nan start")
    from paper_2312_14832_amd import warmstart
    data = gen.tiny_lp(2)
    x = np.zeros(data.n)
    x[np.flatnonzero(~np.isfinite(data.l) & ~np.isfinite(data.u))[0]] = np.nan   # a free variable keeps the NaN
    p = lpmod.Problem(data)
    p.set_start(x, None)
    info = p.solve(1e-6, 5000)
    assert info["status"] == "NUMERICAL", info
    assert info["iterations"] <= 64
    p.close()
    o = oracle_mod.Oracle(data)
    o.set_start(x, None)
    _, _, _, io = o.solve(1e-6, 5000)
    assert io["status"] == "NUMERICAL"
    info, _, fallback = warmstart.solve_with_start(data, np.concatenate([x, np.zeros(data.m)]), tol=1e-6)
    assert fallback and info["status"] == "OPTIMAL"


def test_time_limit(lpmod):
    say("case time limit")
    data = gen.large_lp(seed=3, n=200_000, m1=50_000, m2=50_000)
    p = lpmod.Problem(data)
    info = p.solve(1e-12, 10**8, 0.3)
    assert info["status"] == "TIME_LIMIT", info
    assert 0.3 <= info["seconds"] < 5.0
    x, y, lam, info2 = p.result()
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    assert info2["rel_kkt"] == info["rel_kkt"] > 1e-12


def test_infeasible_lp_detected_or_runs_to_the_limit(lpmod, oracle_mod):
    """x >= 0 with x1 + x2 = -1 has no feasible point.  With the ray test
    both paths report PRIMAL_INFEASIBLE with a dual ray y < 0; with
    infeas_tol = 0 both stop at max_iters."""
    say("case infeasible")
    data = gen.from_dense(np.array([[1.0, 1.0]]), [1.0, 1.0], [-1.0], [0.0, 0.0], [np.inf, np.inf], 1)
    p = lpmod.Problem(data)
    info = p.solve(1e-6, 200_000)
    _, _, _, io = oracle_mod.Oracle(data).solve(1e-6, 200_000)
    assert info["status"] == io["status"] == "PRIMAL_INFEASIBLE"
    _, y, _, _ = p.result()
    assert y[0] < 0 and info["dobj"] > 0
    p0 = lpmod.Problem(data, infeas_tol=0.0)
    info = p0.solve(1e-6, 2000)
    assert info["status"] == "ITERATION_LIMIT" and info["iterations"] == 2000
    assert info["rel_primal"] > 1e-3
    _, _, _, io = oracle_mod.Oracle(data, infeas_tol=0.0).solve(1e-6, 2000)
    assert io["status"] == "ITERATION_LIMIT"


def test_verbose_trace_lines(lpmod, capfd):
    say("case verbose")
    p = lpmod.Problem(gen.tiny_lp(4), verbose=1)
    info = p.solve(1e-6, 200_000)
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("[lp] k=")]
    assert lines and lines[-1].endswith("(done)")
    assert f"k={info['iterations']} " in lines[-1]
    assert "KKT_omega" in lines[0] and "rel_gap" in lines[0]
