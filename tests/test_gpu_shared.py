"""Batched solves of one family over a shared matrix (lp_shared_*): each
instance follows the single-LP method with its own step size, primal
weight, restarts and termination, while every product reads K once for all
instances.  Checked per instance against the FP64 oracle: lockstep steps to
1e-10 (across checks and restarts), free-running steps inside the first
check window, warm starts, and 1e-4 results held to the measured objective
bar."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from gpu_helpers import (gpu_state, ints_equal, kkt_scale, objective_spread, say, scalar_diff, step_condition,
                         vec_diff)

pytestmark = pytest.mark.gpu

PER_STEP_TOL = 1e-10
U64 = 2.0 ** -53


def family(count, n=3000, m1=600, m2=900, per_col=5, seed=41, with_bounds=False):
    """count members of a small parametric family (the warm-start family's
    generator at a small size).  with_bounds: members also get their own
    bounds (each finite upper bound raised by U(0, 2), which keeps the
    member's certificate feasible)."""
    base = gen.parametric_base(seed=seed, n=n, m1=m1, m2=m2, per_col=per_col)
    lps = [gen.parametric_instance(base, 500 + i) for i in range(count)]
    if with_bounds:
        out = []
        for i, p in enumerate(lps):
            rng = np.random.default_rng(900 + i)
            l = p.l.copy()
            u = p.u.copy()
            fin = np.isfinite(u)
            u[fin] = np.maximum(u[fin] + rng.uniform(0, 2, fin.sum()), p.x0[fin])
            out.append(gen.LPData(m=p.m, n=p.n, m1=p.m1, row_ptr=p.row_ptr, col=p.col, val=p.val, c=p.c, q=p.q,
                                  l=l, u=u, x0=p.x0, y0=p.y0, lam0=p.lam0, s=p.s))
        lps = out
    return lps


def check_close(sg, so, prev, o, p, label):
    assert ints_equal(sg, so), label
    wv, vv = vec_diff(sg, so)
    assert wv < PER_STEP_TOL, (label, vv, wv)
    kap = step_condition(prev, so)
    Dr, Dc, _ = o.scaling()
    for name, r in scalar_diff(sg, so).items():
        if name == "KKT0":
            assert abs(sg["KKT0"] - so["KKT0"]) <= PER_STEP_TOL * kkt_scale(so, Dr, Dc, p), (label, name)
        else:
            assert r < max(PER_STEP_TOL, 64 * U64 * kap), (label, name, r, kap)


@pytest.mark.parametrize("count,steps", [(5, 1), (5, 8), (1, 1), (33, 1), (100, 1)])
def test_shared_lockstep(lpmod, oracle_mod, count, steps):
    """From each instance's oracle state, `steps` steps on the GPU equal the
    oracle's next states; 8-step windows straddle the check at k = 64 (and
    its restarts).  count = 5 pads to 8 interleaved instances, 33 to 64, 100
    to 128 (two wavefronts per instance in the per-instance sums)."""
    lps = family(count)
    sh = lpmod.Shared(lps)
    oracles = [oracle_mod.Oracle(p) for p in lps]
    for k in ([0, 5, 63, 200] if steps == 1 else [58, 60, 62, 124]):
        say(f"case shared lockstep count={count} k={k} steps={steps}")
        raws, prevs, nexts = [], [], []
        for o in oracles:
            o.solve(1e-30, k)
            raws.append(o.get_state_raw())
            o.solve(1e-30, k + steps - 1)
            prevs.append(o.get_state())
            o.solve(1e-30, k + steps)
            nexts.append(o.get_state())
        for i, raw in enumerate(raws):
            sh.set_state(i, raw)
        sh.solve(1e-30, k + steps)
        for i, (p, o) in enumerate(zip(lps, oracles)):
            so = nexts[i]
            if so["k"] < k + steps:
                continue
            sg = lpmod.unpack_state(sh.get_state(i), p.n, p.m)
            check_close(sg, so, prevs[i], o, p, (k, i))


def check_free(sg, so, label):
    """Free-running runs (no resynchronisation per step): counters equal and
    vectors to 1e-10, as in the single-LP free-running test; the step-size
    scalars carry the rounding of every earlier step's eta_bar ratio, so they
    are compared through the vectors and counters they drive."""
    assert ints_equal(sg, so), label
    wv, vv = vec_diff(sg, so)
    assert wv < PER_STEP_TOL, (label, vv, wv)


def test_shared_free_running_first_window(lpmod, oracle_mod):
    """Fresh solves of 64 steps from the cold start: every instance equals its
    oracle run to 1e-10 (inside the first check window the method's own
    amplification of rounding stays below that)."""
    lps = family(6, with_bounds=True)
    sh = lpmod.Shared(lps)
    sh.solve(1e-30, 64)
    for i, p in enumerate(lps):
        say(f"case shared free i={i}")
        o = oracle_mod.Oracle(p)
        o.solve(1e-30, 64)
        sg = lpmod.unpack_state(sh.get_state(i), p.n, p.m)
        check_free(sg, o.get_state(), i)


def test_shared_warm_start_lockstep(lpmod, oracle_mod):
    """Per-instance start points and primal weights (lp_shared_set_start) give
    the oracle's 40 free-running steps from the same start; instances without
    a start are cold."""
    lps = family(4)
    sh = lpmod.Shared(lps)
    rng = np.random.default_rng(5)
    oracles = []
    for i, p in enumerate(lps):
        o = oracle_mod.Oracle(p)
        if i % 2 == 0:
            x0 = p.x0 + 0.1 * rng.standard_normal(p.n)
            y0 = p.y0 + 0.1 * rng.standard_normal(p.m)
            om = 0.5 + i
            sh.set_start(i, x0, y0, om)
            o.set_start(x0, y0)
            o.set_start_weight(om)
        oracles.append(o)
    sh.solve(1e-30, 40)
    for i, (p, o) in enumerate(zip(lps, oracles)):
        say(f"case shared warm i={i}")
        o.solve(1e-30, 40)
        sg = lpmod.unpack_state(sh.get_state(i), p.n, p.m)
        check_free(sg, o.get_state(), i)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shared_solves_to_1e4(lpmod, oracle_mod, precision):
    """Every instance ends OPTIMAL; its point, evaluated by the oracle on the
    original data, meets the criteria at 1e-4, and its objective lies within
    the measured bar of the oracle's (perturbing at the iterates' unit
    roundoff)."""
    lps = family(7, with_bounds=True)
    sh = lpmod.Shared(lps, precision=precision)
    sh.solve(1e-4, 200000, 120.0)
    rel = 1e-15 if precision == "fp64" else 2.0 ** -24
    for i, p in enumerate(lps):
        x, y, lam, info = sh.result(i)
        say(f"case shared {precision} i={i}: {info['status']} k={info['iterations']} pobj={info['pobj']:.9g}")
        assert info["status"] == "OPTIMAL", (i, info)
        ev = oracle_mod.Oracle(p).eval_unscaled(x, y)
        assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6), (i, ev)
        if precision == "mixed":
            # the reported criteria are the FP64 re-check's, i.e. the oracle's evaluation
            for k, kk in (("rel_primal", "rel_p"), ("rel_dual", "rel_d"), ("rel_gap", "rel_g")):
                assert info[k] == pytest.approx(ev[kk], rel=1e-8, abs=1e-14), (i, k, info[k], ev[kk])
        io, dev, bar = objective_spread(oracle_mod, p, 1e-4, rel=rel)
        assert abs(info["pobj"] - io["pobj"]) <= bar, (i, info["pobj"], io["pobj"], dev)
        fl, fu = np.isfinite(p.l), np.isfinite(p.u)
        assert np.all(lam[~fl & ~fu] == 0) and np.all(lam[fl & ~fu] >= 0) and np.all(lam[~fl & fu] <= 0)


def test_shared_matches_single_lp_handles(lpmod):
    """The same instances through single-LP handles: the first 64 steps agree
    to 1e-10 (only the summation order of the products differs)."""
    lps = family(3)
    sh = lpmod.Shared(lps)
    sh.solve(1e-30, 64)
    for i, p in enumerate(lps):
        say(f"case shared vs single i={i}")
        single = lpmod.Problem(p)
        single.solve(1e-30, 64)
        sg = lpmod.unpack_state(sh.get_state(i), p.n, p.m)
        ss = gpu_state(lpmod, single)
        assert ints_equal(sg, ss), i
        wv, vv = vec_diff(sg, ss)
        assert wv < PER_STEP_TOL, (i, vv, wv)


def test_shared_rejects_bad_input(lpmod):
    lps = family(2)
    bad = lps[1]
    c = bad.c.copy()
    c[3] = np.nan
    with pytest.raises(lpmod.LPError) as e:
        lpmod.Shared([lps[0], gen.LPData(m=bad.m, n=bad.n, m1=bad.m1, row_ptr=bad.row_ptr, col=bad.col,
                                         val=bad.val, c=c, q=bad.q, l=bad.l, u=bad.u)])
    assert e.value.code == -3
    u = bad.u.copy()
    u[0] = bad.l[0] - 1.0
    with pytest.raises(lpmod.LPError) as e:
        lpmod.Shared([lps[0], gen.LPData(m=bad.m, n=bad.n, m1=bad.m1, row_ptr=bad.row_ptr, col=bad.col,
                                         val=bad.val, c=bad.c, q=bad.q, l=bad.l, u=u)])
    assert e.value.code == -4
    with pytest.raises(lpmod.LPError) as e:
        lpmod.Shared(lps * 129)   # 258 > 256 instances
    assert e.value.code == -1
