"""Mixed precision (FP32 matrix values and iterates; FP64 reductions, step
size, primal weight and KKT) against the FP64 oracle.

Tolerances come from the arithmetic: every FP32 vector entry of one step is
a handful of FP32 operations (unit roundoff u32 = 2^-24 ~ 6e-8) on inputs
that are themselves FP32 roundings of the oracle's doubles, so a normwise
relative difference of 64*u32 ~ 4e-6 bounds one step; the scalars follow
the same conditioning argument as in FP64 with u32 in place of u64."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from lp_helpers import objective_band
from gpu_helpers import gpu_state, ints_equal, say, scalar_diff, step_condition, vec_diff

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
VEC_TOL = 64 * U32


def scalar_tol32(kappa):
    return 64 * U32 * max(kappa, 1.0)


@pytest.mark.parametrize("seed", [0, 3])
def test_mixed_scaling_and_spmv(lpmod, oracle_mod, seed):
    say(f"case mixed spmv seed={seed}")
    data = gen.tiny_lp(seed)
    p = lpmod.Problem(data, precision="mixed", slice_kib=1)
    o = oracle_mod.Oracle(data)
    Dr, Dc = p.scaling()
    Dr_o, Dc_o, _ = o.scaling()
    # the scaling itself runs in FP64 in both precisions
    assert np.max(np.abs(Dr - Dr_o) / Dr_o) < 1e-13
    assert np.max(np.abs(Dc - Dc_o) / Dc_o) < 1e-13
    rng = np.random.default_rng(5)
    for tr, ln in [(False, data.n), (True, data.m)]:
        v = rng.standard_normal(ln).astype(np.float32).astype(np.float64)
        g = p.spmv(v, transpose=tr)
        r = o.spmv(v, transpose=tr)
        assert np.linalg.norm(g - r) <= VEC_TOL * np.linalg.norm(r), tr


@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_lockstep(lpmod, oracle_mod, seed):
    """One accepted step from the oracle's state (rounded to FP32) against the
    oracle's next state."""
    data = gen.tiny_lp(seed)
    p = lpmod.Problem(data, precision="mixed")
    o = oracle_mod.Oracle(data)
    for k in [0, 5, 63, 200, 511]:
        say(f"case mixed lockstep seed={seed} k={k}")
        o.solve(1e-30, k)
        raw = o.get_state_raw()
        prev = o.get_state()
        o.solve(1e-30, k + 1)
        so = o.get_state()
        if so["k"] < k + 1:
            break
        p.set_state(raw)
        p.solve(1e-30, k + 1)
        sg = gpu_state(lpmod, p)
        assert ints_equal(sg, so), k
        wv, vv = vec_diff(sg, so)
        assert wv < VEC_TOL, (k, vv, wv)
        kap = step_condition(prev, so)
        for name, r in scalar_diff(sg, so).items():
            if name == "KKT0":
                continue  # compared through the decisions (restart counts) above
            assert r < scalar_tol32(kap), (k, name, r, kap)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_mixed_solves_to_1e4(lpmod, oracle_mod, seed):
    """The mixed-precision result, unscaled and evaluated by the oracle on the
    FP64 data, meets the termination criteria at 1e-4 (up to the FP32
    rounding of the data, 2e-6), and its objective is within the gap
    tolerance of the FP64 oracle's."""
    say(f"case mixed solve seed={seed}")
    data = gen.tiny_lp(seed)
    p = lpmod.Problem(data, precision="mixed")
    info = p.solve(1e-4, 200000)
    assert info["status"] == "OPTIMAL"
    x, y, lam, _ = p.result()
    o = oracle_mod.Oracle(data)
    ev = o.eval_unscaled(x, y)
    assert ev["rel_kkt"] <= 1e-4 + 2e-6, ev
    xo, yo, _, io = o.solve(1e-4, 200000)
    assert abs(info["pobj"] - io["pobj"]) <= objective_band(1e-4, data, xo, yo, io["pobj"], io["dobj"])
    say(f"  mixed pobj {info['pobj']:.9g} fp64-oracle pobj {io['pobj']:.9g} "
        f"rel diff {abs(info['pobj'] - io['pobj']) / abs(io['pobj']):.2e}; oracle-evaluated rel_kkt {ev['rel_kkt']:.3e}")


def test_mixed_full_size(lpmod, oracle_mod):
    """The 4e6 x 2e6, ~4e7-nonzero mixed-precision workload: scaling and both
    products on full vectors against the oracle, and one lockstep step."""
    say("case mixed full size: generate")
    data = gen.large_lp(seed=2, n=4_000_000, m1=1_000_000, m2=1_000_000)
    say("case mixed full size: load")
    p = lpmod.Problem(data, precision="mixed")
    assert p.layout() == (8, 4)
    o = oracle_mod.Oracle(data)
    Dr, Dc = p.scaling()
    Dr_o, Dc_o, _ = o.scaling()
    assert np.max(np.abs(Dr - Dr_o) / Dr_o) < 1e-12
    rng = np.random.default_rng(7)
    for tr, ln in [(False, data.n), (True, data.m)]:
        say(f"case mixed full size: spmv transpose={tr}")
        v = rng.standard_normal(ln).astype(np.float32).astype(np.float64)
        g = p.spmv(v, transpose=tr)
        r = o.spmv(v, transpose=tr)
        assert np.linalg.norm(g - r) <= VEC_TOL * np.linalg.norm(r), tr
    say("case mixed full size: lockstep k=0")
    o.solve(1e-30, 0)
    raw = o.get_state_raw()
    o.solve(1e-30, 1)
    so = o.get_state()
    p.set_state(raw)
    p.solve(1e-30, 1)
    sg = gpu_state(lpmod, p)
    assert ints_equal(sg, so)
    wv, vv = vec_diff(sg, so)
    assert wv < VEC_TOL, (vv, wv)
