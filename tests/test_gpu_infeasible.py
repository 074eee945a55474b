"""GPU parity of the infeasibility and unboundedness certificates (Farkas
rays: differences of the current iterate from the restart anchor, tested at
each check) against the FP64 CPU oracle, on LPs that HiGHS confirms have no
solution, single and batched."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from lp_helpers import farkas_ratios
from gpu_helpers import say

pytestmark = pytest.mark.gpu

WANT = {"primal": "PRIMAL_INFEASIBLE", "dual": "DUAL_INFEASIBLE"}


def assert_certificate(lp, x, y, kind, tol):
    """The returned rays meet Farkas' conditions on the unscaled data."""
    dobj, dres, pobj, pres = farkas_ratios(lp, x, y)
    if kind == "primal":
        assert dobj > 0 and dres <= tol * dobj * (1 + 1e-6), (dobj, dres)
    else:
        assert pobj < 0 and pres <= tol * -pobj * (1 + 1e-6), (pobj, pres)


@pytest.mark.parametrize("kind", ["primal", "dual"])
@pytest.mark.parametrize("seed", [0, 1])
def test_status_and_certificate_match_oracle(lpmod, oracle_mod, kind, seed):
    """Same status as the oracle, a valid certificate, and (the iteration is
    chaotic) a detection point within 4x of the oracle's."""
    say(f"case infeasible {kind} seed={seed}")
    lp = gen.infeasible_lp(seed, kind)
    p = lpmod.Problem(lp)
    info = p.solve(1e-8, 600_000)
    _, _, _, io = oracle_mod.Oracle(lp).solve(1e-8, 600_000)
    say(f"  gpu {info['status']} at {info['iterations']}, oracle {io['status']} at {io['iterations']}")
    assert io["status"] == WANT[kind] and info["status"] == WANT[kind]
    x, y, lam, _ = p.result()
    assert_certificate(lp, x, y, kind, 1e-8)
    if kind == "primal":
        assert info["dobj"] == pytest.approx(farkas_ratios(lp, x, y)[0], rel=1e-9)
    else:
        assert info["pobj"] == pytest.approx(farkas_ratios(lp, x, y)[2], rel=1e-9)
    assert 0.25 * io["iterations"] <= info["iterations"] <= 4.0 * io["iterations"]


@pytest.mark.parametrize("kind", ["primal", "dual"])
def test_detection_window_lockstep(lpmod, oracle_mod, kind):
    """From the oracle's state at the check before it detects, the GPU runs
    the same 64-step window and detects at the same check, with rays equal
    to the oracle's (relative to their size)."""
    lp = gen.infeasible_lp(0, kind)
    o = oracle_mod.Oracle(lp)
    _, _, _, io = o.solve(1e-8, 600_000)
    kd = io["iterations"]
    xo, yo, _, _ = o.result()
    assert kd % 64 == 0 and kd >= 128
    say(f"case infeasible lockstep {kind}: oracle detects at {kd}")
    o2 = oracle_mod.Oracle(lp)
    o2.solve(1e-8, kd - 64)
    assert o2.result()[3]["status"] == "ITERATION_LIMIT"
    p = lpmod.Problem(lp)
    p.set_state(o2.get_state_raw())
    info = p.solve(1e-8, kd + 64 * 20)
    assert info["status"] == WANT[kind] and info["iterations"] == kd
    x, y, _, _ = p.result()
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo) + 1e-300
    assert np.linalg.norm(y - yo) <= 1e-8 * np.linalg.norm(yo) + 1e-300


def test_mixed_precision_detects(lpmod):
    """FP32 iterates: rays still certify, at a tolerance above FP32 rounding."""
    for kind in ("primal", "dual"):
        say(f"case infeasible mixed {kind}")
        lp = gen.infeasible_lp(0, kind)
        p = lpmod.Problem(lp, precision="mixed", infeas_tol=1e-5)
        info = p.solve(1e-4, 600_000)
        assert info["status"] == WANT[kind], info
        x, y, _, _ = p.result()
        assert_certificate(lp, x, y, kind, 2e-5)


def test_batch_reports_each_instance(lpmod):
    """A batch of a feasible LP and both kinds without a solution: each
    instance gets its own status and certificate."""
    say("case infeasible batch")
    lps = [gen.tiny_lp(3), gen.infeasible_lp(1, "primal"), gen.infeasible_lp(1, "dual")]
    bt = lpmod.Batch(lps)
    bt.solve(1e-8, 600_000)
    want = ["OPTIMAL", "PRIMAL_INFEASIBLE", "DUAL_INFEASIBLE"]
    for i, lp in enumerate(lps):
        x, y, lam, info = bt.result(i)
        assert info["status"] == want[i], (i, info)
        if i > 0:
            assert_certificate(lp, x, y, ("primal", "dual")[i - 1], 1e-8)


def test_detection_off(lpmod):
    """infeas_tol = 0: no certificate test, the run ends at the limit."""
    say("case infeasible detection off")
    lp = gen.infeasible_lp(0, "primal")
    info = lpmod.Problem(lp, infeas_tol=0.0).solve(1e-8, 30_000)
    assert info["status"] == "ITERATION_LIMIT"
