"""The pins have teeth: the oracle is rebuilt with one planted mistake at a
time (a flipped sign, a dropped term, a wrong exponent or index, a wrong
averaging weight) and at least one pin must fail for each.  The planted
builds live in a temporary directory and are used by this file only."""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild
import test_oracle_highprec as highprec
import test_oracle_pins as pins

HERE = os.path.dirname(os.path.abspath(__file__))


def check_infeasibility_bounded(om, libpath=None):
    """The certificate pins; on a planted-mistake build in a child process
    under a 20 s limit (it needs about 1 s), since a wrong step can loop on rejected steps
    forever, and a pin that does not finish fails."""
    if libpath is None:
        return pins.check_infeasibility(om)
    code = ("import sys; sys.path[:0] = [%r, %r]\n"
            "from oracle import oracle as O\nimport test_oracle_pins as p\n"
            "p.check_infeasibility(O, libpath=%r)\n") % (HERE, os.path.dirname(HERE), libpath)
    try:
        r = subprocess.run([sys.executable, "-c", code], timeout=20, capture_output=True)
    except subprocess.TimeoutExpired:
        raise AssertionError("infeasibility pins did not finish in 20 s")
    assert r.returncode == 0, r.stderr.decode()[-400:]

def check_highprec_bounded(om, libpath=None):
    """The 50-digit replay (both cases); on a planted-mistake build in a child
    process under a 60 s limit (it needs about 2 s)."""
    if libpath is None:
        for case in highprec.CASES:
            highprec.check_highprec_replay(om, case)
        return
    code = ("import sys; sys.path[:0] = [%r, %r]\n"
            "from oracle import oracle as O\nimport test_oracle_highprec as h\n"
            "[h.check_highprec_replay(O, c, libpath=%r) for c in h.CASES]\n") % (HERE, os.path.dirname(HERE), libpath)
    try:
        r = subprocess.run([sys.executable, "-c", code], timeout=60, capture_output=True)
    except subprocess.TimeoutExpired:
        raise AssertionError("50-digit replay did not finish in 60 s")
    assert r.returncode == 0, r.stderr.decode()[-400:]


MUTATIONS = {
    1: "primal step uses c + K'y",
    2: "dual step drops the extrapolation (K x+ instead of K(2x+ - x))",
    3: "Lambda = R+ case returns c - K'y unprojected",
    4: "dual objective adds +u lam- instead of -u lam-",
    5: "step-rule shrink exponent -0.03 instead of -0.3",
    6: "Ruiz column factor taken from the row maxima",
    7: "uniform instead of step-size weights in the averages",
    8: "KKT_omega uses omega instead of omega^2",
    9: "dual ray objective adds +u lam- instead of -u lam-",
    10: "primal ray test ignores the bounds' recession cone",
    11: "restart candidate is always the average",
    12: "KKT at the previous check never recorded (restart condition 2 cannot fire)",
}

CHECKS = [
    ("two PDHG steps by hand", pins.check_two_steps_golden),
    ("exact rational replay", pins.check_rational_replay),
    ("KKT_omega by hand", pins.check_kkt_omega_golden),
    ("termination quantities by hand", pins.check_termination_golden),
    ("scaling by hand", pins.check_scaling_golden),
    ("step rule constants", pins.check_step_rule),
    ("restart candidate and condition 2 by hand", pins.check_restart_golden),
    ("step-weighted averages", pins.check_step_weighted_averages),
    ("vertex enumeration", lambda om, libpath=None: pins.check_vertex_objective(om, 11, 3, 1, 2, libpath,
                                                                                  max_iters=200_000)),
    ("infeasibility certificates", check_infeasibility_bounded),
    ("50-digit replay", check_highprec_bounded),
]


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


def test_pins_pass_on_the_oracle(oracle_mod):
    for name, fn in CHECKS:
        fn(oracle_mod)


@pytest.mark.parametrize("mut", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(oracle_mod, mutant_dir, mut):
    path = obuild.build(force=True, mutation=mut, out=str(mutant_dir / f"liborc_mut{mut}.so"))
    caught = []
    for name, fn in CHECKS:
        try:
            fn(oracle_mod, libpath=path)
        except AssertionError:
            caught.append(name)
    assert caught, f"no pin fails with mistake {mut}: {MUTATIONS[mut]}"
