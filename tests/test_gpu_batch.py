"""Batched solves (lp_batch_*): every instance of one batch follows the same
method as a single solve, with its own step size, primal weight, restarts and
termination.  Checked per instance against the FP64 oracle (lockstep steps,
1e-4 results) and against single-LP GPU runs."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from gpu_helpers import (free_running_band, gpu_state, ints_equal, kkt_scale, objective_spread, say,
                         scalar_diff, step_condition, vec_diff)

pytestmark = pytest.mark.gpu

PER_STEP_TOL = 1e-10
U64 = 2.0 ** -53


def small_batch(count=10, seed0=1000):
    """Uneven small members of the batched workload (n log-uniform in
    [200, 6000]) plus a box-only instance (m = 0) and one with long rows."""
    lps = [gen.batch_member(seed0 + i, n_lo=200, n_hi=6000) for i in range(count)]
    lps.append(gen.box_only_lp(5, n=300))
    rng = np.random.Generator(np.random.PCG64(77))
    counts = rng.integers(0, 5, size=400)
    counts[:3] = [600, 900, 2400]   # a row of K' longer than one LDS row block
    lps.append(gen.certificate_lp(rng, 1000, 1500, counts.astype(np.int64)))
    return lps


def tiny_batch(count=8, seed0=5000):
    """Small LPs for the one-workgroup-per-instance loop: 200 to 900 columns
    (some past 512, so each thread holds two columns and rows), 2 to 5
    nonzeros per column."""
    rng = np.random.Generator(np.random.PCG64(seed0))
    lps = []
    for i in range(count):
        n = int(rng.integers(200, 900))
        lps.append(gen.tiny_lp(seed0 + i, n=n, m1=int(rng.integers(n // 10, n // 4)),
                               m2=int(rng.integers(n // 10, n // 4)), per_col=int(rng.integers(2, 6))))
    return lps


@pytest.mark.parametrize("split", [-1, 1])
def test_batch_lockstep_fp64(lpmod, oracle_mod, split):
    """split: the products' short-row blocks summed one row per thread (the
    default) or split by entries."""
    lps = small_batch()
    bt = lpmod.Batch(lps, split_sums=split)
    assert bt.loop_form() == 0
    batch_lockstep(lpmod, oracle_mod, lps, bt, [0, 1, 63, 64, 200, 511])


def test_small_batch_one_workgroup_lockstep(lpmod, oracle_mod):
    """A batch of small LPs runs one workgroup per instance, each on its own
    whole loop; every instance still follows the oracle step by step."""
    lps = tiny_batch()
    bt = lpmod.Batch(lps)
    assert bt.loop_form() == 1
    batch_lockstep(lpmod, oracle_mod, lps, bt, [0, 1, 63, 64, 200])


def batch_lockstep(lpmod, oracle_mod, lps, bt, ks):
    oracles = [oracle_mod.Oracle(p) for p in lps]
    for k in ks:
        say(f"case batch lockstep k={k}")
        raws, prevs, nexts = [], [], []
        for o in oracles:
            o.solve(1e-30, k)
            raws.append(o.get_state_raw())
            prevs.append(o.get_state())
            o.solve(1e-30, k + 1)
            nexts.append(o.get_state())
        for i, raw in enumerate(raws):
            bt.set_state(i, raw)
        bt.solve(1e-30, k + 1)
        for i, (p, o) in enumerate(zip(lps, oracles)):
            so = nexts[i]
            if so["k"] < k + 1:
                continue  # the oracle met rel KKT <= 1e-30 exactly
            sg = lpmod.unpack_state(bt.get_state(i), p.n, p.m)
            assert ints_equal(sg, so), (k, i)
            wv, vv = vec_diff(sg, so)
            assert wv < PER_STEP_TOL, (k, i, vv, wv)
            kap = step_condition(prevs[i], so)
            Dr, Dc, _ = o.scaling()
            for name, r in scalar_diff(sg, so).items():
                if name == "KKT0":
                    assert abs(sg["KKT0"] - so["KKT0"]) <= PER_STEP_TOL * kkt_scale(so, Dr, Dc, p), (k, i)
                else:
                    assert r < max(PER_STEP_TOL, 64 * U64 * kap), (k, i, name, r, kap)


def test_batch_matches_single_lp_runs(lpmod):
    """Free-running batch instances against single-LP GPU runs of the same
    instances inside the first check window (both deterministic; only the
    summation order of the reductions differs)."""
    lps = small_batch(6, seed0=2000)
    bt = lpmod.Batch(lps)
    bt.solve(1e-30, 40)
    for i, p in enumerate(lps):
        say(f"case batch vs single i={i}")
        single = lpmod.Problem(p)
        single.solve(1e-30, 40)
        sg = lpmod.unpack_state(bt.get_state(i), p.n, p.m)
        ss = gpu_state(lpmod, single)
        assert ints_equal(sg, ss), i
        wv, vv = vec_diff(sg, ss)
        assert wv < PER_STEP_TOL, (i, vv, wv)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_solves_to_1e4(lpmod, oracle_mod, precision):
    lps = small_batch(10, seed0=3000)
    bt = lpmod.Batch(lps, precision=precision)
    bt.solve(1e-4, 200000, 120.0)
    for i, p in enumerate(lps):
        x, y, lam, info = bt.result(i)
        say(f"case batch {precision} i={i}: {info['status']} k={info['iterations']} pobj={info['pobj']:.9g}")
        assert info["status"] == "OPTIMAL", (i, info)
        o = oracle_mod.Oracle(p)
        ev = o.eval_unscaled(x, y)
        assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6), (i, ev)
        if precision == "mixed":
            # the reported criteria are the FP64 re-check's, i.e. the oracle's evaluation
            for k, kk in (("rel_primal", "rel_p"), ("rel_dual", "rel_d"), ("rel_gap", "rel_g")):
                assert info[k] == pytest.approx(ev[kk], rel=1e-8, abs=1e-14), (i, k, info[k], ev[kk])
        # the measured objective bar, perturbing at the unit roundoff of the
        # iterates (FP64, or FP32 in mixed precision)
        io, dev, bar = objective_spread(oracle_mod, p, 1e-4, rel=1e-15 if precision == "fp64" else 2.0 ** -24)
        assert abs(info["pobj"] - io["pobj"]) <= bar, (i, info["pobj"], io["pobj"], dev)


def test_batch_resume_bitwise(lpmod):
    say("case batch resume")
    lps = small_batch(5, seed0=4000)
    bt = lpmod.Batch(lps)
    bt.solve(1e-30, 256)
    full = [bt.get_state(i) for i in range(len(lps))]
    bt.solve(1e-30, 128)
    mid = [bt.get_state(i) for i in range(len(lps))]
    for i, s in enumerate(mid):
        bt.set_state(i, s)
    bt.solve(1e-30, 256)
    for i in range(len(lps)):
        if full[i][5] < 256:
            continue  # met rel KKT <= 1e-30 exactly before 256 steps: its state stopped there
        assert np.array_equal(bt.get_state(i)[16:], full[i][16:]), i


def test_batch_autotuned_layout(lpmod):
    """With autotune the batch keeps one of the four timed row-block shapes
    per product, and the method is unchanged: one step from the same state
    matches the untuned batch to 1e-10 (only the summation order of rows
    longer than a block can differ; 40 steps stay inside the first check
    window), and every instance still solves to 1e-4."""
    say("case batch autotune")
    lps = small_batch(8, seed0=4000)
    tuned = lpmod.Batch(lps, autotune=1)
    plain = lpmod.Batch(lps)
    shapes = {(2048, 1024), (1024, 1024), (2048, 256), (1024, 256)}
    assert tuned.layout_blocks(0) in shapes and tuned.layout_blocks(1) in shapes
    assert plain.layout_blocks(0) == (2048, 1024) == plain.layout_blocks(1)
    tuned.solve(1e-30, 40)
    plain.solve(1e-30, 40)
    for i, p in enumerate(lps):
        st, sp = (lpmod.unpack_state(b.get_state(i), p.n, p.m) for b in (tuned, plain))
        assert ints_equal(st, sp), i
        wv, vv = vec_diff(st, sp)
        assert wv < PER_STEP_TOL, (i, vv, wv)
    tuned.solve(1e-4, 200000, 120.0)
    for i in range(len(lps)):
        assert tuned.info(i)["status"] == "OPTIMAL", i


def test_batch_full_size_sampled(lpmod, oracle_mod):
    """The 512-member batch the bench times (1.2e8 nonzeros), in its launch
    configuration (FP32 iterates, autotuned row blocks): every instance is
    set to the oracle's state of its own LP, one step is taken for all at
    once, and sampled instances (smallest, largest, spread between) are
    held to the FP32 one-step bound against the oracle's next state; every
    other instance must have advanced exactly one accepted step."""
    say("case batch full size: generate")
    lps = [gen.batch_member(1000 + i) for i in range(512)]
    say("case batch full size: load")
    bt = lpmod.Batch(lps, precision="mixed", autotune=1)
    sizes = np.array([p.nnz for p in lps])
    order = np.argsort(sizes)
    sample = sorted(set(int(i) for i in order[[0, 1, 128, 256, 384, 510, 511]]))
    k = 63   # the step that closes the first check window
    oracles = {}
    for i in sample:
        say(f"case batch full size: oracle {i} (nnz {sizes[i]})")
        o = oracle_mod.Oracle(lps[i])
        o.solve(1e-30, k)
        raw = o.get_state_raw()
        prev = o.get_state()
        o.solve(1e-30, k + 1)
        oracles[i] = (raw, prev, o.get_state())
    bt.solve(1e-30, k)   # every instance at k accepted steps of its own run
    for i, (raw, _, _) in oracles.items():
        bt.set_state(i, raw)
    others = [i for i in range(512) if i not in oracles]
    for i in others:
        bt.set_state(i, bt.get_state(i))
    say("case batch full size: one step for all 512")
    bt.solve(1e-30, k + 1)
    for i, (raw, prev, so) in oracles.items():
        p = lps[i]
        sg = lpmod.unpack_state(bt.get_state(i), p.n, p.m)
        assert ints_equal(sg, so), i
        wv, vv = vec_diff(sg, so)
        assert wv < 64 * 2.0 ** -24, (i, vv, wv)
    for i in others[::37]:
        assert bt.info(i)["iterations"] == k + 1, i


def test_batch_with_dense_rows(lpmod, oracle_mod):
    """A batch holding PageRank LPs (a 20,000-entry row each, summed by one
    workgroup in the batch path) next to small LPs: the first 40 free-running
    steps stay within the band in which the oracle differs from itself after a
    1e-15 perturbation of its first step (x100, as for the single-LP
    free-running test; the step-size rule amplifies ulp differences on these
    LPs), and every instance solves to 1e-6."""
    lps = [gen.pagerank_lp(5, 20000), gen.tiny_lp(1), gen.pagerank_lp(6, 12000)]
    bt = lpmod.Batch(lps)
    bt.solve(1e-30, 40)
    for i, p in enumerate(lps):
        say(f"case batch dense rows i={i}")
        o = oracle_mod.Oracle(p)
        o.solve(1e-30, 40)
        sg = lpmod.unpack_state(bt.get_state(i), p.n, p.m)
        so = o.get_state()
        assert ints_equal(sg, so), i
        wv, vv = vec_diff(sg, so)
        band = free_running_band(oracle_mod, p, 40, so)
        say(f"  gpu-vs-oracle {wv:.2e} ({vv}), oracle-vs-perturbed-oracle {band:.2e}")
        assert wv <= max(PER_STEP_TOL, 100.0 * band), (i, vv, wv, band)
    bt2 = lpmod.Batch(lps)
    bt2.solve(1e-6, 200_000)
    for i, p in enumerate(lps):
        x, y, lam, info = bt2.result(i)
        assert info["status"] == "OPTIMAL", (i, info)
        ev = oracle_mod.Oracle(p).eval_unscaled(x, y)
        assert ev["rel_kkt"] <= 1e-6 * (1 + 1e-6), (i, ev)


@pytest.mark.parametrize("autotune", [0, 1])
def test_batch_resume_on_dirty_memory(lpmod, oracle_mod, monkeypatch, autotune):
    """A batch whose device memory starts as 0xFF bytes (NaN in every float;
    the library's PDLP_DEBUG_FILL_BYTE test hook) resumes exactly: the chunk
    padding and the autotuner's trial buffers read as the zeros the load
    writes, not as what the memory held before."""
    say(f"case batch resume on dirty memory autotune={autotune}")
    monkeypatch.setenv("PDLP_DEBUG_FILL_BYTE", "255")
    lps = small_batch()
    bt = lpmod.Batch(lps, autotune=autotune)
    monkeypatch.delenv("PDLP_DEBUG_FILL_BYTE")
    oracles = [oracle_mod.Oracle(p) for p in lps]
    raws, nexts = [], []
    for o in oracles:
        o.solve(1e-30, 0)
        raws.append(o.get_state_raw())
        o.solve(1e-30, 1)
        nexts.append(o.get_state())
    for i, raw in enumerate(raws):
        bt.set_state(i, raw)
    bt.solve(1e-30, 1)
    for i, p in enumerate(lps):
        sg = lpmod.unpack_state(bt.get_state(i), p.n, p.m)
        so = nexts[i]
        assert ints_equal(sg, so), i
        for name in ("eta_hat", "omega", "W", "eta_last"):
            assert abs(sg[name] - so[name]) <= 1e-9 * abs(so[name]) + 1e-300, (i, name, sg[name], so[name])


def test_batch_narrowed_launches_change_nothing(lpmod):
    """Once half of the instances have finished, the batch launches only the
    chunks and row blocks of the others.  An instance's arithmetic does not
    depend on its neighbours, so the instances that finish last end bit for
    bit where they end when solved alone (a batch of one, never narrowed)."""
    say("case batch narrowing")
    lps = small_batch(10, seed0=4000)
    bt = lpmod.Batch(lps, autotune=0)
    assert bt.loop_form() == 0
    bt.solve(1e-6, 200_000, 120.0)
    infos = [bt.info(i) for i in range(len(lps))]
    order = sorted(range(len(lps)), key=lambda i: infos[i]["iterations"])
    last = order[-1]
    # more than half finished at least a window (64 slots) before the last one
    early = sum(1 for d in infos if d["iterations"] + 64 <= infos[last]["iterations"])
    say(f"  iterations {[d['iterations'] for d in infos]}; {early} finished a window or more before the last")
    assert 2 * early > len(lps)
    for i in order[-2:]:
        alone = lpmod.Batch([lps[i]], autotune=0, persistent=0)   # the same launches, never narrowed
        alone.solve(1e-6, 200_000, 120.0)
        a = alone.info(0)
        assert a["status"] == infos[i]["status"] == "OPTIMAL", (i, a, infos[i])
        assert a["iterations"] == infos[i]["iterations"], (i, a["iterations"], infos[i]["iterations"])
        assert np.array_equal(alone.get_state(0), bt.get_state(i)), i


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_batch_one_workgroup_solves(lpmod, oracle_mod, precision):
    """The one-workgroup-per-instance batch and the batched launches both
    solve every instance to 1e-4; the returned points meet the criteria in
    the oracle's evaluation and their objectives lie within the measured bar."""
    lps = tiny_batch(4, seed0=6000)   # (the fifth of this family stalls short of 1e-4 in FP32 iterates)
    one = lpmod.Batch(lps, precision=precision)
    launches = lpmod.Batch(lps, precision=precision, persistent=0)
    assert one.loop_form() == 1 and launches.loop_form() == 0
    for bt in (one, launches):
        bt.solve(1e-4, 200_000, 60.0)
        for i, p in enumerate(lps):
            x, y, lam, info = bt.result(i)
            say(f"case small batch {precision} form={bt.loop_form()} i={i}: {info['status']} k={info['iterations']}")
            assert info["status"] == "OPTIMAL", (i, info)
            ev = oracle_mod.Oracle(p).eval_unscaled(x, y)
            assert ev["rel_kkt"] <= 1e-4 * (1 + 1e-6), (i, ev)
            if precision == "mixed":
                # the reported criteria are the FP64 re-check's, i.e. the oracle's evaluation
                for k, kk in (("rel_primal", "rel_p"), ("rel_dual", "rel_d"), ("rel_gap", "rel_g")):
                    assert info[k] == pytest.approx(ev[kk], rel=1e-8, abs=1e-14), (i, k, info[k], ev[kk])
            io, dev, bar = objective_spread(oracle_mod, p, 1e-4, rel=1e-15 if precision == "fp64" else 2.0 ** -24)
            assert abs(info["pobj"] - io["pobj"]) <= bar, (i, info["pobj"], io["pobj"], dev)


def test_small_batch_one_workgroup_resume_bitwise(lpmod):
    """N + N resumed steps of the one-workgroup batch equal 2N steps bit for bit."""
    lps = tiny_batch(4, seed0=7000)
    bt = lpmod.Batch(lps)
    assert bt.loop_form() == 1
    bt.solve(1e-30, 256)
    full = [bt.get_state(i) for i in range(len(lps))]
    bt.solve(1e-30, 128)
    for i in range(len(lps)):
        bt.set_state(i, bt.get_state(i))
    bt.solve(1e-30, 256)
    for i in range(len(lps)):
        if full[i][5] < 256:
            continue  # met rel KKT <= 1e-30 exactly before 256 steps
        assert np.array_equal(bt.get_state(i)[16:], full[i][16:]), i
