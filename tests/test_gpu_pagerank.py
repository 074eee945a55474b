"""GPU parity on the PageRank LP of a random graph (m = n + 1, one dense
row): the dense row is cut into chunks whose dot products the epilogue adds,
so these cases run that path in both products, under every slicing, against
the FP64 CPU oracle and against the PageRank vector itself."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from gpu_helpers import gpu_state, ints_equal, kkt_scale, say, step_condition, state_diff
from test_gpu_parity import assert_states_close
from test_oracle_pins import pagerank_vector

pytestmark = pytest.mark.gpu


def dense_rows_lp(seed, n=30000, m1=3, m2=2000):
    """Rows of every kind: five longer than the chunking threshold (8192
    entries), placed first, back to back, in the middle and last, one exactly
    at the threshold, the rest with 0-6 entries; N(0,1) values."""
    rng = np.random.default_rng(seed)
    m = m1 + m2
    lens = rng.integers(0, 7, size=m)
    for r, L in ((0, n), (1, 9000), (2, 8193), (7, 8192), (m // 2, 20000), (m - 1, 12000)):
        lens[r] = L
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([np.sort(rng.choice(n, int(L), replace=False)) for L in lens])
    vals = rng.standard_normal(rows.size)
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    np.cumsum(lens, out=row_ptr[1:])
    return gen.LPData(m=m, n=n, m1=m1, row_ptr=row_ptr, col=cols.astype(np.int32), val=vals,
                      c=rng.standard_normal(n), q=rng.standard_normal(m), l=np.zeros(n), u=np.full(n, 10.0))


@pytest.mark.parametrize("split", [-1, 1])
@pytest.mark.parametrize("slice_kib", [2048, 1])
@pytest.mark.parametrize("maker", ["pagerank", "dense_rows"])
def test_spmv_long_rows(lpmod, oracle_mod, maker, slice_kib, split):
    """K x and K' y against the oracle's CSR loops, default layout and 1 KiB
    slices (32 slices: every dense row is split over them); split = 1 sums
    the short-row blocks split by entries next to the long-row chunks."""
    say(f"case spmv {maker} slice_kib={slice_kib} split={split}")
    data = gen.pagerank_lp(2, 20000) if maker == "pagerank" else dense_rows_lp(3)
    p = lpmod.Problem(data, slice_kib=slice_kib, split_sums=split)
    o = oracle_mod.Oracle(data)
    rng = np.random.default_rng(1)
    for tr, v in [(False, rng.standard_normal(data.n)), (True, rng.standard_normal(data.m))]:
        assert_product_close(data, o, p, p.spmv(v, transpose=tr), o.spmv(v, transpose=tr), v, tr)


def assert_product_close(data, o, p, g, r, v, tr):
    """Per row: two summation orders of a row of length L differ by at most
    about 2 L u times the row's sum of |terms| (|K~| |v|, K~ the scaled
    matrix), and each side scales K with its own factors, whose relative
    difference dr_i + dc_j carries into the entry K~_ij."""
    Dr, Dc, _ = o.scaling()
    Drg, Dcg = p.scaling()
    eps = np.finfo(float).eps
    dr = np.abs(Drg - Dr) / Dr + eps
    dc = np.abs(Dcg - Dc) / Dc + eps
    K = data.csr()
    K.data = np.abs(K.data)
    K = K.multiply(1.0 / Dr[:, None]).multiply(1.0 / Dc[None, :]).tocsr()   # |K~|
    av = np.abs(v)
    if tr:   # rows of K~' are columns of K~; v is indexed by rows of K~
        M = K.T.tocsr()
        scal = dc * (M @ av) + M @ (dr * av)
    else:
        M = K
        scal = dr * (M @ av) + M @ (dc * av)
    bound = (2.0 * np.diff(M.indptr) + 4.0) * eps * (M @ av) + 2.0 * scal + 1e-300
    ratio = np.abs(g - r) / bound
    assert np.max(ratio) <= 1.0, (tr, np.max(ratio), int(np.argmax(ratio)))


@pytest.mark.parametrize("slice_kib", [2048, 1])
def test_pagerank_lockstep(lpmod, oracle_mod, slice_kib):
    """One accepted step from the oracle's state after k steps equals the
    oracle's next state to 1e-10 (the dense row's total enters the dual
    step and every check)."""
    data = gen.pagerank_lp(4, 20000)
    p = lpmod.Problem(data, slice_kib=slice_kib)
    o = oracle_mod.Oracle(data)
    Dr, Dc, _ = o.scaling()
    for k in [0, 1, 62, 63, 64, 65, 127, 128]:
        say(f"case pagerank lockstep slice_kib={slice_kib} k={k}")
        o.solve(1e-30, k)
        sk = o.get_state()
        raw = o.get_state_raw()
        o.solve(1e-30, k + 1)
        so = o.get_state()
        p.set_state(raw)
        p.solve(1e-30, k + 1)
        sg = gpu_state(lpmod, p)
        assert ints_equal(sg, so), k
        kap = step_condition(sk, so)
        say("  k=%5d kappa=%9.3g  vec %9.2e (%s)  scalar %9.2e (%s)" % ((k, kap) + state_diff(sg, so)))
        assert_states_close(sg, so, kap, f"k={k}", kkt_scale(so, Dr, Dc, data))


@pytest.mark.parametrize("precision,tol,xtol", [("fp64", 1e-8, 1e-5), ("mixed", 1e-4, 1e-2)])
def test_pagerank_solves_to_pagerank_vector(lpmod, oracle_mod, precision, tol, xtol):
    """Solved to rel KKT tol, the point meets the criteria when the oracle
    evaluates it on the original data and lies within xtol (relative, 2-norm)
    of the PageRank vector; FP64 iteration counts stay within 2x of the
    oracle's."""
    say(f"case pagerank solve {precision} tol={tol}")
    data = gen.pagerank_lp(11, 20000)
    xs = pagerank_vector(data)
    p = lpmod.Problem(data, precision=precision)
    info = p.solve(tol, 200000)
    assert info["status"] == "OPTIMAL"
    x, y, lam, _ = p.result()
    o = oracle_mod.Oracle(data)
    ev = o.eval_unscaled(x, y)
    assert ev["rel_kkt"] <= tol * (1 + 1e-6)
    assert np.linalg.norm(x - xs) <= xtol * np.linalg.norm(xs)
    assert x.min() >= 0.0
    if precision == "fp64":
        _, _, _, io = o.solve(tol, 200000)
        assert 0.5 * io["iterations"] <= info["iterations"] <= 2.0 * io["iterations"]


def test_pagerank_full_size(lpmod, oracle_mod):
    """The 1e6-node graph LP (about 8e6 nonzeros, a dense row of 1e6) in the
    layout the benchmark times: scaling, both products on full vectors, and
    lockstep steps across the first check, against the oracle."""
    say("case pagerank full size: generate")
    data = gen.pagerank_lp(1, 1_000_000)
    say("case pagerank full size: load")
    p = lpmod.Problem(data)
    assert (p.layout_split(0), p.layout_split(1)) == (1, 1)
    o = oracle_mod.Oracle(data)
    Dr, Dc = p.scaling()
    Dr_o, Dc_o, _ = o.scaling()
    assert np.max(np.abs(Dr - Dr_o) / Dr_o) < 1e-12
    assert np.max(np.abs(Dc - Dc_o) / Dc_o) < 1e-12
    rng = np.random.default_rng(2)
    for tr, ln in [(False, data.n), (True, data.m)]:
        say(f"case pagerank full size: spmv transpose={tr}")
        v = rng.standard_normal(ln)
        assert_product_close(data, o, p, p.spmv(v, transpose=tr), o.spmv(v, transpose=tr), v, tr)
    for k in [0, 63]:
        say(f"case pagerank full size: lockstep k={k}")
        o.solve(1e-30, k)
        raw = o.get_state_raw()
        prev = o.get_state()
        o.solve(1e-30, k + 1)
        so = o.get_state()
        p.set_state(raw)
        p.solve(1e-30, k + 1)
        sg = gpu_state(lpmod, p)
        assert ints_equal(sg, so), k
        assert_states_close(sg, so, step_condition(prev, so), f"pagerank full k={k}", kkt_scale(so, Dr_o, Dc_o, data))
