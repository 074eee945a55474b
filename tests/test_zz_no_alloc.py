"""lp_spmv_noalloc, the product entry point that allocates nothing (its
intermediates live in a fixed device array), against lp_spmv on the same
handle: equal bit for bit (same kernels, same layout, same summation order),
on two calls in a row with the second input smaller, in both precisions,
plus the size limit and the wrong-device/NULL errors."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _noalloc_product(lpmod, p, v, transpose):
    import torch
    m, n = p.presolved_size()
    d_in = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    # NaN-filled output: every entry must be written
    d_out = torch.full((n if transpose else m,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    p.spmv_noalloc(d_in, d_out, transpose)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_spmv_on_two_calls(lpmod, precision):
    rng = np.random.default_rng(11)
    # a larger LP (many slices and long rows) and then a smaller one, so the
    # second call reuses the array the first call filled with larger vectors
    big = gen.pagerank_lp(3, 30000)
    small = gen.tiny_lp(2)
    for label, data, kib in (("big", big, 16), ("small", small, 2048)):
        p = lpmod.Problem(data, precision=precision, slice_kib=kib)
        for tr in (False, True):
            say(f"case noalloc {precision} {label} transpose={tr} layout={p.layout()}")
            ln = data.m if tr else data.n
            v = rng.standard_normal(ln)
            if precision == "mixed":
                v = v.astype(np.float32).astype(np.float64)
            want = p.spmv(v, transpose=tr)
            got = _noalloc_product(lpmod, p, v, tr)
            assert np.array_equal(got, want), (label, tr, np.max(np.abs(got - want)))
        p.close()


def test_noalloc_rejects_products_beyond_the_array(lpmod):
    """A product whose partial vectors exceed the 64 MiB array is refused with
    LP_ERR_NOMEM and a message naming the size; the handle keeps working, and
    a smaller handle's call afterwards still matches lp_spmv."""
    import torch
    say("case noalloc size limit")
    data = gen.large_lp(seed=9, n=1_200_000, m1=300_000, m2=300_000)
    p = lpmod.Problem(data, slice_kib=256)
    S_K, S_KT = p.layout()
    need = {False: S_K * data.m * 8, True: S_KT * data.n * 8}
    say(f"  layout {S_K}/{S_KT}, partial bytes K {need[False]}, K' {need[True]}")
    assert max(need.values()) > 64 << 20
    rng = np.random.default_rng(3)
    for tr in (False, True):
        ln, lo = (data.m, data.n) if tr else (data.n, data.m)
        if need[tr] > 64 << 20:
            d_in = torch.zeros(ln, dtype=torch.float64, device="cuda")
            d_out = torch.zeros(lo, dtype=torch.float64, device="cuda")
            with pytest.raises(lpmod.LPError) as e:
                p.spmv_noalloc(d_in, d_out, tr)
            assert e.value.code == -8 and "scratch" in str(e.value), str(e.value)
        else:
            v = rng.standard_normal(ln)
            assert np.array_equal(_noalloc_product(lpmod, p, v, tr), p.spmv(v, transpose=tr))
    v = rng.standard_normal(data.n)
    assert np.isfinite(p.spmv(v)).all()
    p.close()
    small = gen.tiny_lp(4)
    q = lpmod.Problem(small)
    v = rng.standard_normal(small.n)
    assert np.array_equal(_noalloc_product(lpmod, q, v, False), q.spmv(v))
