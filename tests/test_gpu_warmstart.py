"""The learned warm start: GEMM kernel, network forward/backward/Adam on the
GPU against the FP64 reference network, and what a trained network gains
over the method without it (with the cold solve as fallback)."""
import numpy as np
import pytest

from paper_2312_14832_amd import gen
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    import torch
    assert torch.cuda.is_available()
    from paper_2312_14832_amd import warmstart
    return warmstart


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def cosine(a, b):
    a = np.asarray(a, np.float64).ravel(); b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (100, 70, 45), (3, 130, 300), (257, 65, 1000),
                                   # >= 128 tiles of 128x128: the large-tile MFMA kernel in BF16, with ragged
                                   # M, N, K edges, and an odd leading dimension (per-element staging)
                                   (1030, 2100, 300), (1031, 2049, 301)])
def test_gemm_matches_numpy(ws, precision, ta, tb, M, N, K):
    import torch
    say(f"case gemm {precision} ta={ta} tb={tb} {M}x{N}x{K}")
    g = torch.Generator().manual_seed(M * 7 + N * 3 + K)
    A = torch.randn((K, M) if ta else (M, K), generator=g)
    B = torch.randn((N, K) if tb else (K, N), generator=g)
    dt = torch.bfloat16 if precision == "bf16" else torch.float32
    Ad, Bd = A.to(dt).cuda().contiguous(), B.to(dt).cuda().contiguous()
    Cg = ws.gemm(Ad, Bd, ta, tb, precision).cpu().numpy()
    An = Ad.float().cpu().numpy().astype(np.float64)
    Bn = Bd.float().cpu().numpy().astype(np.float64)
    ref = (An.T if ta else An) @ (Bn.T if tb else Bn)
    # FP32 accumulation of K exactly representable products
    assert rel(Cg, ref) < 1e-5, rel(Cg, ref)


def make_pair(ws, precision, in_dim=16, hidden=32, layers=3, rank=8, out_dim=50, B=12, seed=0):
    import torch
    from oracle.mlp_oracle import MLPRef
    net = ws.Net(out_dim, in_dim=in_dim, hidden=hidden, layers=layers, rank=rank, max_batch=max(B, 16),
                 precision=precision)
    ref = MLPRef(in_dim, hidden, layers, rank, out_dim)
    rng = np.random.default_rng(seed)
    p = net.init_params(seed, out_bias=rng.standard_normal(out_dim))
    mu = rng.standard_normal(in_dim).astype(np.float32) * 0.1
    sig = (1 + rng.random(in_dim)).astype(np.float32)
    net.set_norm(mu, sig)
    X = rng.standard_normal((B, in_dim)).astype(np.float32)
    Zs = rng.standard_normal((B, out_dim)).astype(np.float32)
    return net, ref, p, mu, sig, X, Zs, torch.from_numpy(X).cuda(), torch.from_numpy(Zs).cuda()


def test_forward_and_gradients_fp32(ws):
    net, ref, p, mu, sig, X, Zs, Xd, Zd = make_pair(ws, "fp32")
    Z = net.forward(Xd).cpu().numpy()
    Zr = ref.forward(p, X, mu, sig)[-1]
    assert rel(Z, Zr) < 1e-5
    loss = net.loss_grad(Xd, Zd)
    lr_, gr = ref.loss_grad(p.astype(np.float64), X, Zs, mu, sig)
    assert abs(loss - lr_) <= 1e-5 * lr_
    g = net.grads()
    for off, a, b in ref.shapes:
        assert rel(g[off:off + a * b], gr[off:off + a * b]) < 1e-5, (off, a, b)
        assert rel(g[off + a * b:off + a * b + b], gr[off + a * b:off + a * b + b]) < 1e-5


U_BF16 = 2.0 ** -8


def test_forward_and_gradients_bf16(ws):
    """BF16 operands (unit roundoff 2^-8), FP32 accumulation.  Forward output:
    cosine >= 0.999 and relative error <= 2e-2.  Weight gradients dW = X' dY
    sum over the batch with cancellation, so each is held to the running
    componentwise bound |dW - dW_ref| <= c u |X|'M where M is the magnitude of
    dY propagated back through |W| (M_L = |dZ|, M_(l-1) = (M_l |W_l|') masked
    by the units that may be active within rounding), with c = 4 (L+1): each of the L+1 stages rounds at most an
    operand and a result to bf16 on the forward path and again on the backward
    path; the whole gradient vector also has cosine >= 0.999."""
    net, ref, p, mu, sig, X, Zs, Xd, Zd = make_pair(ws, "bf16", in_dim=64, hidden=128, rank=16, out_dim=300, B=40)
    Z = net.forward(Xd).cpu().numpy()
    Zr = ref.forward(p, X, mu, sig)[-1]
    assert cosine(Z, Zr) >= 0.999 and rel(Z, Zr) <= 2e-2, (cosine(Z, Zr), rel(Z, Zr))
    net.loss_grad(Xd, Zd)
    g = net.grads()
    _, gr = ref.loss_grad(p.astype(np.float64), X, Zs, mu, sig)
    assert cosine(g, gr) >= 0.999
    # forward magnitudes; a ReLU unit whose pre-activation lies within the
    # forward rounding of 0 may switch on either side, so it counts as active
    params = ref.unpack(p.astype(np.float64))
    nl = len(params)
    c = 4.0 * (nl + 1) * U_BF16
    A = [(X.astype(np.float64) - mu) / sig]
    masks = []
    for (W, bvec), r in zip(params, ref.relu):
        z = A[-1] @ W + bvec
        zmag = np.abs(A[-1]) @ np.abs(W) + np.abs(bvec)
        masks.append(z > -c * zmag if r else None)
        A.append(np.maximum(z, 0.0) if r else z)
    Mag = np.abs(2.0 * (A[-1] - Zs) / A[-1].size)
    for li in range(nl - 1, -1, -1):
        off, a, b = ref.shapes[li]
        if masks[li] is not None:
            Mag = Mag * masks[li]
        bound = c * np.abs(A[li]).T @ Mag
        err = np.abs(g[off:off + a * b].reshape(a, b) - gr[off:off + a * b].reshape(a, b))
        assert np.all(err <= bound + 1e-12), (li, float((err / (bound + 1e-30)).max()))
        Mag = Mag @ np.abs(params[li][0]).T


def test_full_size_network_bf16(ws):
    """The configured network (256 -> 3x1024 ReLU -> 64 -> 300000) on 32 rows."""
    say("case full-size network")
    net, ref, p, mu, sig, X, Zs, Xd, Zd = make_pair(ws, "bf16", in_dim=256, hidden=1024, layers=3, rank=64,
                                                     out_dim=300_000, B=32, seed=3)
    Z = net.forward(Xd).cpu().numpy()
    Zr = ref.forward(p, X, mu, sig)[-1]
    assert cosine(Z - p[-300_000:], Zr - p[-300_000:]) >= 0.999
    net.loss_grad(Xd, Zd)
    g = net.grads()
    _, gr = ref.loss_grad(p.astype(np.float64), X, Zs, mu, sig)
    assert cosine(g, gr) >= 0.999


def test_adam_step_matches_reference(ws):
    from oracle.mlp_oracle import MLPRef
    net, ref, p, mu, sig, X, Zs, Xd, Zd = make_pair(ws, "fp32")
    net.train_step(Xd, Zd, 1e-3)
    _, gr = ref.loss_grad(p.astype(np.float64), X, Zs, mu, sig)
    q, _, _ = MLPRef.adam(p.astype(np.float64), gr, np.zeros_like(gr), np.zeros_like(gr), 1, 1e-3)
    # moved entries agree; the first Adam step is ~lr*sign(g), so compare the update
    upd, upd_ref = net.params() - p, q - p
    big = np.abs(gr) > 1e-6 * np.abs(gr).max()
    assert rel(upd[big], upd_ref[big]) < 1e-4


def test_sketch_matches_numpy(ws):
    import torch
    fam_base = gen.parametric_base(5, n=3000, m1=700, m2=800)
    fam = ws.Family(fam_base)
    lps = [gen.parametric_instance(fam_base, 100 + i) for i in range(5)]
    X = fam.sketch(lps).cpu().numpy()
    rp, ci, v = [t.cpu().numpy() for t in fam.S]
    import scipy.sparse as sp
    S = sp.csr_matrix((v.astype(np.float64), ci, rp), shape=(fam.rows, fam.dim))
    D = np.stack([np.concatenate([p.q - fam_base.q, p.c - fam_base.c]) for p in lps]).astype(np.float32)
    ref = (S @ D.astype(np.float64).T).T
    assert rel(X, ref) < 1e-6


def test_trained_network_beats_cold_start(ws):
    """Train on 384 solved members of a small family (targets: the scaled
    solution and the log primal weight of each member's solve), then solve 48
    held-out members to rel KKT 1e-4 from four starts: cold; the base
    solution (the mean training solution) with the default primal weight,
    which is the method without the network; the base solution with the
    family's primal weight (their geometric mean); and the network's
    prediction (point and primal weight).  Every solve ends OPTIMAL, the
    network start takes fewer iterations than the cold and the base-solution
    starts, and a hopeless start falls back to cold."""
    import torch
    base = gen.parametric_base(6, n=2000, m1=500, m2=500, per_col=8)
    fam = ws.Family(base)
    train_lps = [gen.parametric_instance(base, 10_000 + i) for i in range(384)]
    test_lps = [gen.parametric_instance(base, 30_000 + i) for i in range(48)]
    say("case warm start: labels")
    Z, infos = ws.solve_labels(train_lps, tol=1e-5, group=128)
    assert all(i["status"] == "OPTIMAL" for i in infos)
    T = fam.encode(Z, [i["omega"] for i in infos])
    X = fam.sketch(train_lps)
    mu = X.mean(0).cpu().numpy(); sig = X.std(0).cpu().numpy() + 1e-6
    tbase = T.mean(0)
    net = ws.Net(fam.out_dim, hidden=256, layers=3, rank=32, max_batch=128)
    net.init_params(0, out_bias=tbase)
    net.set_norm(mu, sig)
    Td = torch.from_numpy(T).cuda()
    say("case warm start: train")
    losses = ws.train(net, X, Td, epochs=80, batch=128, lr=1e-3)
    say(f"  training loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    assert losses[-1] < 0.8 * losses[0], (losses[0], losses[-1])
    say("case warm start: evaluate")
    pred = net.forward(fam.sketch(test_lps)).cpu().numpy()
    xb, yb, om_fam = fam.decode(tbase)
    zb = Z.mean(0).astype(np.float64)
    assert np.allclose(xb, zb[:base.n], rtol=1e-5, atol=1e-5)
    starts = {"cold": [None] * len(test_lps),
              "base": [(xb, yb, 0.0)] * len(test_lps),
              "base+family omega": [(xb, yb, om_fam)] * len(test_lps),
              "network": [fam.decode(r) for r in pred]}
    res = {k: ws.solve_starts(test_lps, v, tol=1e-4) for k, v in starts.items()}
    mean = {}
    for k, r in res.items():
        assert all(t["status"] == "OPTIMAL" for t in r), k
        mean[k] = float(np.mean([t["iterations"] for t in r]))
    say("  mean iterations: " + ", ".join(f"{k} {v:.0f}" for k, v in mean.items()))
    assert mean["network"] < mean["cold"]
    assert mean["network"] < mean["base"]
    bad = np.full(base.n + base.m, 1e30)
    info, _, fb = ws.solve_with_start(test_lps[0], bad, max_iters=4000)
    assert fb and info["status"] == "OPTIMAL"
