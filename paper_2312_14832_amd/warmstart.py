"""Learned warm start for a parametric LP family (fixed K; b, h, c vary).

Thin ctypes binding of the lpw_* entry points (include/lp.h) plus the
pipeline around them: solve a training set with this solver, sketch each
instance's perturbation (dq, dc) to 256 features, train the network on the
GPU with its own kernels, and seed lp_set_start with its prediction.  A warm
solve that ends without OPTIMAL is redone from the cold start (the fallback).

Device memory for the data is torch tensors (plumbing only); every step of
the network and of the solver runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import lp as lpmod

LPW_BF16, LPW_FP32 = 0, 1


class LPWConfig(C.Structure):
    _fields_ = [("in_dim", C.c_int), ("hidden", C.c_int), ("layers", C.c_int), ("rank", C.c_int),
                ("out_dim", C.c_int), ("max_batch", C.c_int), ("precision", C.c_int), ("stream", C.c_void_p)]


_bound = False


def _lib():
    global _bound
    L = lpmod.library()
    if not _bound:
        fp = C.POINTER(C.c_float)
        vp = C.c_void_p
        L.lpw_default_config.argtypes = [C.POINTER(LPWConfig)]
        L.lpw_default_config.restype = None
        L.lpw_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(LPWConfig)]
        L.lpw_param_count.argtypes = [vp]
        L.lpw_param_count.restype = C.c_int64
        L.lpw_set_params.argtypes = [vp, fp]
        L.lpw_get_params.argtypes = [vp, fp]
        L.lpw_set_norm.argtypes = [vp, fp, fp]
        L.lpw_forward.argtypes = [vp, vp, C.c_int, vp]
        L.lpw_loss_grad.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_double)]
        L.lpw_get_grads.argtypes = [vp, fp]
        L.lpw_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        L.lpw_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_float, C.POINTER(C.c_double)]
        L.lpw_gemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int,
                               vp, C.c_int, vp]
        L.lpw_sketch.argtypes = [vp, vp, vp, C.c_int, vp, C.c_int, C.c_int, vp, vp]
        L.lpw_free.argtypes = [vp]
        L.lpw_free.restype = None
        L.lpw_last_error.argtypes = [vp]
        L.lpw_last_error.restype = C.c_char_p
        _bound = True
    return L


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _dev(t):
    """Device pointer of a contiguous float32 (or int32 / bf16-bits) torch tensor."""
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Net:
    """The warm-start network on the GPU (lpw_create ... lpw_free)."""

    def __init__(self, out_dim, in_dim=256, hidden=1024, layers=3, rank=64, max_batch=256, precision="bf16"):
        L = _lib()
        cfg = LPWConfig()
        L.lpw_default_config(C.byref(cfg))
        cfg.in_dim, cfg.hidden, cfg.layers, cfg.rank = in_dim, hidden, layers, rank
        cfg.out_dim, cfg.max_batch = out_dim, max_batch
        cfg.precision = LPW_BF16 if precision == "bf16" else LPW_FP32
        cfg.stream = _stream()
        self.cfg = cfg
        h = C.c_void_p()
        rc = L.lpw_create(C.byref(h), C.byref(cfg))
        if rc != 0:
            raise lpmod.LPError(rc, "lpw_create")
        self.h = h
        self.nparam = L.lpw_param_count(h)
        self.dims = [in_dim] + [hidden] * layers + [rank, out_dim]

    def _check(self, rc):
        if rc != 0:
            raise lpmod.LPError(rc, _lib().lpw_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None:
            _lib().lpw_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def init_params(self, seed=0, out_bias=None):
        """He-uniform ReLU layers, small linear layers, output bias = out_bias."""
        rng = np.random.Generator(np.random.PCG64(seed))
        parts = []
        nl = len(self.dims) - 1
        for li, (a, b) in enumerate(zip(self.dims[:-1], self.dims[1:])):
            lim = np.sqrt(6.0 / a) if li < nl - 2 else np.sqrt(1.0 / a) * 0.1
            parts.append(rng.uniform(-lim, lim, size=a * b))
            bias = np.zeros(b)
            if li == nl - 1 and out_bias is not None:
                bias = np.asarray(out_bias, np.float64)
            parts.append(bias)
        p = np.concatenate(parts).astype(np.float32)
        self.set_params(p)
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.nparam
        self._check(_lib().lpw_set_params(self.h, _fptr(p)))

    def params(self):
        p = np.empty(self.nparam, np.float32)
        self._check(_lib().lpw_get_params(self.h, _fptr(p)))
        return p

    def set_norm(self, mu, sigma):
        mu = np.ascontiguousarray(mu, np.float32)
        sigma = np.ascontiguousarray(sigma, np.float32)
        self._check(_lib().lpw_set_norm(self.h, _fptr(mu), _fptr(sigma)))

    def forward(self, X):
        import torch
        Z = torch.empty((X.shape[0], self.dims[-1]), dtype=torch.float32, device=X.device)
        self._check(_lib().lpw_forward(self.h, _dev(X), X.shape[0], _dev(Z)))
        return Z

    def loss_grad(self, X, Zs):
        loss = C.c_double()
        self._check(_lib().lpw_loss_grad(self.h, _dev(X), _dev(Zs), X.shape[0], C.byref(loss)))
        return loss.value

    def grads(self):
        g = np.empty(self.nparam, np.float32)
        self._check(_lib().lpw_get_grads(self.h, _fptr(g)))
        return g

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(_lib().lpw_adam_step(self.h, lr, beta1, beta2, eps))

    def train_step(self, X, Zs, lr):
        loss = C.c_double()
        self._check(_lib().lpw_train_step(self.h, _dev(X), _dev(Zs), X.shape[0], lr, C.byref(loss)))
        return loss.value


def gemm(A, B, trans_a=False, trans_b=False, precision="bf16"):
    """C = op(A) op(B) with the library's GEMM kernel (torch tensors on the
    GPU; bf16 mode takes torch.bfloat16 inputs)."""
    import torch
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[0] if trans_b else B.shape[1]
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    rc = _lib().lpw_gemm(LPW_BF16 if precision == "bf16" else LPW_FP32, int(trans_a), int(trans_b), M, N, K,
                         _dev(A), A.shape[1], _dev(B), B.shape[1], _dev(Cm), N, _stream())
    if rc != 0:
        raise lpmod.LPError(rc, "lpw_gemm")
    return Cm


class Family:
    """A parametric family: base LP, sketch of the perturbation vectors, the
    scaling of its shared matrix, and the coding of a member's solution as
    the network's output.

    The network's targets are a member's solution in the scaled space the
    method iterates in (x~ = x Dc, y~ = y Dr; the scaling depends on K alone,
    so it is the same for every member) followed by one more coordinate, the
    log of the primal weight the member's solve converged to, times
    sqrt(n + m) so that its squared error weighs about as much as the whole
    solution's in the mean squared error."""

    def __init__(self, base, sketch_rows=256, sketch_seed=4242):
        import torch
        from . import gen
        self.base = base
        self.n, self.m = base.n, base.m
        self.dim = base.m + base.n
        self.out_dim = self.dim + 1
        self.omega_scale = float(np.sqrt(self.dim))
        rp, ci, v = gen.sketch_matrix(self.dim, rows=sketch_rows, seed=sketch_seed)
        self.S = (torch.from_numpy(rp.astype(np.int32)).cuda(), torch.from_numpy(ci.astype(np.int32)).cuda(),
                  torch.from_numpy(v).cuda())
        self.rows = sketch_rows
        self.q0 = base.q.copy()
        self.c0 = base.c.copy()
        p = lpmod.Problem(base)
        self.Dr, self.Dc = p.scaling()
        p.close()

    def encode(self, Z, omegas):
        """[N x (n+m+1)] float32 targets from unscaled solutions Z [N x (n+m)]
        and the primal weights their solves converged to."""
        n = self.n
        T = np.empty((Z.shape[0], self.out_dim), np.float32)
        T[:, :n] = Z[:, :n] * self.Dc
        T[:, n:self.dim] = Z[:, n:] * self.Dr
        T[:, self.dim] = self.omega_scale * np.log(np.asarray(omegas, np.float64))
        return T

    def decode(self, out):
        """(x0, y0, omega) of one output row, unscaled, for lp_set_start."""
        out = np.asarray(out, np.float64)
        n = self.n
        return out[:n] / self.Dc, out[n:self.dim] / self.Dr, float(np.exp(out[self.dim] / self.omega_scale))

    def deltas(self, lps):
        """[B x (m+n)] float32 on the GPU: (q - q_base, c - c_base) per instance."""
        import torch
        D = np.stack([np.concatenate([p.q - self.q0, p.c - self.c0]) for p in lps]).astype(np.float32)
        return torch.from_numpy(D).cuda()

    def sketch(self, lps):
        import torch
        D = self.deltas(lps)
        out = torch.empty((len(lps), self.rows), dtype=torch.float32, device="cuda")
        rp, ci, v = self.S
        rc = _lib().lpw_sketch(_dev(rp), _dev(ci), _dev(v), self.rows, _dev(D), self.dim, len(lps), _dev(out),
                               _stream())
        if rc != 0:
            raise lpmod.LPError(rc, "lpw_sketch")
        return out


def solve_labels(lps, tol=1e-5, group=64, precision="fp64", max_iters=200000, log=None, shared=True):
    """Solve the instances (members of one family: the same K) in groups with
    the shared-matrix batch (one SpMM pass over K per product for the whole
    group; shared=False: the general batch, which reads K once per
    instance); returns (Z [N x (n+m)] float32 numpy of the unscaled
    (x*, y*), list of infos)."""
    Zs, infos = [], []
    for g0 in range(0, len(lps), group):
        part = lps[g0:g0 + group]
        t0 = time.perf_counter()
        bt = lpmod.Shared(part, precision=precision) if shared else lpmod.Batch(part, precision=precision)
        bt.solve(tol, max_iters)
        if log:
            log(f"labels {g0 + len(part)}/{len(lps)} ({time.perf_counter() - t0:.1f}s for this group)")
        for i in range(len(part)):
            x, y, _, info = bt.result(i)
            Zs.append(np.concatenate([x, y]).astype(np.float32))
            infos.append(info)
        bt.close()
    return np.stack(Zs), infos


def train(net, X, Z, epochs=50, batch=256, lr=1e-3, seed=0, log=None):
    """Adam on minibatches of (X, Z) (torch tensors on the GPU)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    N = X.shape[0]
    losses = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, N, batch):
            idx = perm[b0:b0 + batch]
            xb = X.index_select(0, idx).contiguous()
            zb = Z.index_select(0, idx).contiguous()
            tot += net.train_step(xb, zb, lr) * len(idx)
            cnt += len(idx)
        losses.append(tot / cnt)
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {losses[-1]:.6g}")
    return losses


def solve_starts(lps, starts, tol=1e-4, group=128, precision="fp64", max_iters=200000):
    """Solve members of one family with the shared batch, member i from
    starts[i] = None (cold) or (x0, y0, omega) (omega <= 0: the default
    weight); a member whose warm solve does not end OPTIMAL is redone cold
    (the fallback, counted in its iterations).  Returns a list of dicts with
    iterations, status and fallback per member."""
    out = [None] * len(lps)
    for g0 in range(0, len(lps), group):
        idx = list(range(g0, min(g0 + group, len(lps))))
        sh = lpmod.Shared([lps[i] for i in idx], precision=precision)
        for k, i in enumerate(idx):
            if starts[i] is not None:
                x0, y0, om = starts[i]
                sh.set_start(k, x0, y0, om)
        sh.solve(tol, max_iters)
        redo = []
        for k, i in enumerate(idx):
            info = sh.info(k)
            out[i] = {"iterations": info["iterations"], "status": info["status"], "fallback": False}
            if starts[i] is not None and info["status"] != "OPTIMAL":
                redo.append((k, i))
        if redo:
            for k, _ in redo:
                sh.set_start(k, None, None, 0.0)
            sh.solve(tol, max_iters)
            for k, i in redo:
                info = sh.info(k)
                out[i] = {"iterations": out[i]["iterations"] + info["iterations"], "status": info["status"],
                          "fallback": True}
        sh.close()
    return out


def solve_with_start(p, start=None, tol=1e-4, max_iters=200000, precision="fp64", omega=0.0):
    """Solve one instance (optionally warm: start point and, if omega > 0, the
    primal weight); a warm solve that does not end OPTIMAL is redone cold.
    Returns (info, seconds, used_fallback)."""
    prob = lpmod.Problem(p, precision=precision)
    t0 = time.perf_counter()
    if start is not None:
        prob.set_start(start[:p.n], start[p.n:])
        prob.set_start_weight(omega)
    info = prob.solve(tol, max_iters)
    fallback = False
    if start is not None and info["status"] != "OPTIMAL":
        prob.set_start(None, None)
        prob.set_start_weight(0.0)
        info = prob.solve(tol, max_iters)
        fallback = True
    dt = time.perf_counter() - t0
    prob.close()
    return info, dt, fallback
