"""Seeded synthetic LP generators.

Every instance has the form of the paper's primal problem (Sec. 2, eq. (LP)):
``min c'x  s.t.  Ax = b, Gx >= h, l <= x <= u`` with ``K = [A; G]`` stored as
CSR (equality rows first) and ``q = [b; h]``.

Feasibility and boundedness come from a primal/dual certificate built into the
data, not from solving anything:

* a primal point ``x0`` inside the bounds with ``b = A x0`` and
  ``h = G x0 - s`` for a slack ``s >= 0``;
* a dual point ``y0`` (sign-constrained on the ``G`` rows) and a bound
  multiplier ``lam0`` in the cone ``Lambda`` of each variable, with
  ``c = K' y0 + lam0``.

Weak duality then sandwiches the optimum: ``dobj(y0, lam0) <= opt <= c'x0``.

This module only draws random numbers and forms the data.  It holds none of the
solver's arithmetic and is shared by the oracle tests and by the GPU tests and
bench, so both sides see the same bytes.  All generators use
``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp


@dataclass
class LPData:
    """One LP in the paper's stacked form.

    ``row_ptr/col/val`` is the CSR of K (m x n, int32 indices, float64 values),
    ``m1`` the number of equality rows (they come first).  ``l``/``u`` use
    -inf/+inf for absent bounds.  ``x0, y0, lam0, s`` are the certificate.
    """
    m: int
    n: int
    m1: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    c: np.ndarray
    q: np.ndarray
    l: np.ndarray
    u: np.ndarray
    x0: np.ndarray | None = None
    y0: np.ndarray | None = None
    lam0: np.ndarray | None = None
    s: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.m, self.n))


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def _distinct_rows_per_column(rng: np.random.Generator, counts: np.ndarray, m: int):
    """For column j draw ``counts[j]`` distinct rows uniformly from [0, m).

    Returns (rows, cols) as int64 arrays sorted by (col, row).
    Duplicates inside a column are redrawn until none remain.
    """
    n = counts.shape[0]
    if np.any(counts > m):
        raise ValueError("a column asks for more distinct rows than exist")
    cols = np.repeat(np.arange(n, dtype=np.int64), counts)
    rows = rng.integers(0, m, size=cols.shape[0], dtype=np.int64)
    while True:
        key = cols * m + rows
        order = np.argsort(key, kind="stable")
        key = key[order]
        rows = rows[order]
        cols = cols[order]
        dup = np.zeros(key.shape[0], dtype=bool)
        dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            return rows, cols
        rows[dup] = rng.integers(0, m, size=nd, dtype=np.int64)


def _to_csr(rows, cols, vals, m, n):
    """Triplets (no duplicates) -> CSR with columns sorted inside each row."""
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    r = rows[order]
    counts = np.bincount(r, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return (row_ptr.astype(np.int32), cols[order].astype(np.int32),
            np.ascontiguousarray(vals[order], dtype=np.float64))


def _bounds(rng, n, box_hi=10.0):
    """n/2 boxed [0, box_hi], n/4 lower-only [0, inf), the rest free.

    Returns (l, u, kind) with kind 0=boxed, 1=lower-only, 2=free, assigned by
    a seeded permutation.
    """
    perm = rng.permutation(n)
    nb, nl = n // 2, n // 4
    kind = np.empty(n, dtype=np.int8)
    kind[perm[:nb]] = 0
    kind[perm[nb:nb + nl]] = 1
    kind[perm[nb + nl:]] = 2
    l = np.where(kind == 2, -np.inf, 0.0)
    u = np.where(kind == 0, box_hi, np.inf)
    return l, u, kind


def certificate_lp(rng: np.random.Generator, m1: int, m2: int, counts: np.ndarray,
                   value_sampler=None, row_scale_exp: float | None = None,
                   meta: dict | None = None) -> LPData:
    """Random sparse K with the given column counts, plus a certificate.

    Draw order (fixed, part of the recipe): rows per column, values, row
    scales (if any), bound kinds, x0, s, y0, lam0.
    """
    n = counts.shape[0]
    m = m1 + m2
    rows, cols = _distinct_rows_per_column(rng, counts, m)
    vals = rng.standard_normal(rows.shape[0]) if value_sampler is None else value_sampler(rows.shape[0])
    if row_scale_exp is not None:
        rs = 10.0 ** rng.uniform(-row_scale_exp, row_scale_exp, size=m)
        vals = vals * rs[rows]
    row_ptr, col, val = _to_csr(rows, cols, vals, m, n)
    K = sp.csr_matrix((val, col, row_ptr), shape=(m, n))
    l, u, kind = _bounds(rng, n)
    x0 = rng.uniform(0.0, 5.0, size=n)
    s = rng.uniform(0.0, 1.0, size=m2)
    y0 = np.concatenate([rng.standard_normal(m1), rng.uniform(0.0, 1.0, size=m2)])
    g = rng.standard_normal(n)
    lam0 = np.where(kind == 0, g, np.where(kind == 1, np.abs(g), 0.0))
    Kx0 = K @ x0
    q = np.concatenate([Kx0[:m1], Kx0[m1:] - s])
    c = K.T @ y0 + lam0
    return LPData(m=m, n=n, m1=m1, row_ptr=row_ptr, col=col, val=val, c=c, q=q,
                  l=l, u=u, x0=x0, y0=y0, lam0=lam0, s=s, meta=dict(meta or {}))


def power_law_counts(rng, n, kmax=200, exponent=1.534):
    """Column counts on {1..kmax} with P(k) proportional to k^-exponent.

    With kmax=200 and exponent 1.534 the mean is 10 (P(k=1) ~ 0.42).
    """
    k = np.arange(1, kmax + 1, dtype=np.float64)
    p = k ** (-exponent)
    p /= p.sum()
    return rng.choice(kmax, size=n, p=p).astype(np.int64) + 1


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def tiny_lp(seed: int = 0, n: int = 1000, m1: int = 200, m2: int = 300, per_col: int = 5) -> LPData:
    """Tiny random LP: n=1000, m1=200, m2=300, 5 nonzeros per column, N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.full(n, per_col, dtype=np.int64)
    return certificate_lp(rng, m1, m2, counts,
                          meta={"workload": "tiny_random_lp", "seed": seed, "n": n, "m1": m1, "m2": m2})


def large_lp(seed: int = 1, n: int = 2_000_000, m1: int = 500_000, m2: int = 500_000) -> LPData:
    """Large LP: power-law column counts (1..200, mean 10), N(0,1) values times
    10^U(-3,3) per row.  Defaults are the 2e6 x 1e6, ~2e7-nonzero instance;
    the 4e6 x 2e6 mixed-precision instance uses n=4e6, m1=m2=1e6, seed 2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = power_law_counts(rng, n)
    return certificate_lp(rng, m1, m2, counts, row_scale_exp=3.0,
                          meta={"workload": "large_powerlaw_lp", "seed": seed, "n": n, "m1": m1, "m2": m2})


def batch_member(seed: int, n_lo: float = 2e3, n_hi: float = 2e5) -> LPData:
    """One member of the batched workload: n log-uniform in [n_lo, n_hi],
    m = n/2 split 2:3 into equality/inequality rows, 3..8 nonzeros per column."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
    m = max(n // 2, 2)
    m1 = (2 * m) // 5
    m2 = m - m1
    counts = rng.integers(3, 9, size=n).astype(np.int64)
    return certificate_lp(rng, m1, m2, counts,
                          meta={"workload": "batch_member", "seed": seed, "n": n, "m1": m1, "m2": m2})


def box_only_lp(seed: int, n: int = 8) -> LPData:
    """m = 0: min c'x over a box (closed form: each x_j at the bound c_j pushes to)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    l = rng.uniform(-3.0, 0.0, size=n)
    u = l + rng.uniform(0.5, 4.0, size=n)
    c = rng.standard_normal(n)
    return LPData(m=0, n=n, m1=0, row_ptr=np.zeros(1, np.int32), col=np.zeros(0, np.int32),
                  val=np.zeros(0), c=c, q=np.zeros(0), l=l, u=u, meta={"workload": "box_only"})


def dense_small_lp(seed: int, n: int, m1: int, m2: int, density: float = 0.7, box: float = 4.0) -> LPData:
    """Small LP with all variables boxed [0, box] (a bounded polytope), random
    sparse K and a certificate; used for brute-force vertex enumeration."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = m1 + m2
    mask = rng.uniform(size=(m, n)) < density
    for i in range(m):
        if not mask[i].any():
            mask[i, rng.integers(n)] = True
    dense = np.where(mask, rng.standard_normal((m, n)), 0.0)
    rows, cols = np.nonzero(dense)
    row_ptr, col, val = _to_csr(rows.astype(np.int64), cols.astype(np.int64), dense[rows, cols], m, n)
    K = sp.csr_matrix((val, col, row_ptr), shape=(m, n))
    l = np.zeros(n)
    u = np.full(n, box)
    x0 = rng.uniform(0.5, box - 0.5, size=n)
    s = rng.uniform(0.0, 1.0, size=m2)
    y0 = np.concatenate([rng.standard_normal(m1), rng.uniform(0.0, 1.0, size=m2)])
    lam0 = rng.standard_normal(n)
    Kx0 = K @ x0
    q = np.concatenate([Kx0[:m1], Kx0[m1:] - s])
    c = K.T @ y0 + lam0
    return LPData(m=m, n=n, m1=m1, row_ptr=row_ptr, col=col, val=val, c=c, q=q, l=l, u=u,
                  x0=x0, y0=y0, lam0=lam0, s=s, meta={"workload": "dense_small", "seed": seed})


def from_dense(Kd, c, q, l, u, m1) -> LPData:
    """Wrap a small dense problem given by hand."""
    Kd = np.atleast_2d(np.asarray(Kd, dtype=np.float64))
    m, n = Kd.shape
    rows, cols = np.nonzero(Kd)
    row_ptr, col, val = _to_csr(rows.astype(np.int64), cols.astype(np.int64), Kd[rows, cols], m, n)
    return LPData(m=m, n=n, m1=int(m1), row_ptr=row_ptr, col=col, val=val,
                  c=np.asarray(c, np.float64), q=np.asarray(q, np.float64),
                  l=np.asarray(l, np.float64), u=np.asarray(u, np.float64), meta={"workload": "hand"})


# ----------------------------------------------------------------------------
# parametric family for the learned warm start
# ----------------------------------------------------------------------------

def parametric_base(seed: int = 4, n: int = 200_000, m1: int = 50_000, m2: int = 50_000,
                    per_col: int = 10) -> LPData:
    """The fixed-K family's base instance: per_col N(0,1) nonzeros per column
    at distinct uniform rows, with its certificate (x0, s, y0, lam0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.full(n, per_col, dtype=np.int64)
    return certificate_lp(rng, m1, m2, counts,
                          meta={"workload": "parametric_base", "seed": seed, "n": n, "m1": m1, "m2": m2})


def parametric_instance(base: LPData, seed: int, rel: float = 0.1) -> LPData:
    """A member of the family: the base certificate perturbed by rel*N(0,1)
    relative noise and kept valid (x0 clipped into its bounds, slack >= 0,
    inequality duals >= 0, lam0 projected onto each variable's cone), then
    b, h, c rebuilt from it, so every member is feasible and bounded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, m, m1 = base.n, base.m, base.m1
    xi = rng.standard_normal(n)
    x0 = np.clip(base.x0 + rel * base.x0 * xi, base.l, base.u)
    s = np.maximum(base.s * (1.0 + rel * rng.standard_normal(m - m1)), 0.0)
    y0 = base.y0 + rel * np.abs(base.y0) * rng.standard_normal(m)
    y0[m1:] = np.maximum(y0[m1:], 0.0)
    lam = base.lam0 + rel * np.abs(base.lam0) * rng.standard_normal(n)
    fl, fu = np.isfinite(base.l), np.isfinite(base.u)
    lam = np.where(fl & fu, lam, np.where(fl, np.maximum(lam, 0.0), np.where(fu, np.minimum(lam, 0.0), 0.0)))
    K = base.csr()
    Kx0 = K @ x0
    q = np.concatenate([Kx0[:m1], Kx0[m1:] - s])
    c = K.T @ y0 + lam
    return LPData(m=m, n=n, m1=m1, row_ptr=base.row_ptr, col=base.col, val=base.val, c=c, q=q,
                  l=base.l, u=base.u, x0=x0, y0=y0, lam0=lam, s=s,
                  meta={"workload": "parametric_instance", "seed": seed})


def sketch_matrix(dim: int, rows: int = 256, per_col: int = 8, seed: int = 4242):
    """Sparse random sketch S (rows x dim): per_col entries +-1/sqrt(per_col)
    in every column at distinct random rows.  Returned as CSR arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = np.argsort(rng.random((dim, rows)), axis=1)[:, :per_col]          # distinct rows per column
    sign = np.where(rng.random((dim, per_col)) < 0.5, -1.0, 1.0) / np.sqrt(per_col)
    cols = np.repeat(np.arange(dim, dtype=np.int64), per_col)
    rr = r.ravel().astype(np.int64)
    rp, ci, v = _to_csr(rr, cols, sign.ravel(), rows, dim)
    return rp, ci, v.astype(np.float32)


# ----------------------------------------------------------------------------
# PageRank-style LP (a second workload with structured sparsity)
# ----------------------------------------------------------------------------

def pagerank_lp(seed: int, n: int, avg_out: float = 6.0, damping: float = 0.85) -> LPData:
    """LP whose unique feasible point is the PageRank vector of a random graph.

    Graph: node j draws 1 + Poisson(avg_out - 1) links to other nodes, uniformly
    with repeats collapsed (so every node links somewhere); A is its
    column-stochastic transition matrix (A_ij = 1/outdeg_j for each link j -> i).  The LP has n variables x >= 0, zero cost, one
    equality row sum(x) = 1 (row 0) and n inequality rows
    ``x_i - damping * (A x)_i >= (1 - damping)/n``.  Summing the inequality
    rows gives (1 - damping) sum(x) >= 1 - damping, so with sum(x) = 1 every
    row is tight and x is the solution of (I - damping A) x = (1 - damping)/n.
    Shape: m = n + 1, nnz = n (row 0) + n (diagonal) + sum of out-degrees.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if n < 2:
        raise ValueError("pagerank_lp needs n >= 2")
    draws = np.minimum(1 + rng.poisson(avg_out - 1.0, size=n), n - 1)
    src = np.repeat(np.arange(n, dtype=np.int64), draws)
    dst = rng.integers(0, n - 1, size=src.size, dtype=np.int64)
    dst += dst >= src                     # uniform over the other n - 1 nodes
    key = np.unique(src * n + dst)        # repeated links collapse to one
    src, dst = key // n, key % n
    deg = np.bincount(src, minlength=n)   # >= 1: a node's first link is never a repeat
    w = -damping / deg[src]
    rows = np.concatenate([np.zeros(n, np.int64), 1 + np.arange(n, dtype=np.int64), 1 + dst])
    cols = np.concatenate([np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64), src])
    vals = np.concatenate([np.ones(n), np.ones(n), w])
    row_ptr, col, val = _to_csr(rows, cols, vals, n + 1, n)
    q = np.concatenate([[1.0], np.full(n, (1.0 - damping) / n)])
    return LPData(m=n + 1, n=n, m1=1, row_ptr=row_ptr, col=col, val=val, c=np.zeros(n), q=q,
                  l=np.zeros(n), u=np.full(n, np.inf),
                  meta={"workload": "pagerank", "seed": seed, "n": n, "avg_out": avg_out, "damping": damping})


# ----------------------------------------------------------------------------
# LPs without a solution (for infeasibility detection)
# ----------------------------------------------------------------------------

def _with_rows_cols(lp: LPData, K: sp.csr_matrix, m1: int, c, q, l, u, meta) -> LPData:
    K = sp.csr_matrix(K)
    K.sort_indices()
    if K.nnz >= 2**31:
        raise ValueError("nnz does not fit int32")
    return LPData(m=K.shape[0], n=K.shape[1], m1=m1, row_ptr=K.indptr.astype(np.int32),
                  col=K.indices.astype(np.int32), val=np.ascontiguousarray(K.data, dtype=np.float64),
                  c=np.asarray(c, float), q=np.asarray(q, float), l=np.asarray(l, float),
                  u=np.asarray(u, float), meta=meta)


def infeasible_lp(seed: int, kind: str) -> LPData:
    """A tiny random LP made to have no primal-dual solution.

    kind "primal": one more equality row asks the boxed variables ([0, 10])
    of a random set of 20 to sum to 10 * 20 + 5, more than their bounds allow.
    kind "dual": one more variable with cost -1, bounds [0, inf), entering only
    inequality rows, with positive coefficients, so x_new -> inf stays feasible
    and lowers the cost without bound (the base LP is feasible).
    """
    base = tiny_lp(seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    K = base.csr()
    A, G = K[:base.m1], K[base.m1:]
    if kind == "primal":
        boxed = np.flatnonzero(np.isfinite(base.l) & np.isfinite(base.u))
        S = rng.choice(boxed, 20, replace=False)
        row = sp.csr_matrix((np.ones(20), (np.zeros(20, int), S)), shape=(1, base.n))
        K2 = sp.vstack([A, row, G])
        q = np.concatenate([base.q[:base.m1], [float(base.u[S].sum()) + 5.0], base.q[base.m1:]])
        return _with_rows_cols(base, K2, base.m1 + 1, base.c, q, base.l, base.u,
                               {"workload": "infeasible_primal", "seed": seed})
    if kind == "dual":
        rows = rng.choice(G.shape[0], 4, replace=False)
        col = sp.csr_matrix((rng.uniform(0.5, 2.0, 4), (rows, np.zeros(4, int))), shape=(G.shape[0], 1))
        K2 = sp.vstack([sp.hstack([A, sp.csr_matrix((base.m1, 1))]), sp.hstack([G, col])])
        return _with_rows_cols(base, K2, base.m1, np.append(base.c, -1.0), base.q, np.append(base.l, 0.0),
                               np.append(base.u, np.inf), {"workload": "infeasible_dual", "seed": seed})
    raise ValueError(kind)


def presolve_lp(seed: int) -> LPData:
    """The tiny LP with every structure the presolve reduces, kept feasible
    (by its certificate point x0) and bounded: 5 boxed variables fixed at
    x0; 5 singleton equality rows a x_j = a x0_j; 5 singleton inequality rows
    a x_j >= a (x0_j - 0.5) with a > 0 and 3 with a < 0 at x0_j + 0.5; an empty
    equality row (0 = 0) and an empty inequality row (0 >= -1); three empty
    columns (cost 1 on [0, inf), cost -1 on [0, 2], cost 0 and free)."""
    base = tiny_lp(seed)
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    n, m1 = base.n, base.m1
    x0 = base.x0
    K = base.csr()
    l, u, c = base.l.copy(), base.u.copy(), base.c.copy()
    boxed = np.flatnonzero(np.isfinite(l) & np.isfinite(u))
    others = np.flatnonzero(~(np.isfinite(l) & np.isfinite(u)))
    fixed = rng.choice(boxed, 5, replace=False)
    l[fixed] = u[fixed] = x0[fixed]
    pick = rng.choice(others, 13, replace=False)
    eq_cols, ge_cols, le_cols = pick[:5], pick[5:10], pick[10:]
    n2 = n + 3

    def rows(cols, coef):
        return sp.csr_matrix((coef, (np.arange(len(cols)), cols)), shape=(len(cols), n2))

    a_eq = rng.uniform(0.5, 2.0, 5) * rng.choice([-1.0, 1.0], 5)
    a_ge = rng.uniform(0.5, 2.0, 5)
    a_le = -rng.uniform(0.5, 2.0, 3)
    Kw = sp.hstack([K, sp.csr_matrix((base.m, 3))]).tocsr()
    A = sp.vstack([Kw[:m1], rows(eq_cols, a_eq), sp.csr_matrix((1, n2))])
    G = sp.vstack([Kw[m1:], rows(ge_cols, a_ge), rows(le_cols, a_le), sp.csr_matrix((1, n2))])
    q = np.concatenate([base.q[:m1], a_eq * x0[eq_cols], [0.0], base.q[m1:], a_ge * (x0[ge_cols] - 0.5),
                        a_le * (x0[le_cols] + 0.5), [-1.0]])
    c = np.concatenate([c, [1.0, -1.0, 0.0]])
    l = np.concatenate([l, [0.0, 0.0, -np.inf]])
    u = np.concatenate([u, [np.inf, 2.0, np.inf]])
    out = _with_rows_cols(base, sp.vstack([A, G]), m1 + 6, c, q, l, u, {"workload": "presolve_lp", "seed": seed})
    out.x0 = np.concatenate([x0, [0.0, 2.0, 0.0]])
    return out
