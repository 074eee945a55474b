// HIP kernels of the restarted-PDHG hot path for gfx950 (MI355X).
//
// One accepted PDHG step (cuPDLP-C paper, Sec. 2, "Restarted PDHG") is the
// pair of sparse products K x' and K' y' with everything elementwise fused
// into their epilogues:
//   k_partial_K + k_dual     : K x', then the dual update
//               y' = proj_Y(y + eta*omega*(q - 2Kx' + Kx)) and the partial
//               sums of the step-size test
//   k_partial_KT + k_update  : K' y' over the CSR of the transpose (so no
//               atomics), step-weighted averages and the next primal trial
//               x'' = proj_X(x' - (eta'/omega)(c - K'y'))
//   k_check_* : every check_every accepted steps, the termination quantities
//               (Sec. 2, "Optimality termination criteria") and KKT_omega
//               (Sec. 2, "Restart criteria") for the current and the averaged
//               iterate, the restart decision, and the restart itself.
// Decisions are taken on the device by single-workgroup kernels that write
// the controller block (Ctl); every kernel reads it at its start, so the
// host only polls a done flag once per window of attempts.
//
// Each product is a column-sliced CSR-Stream pass (see Sliced in internal.h):
// a workgroup stages the products v*x[col] of one row block in LDS with
// coalesced streaming loads, then sums the rows from LDS (one row per thread,
// or split by entries over the threads: Sliced::split); the slice of x it
// gathers from stays resident in its XCD's L2.  The fused epilogue kernels
// add the slices' partial rows in a fixed order.
// Reductions are deterministic: each lane accumulates in FP64, wave64
// butterflies and a fixed-order LDS step give one partial per workgroup, and
// a single workgroup sums the partials in a fixed order.  No float atomics.
#include "device.h"

#include <algorithm>
#include <cmath>

namespace pdlp {

// ----------------------------------------------------------------------------
// the iteration kernels
// ----------------------------------------------------------------------------

// K x' partial products (x' = the primal trial).  LONG (here and below): the
// product has rows cut into chunks; SPLIT: its short-row blocks are summed
// split by entries (Sliced::split).
template <typename T, bool LONG, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_partial_K(Dev<T> d)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done) return;
    sliced_partial<LONG, SPLIT>(d.K, (const T *)pick(d.xb, ctl->cur ^ 1));
}

// K' y' partial products, only after an accepted step
template <typename T, bool LONG, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_partial_KT(Dev<T> d)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done || !ctl->accepted) return;
    sliced_partial<LONG, SPLIT>(d.KT, (const T *)pick(d.yb, ctl->cur));
}

template <typename T, int NS, bool LONG>
__global__ __launch_bounds__(kBlock) void k_dual(Dev<T> d, int vb_m)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done) return;
    const int c = ctl->cur;
    const T sigma = (T)(ctl->eta * ctl->omega);
    DualEpi<T> epi{pick(d.yb, c), pick(d.Kxb, c), d.qs, pick(d.yb, c ^ 1), pick(d.Kxb, c ^ 1), d.m1, sigma, 0.0, 0.0};
    for (int vb = blockIdx.x; vb < vb_m; vb += gridDim.x) {
        const int i = vb * kBlock + (int)threadIdx.x;
        T lt;
        const bool lng = long_row_total<LONG>(d.K, vb, lt);
        if (i < d.m) epi(i, lng ? lt : sum_slices<NS>(d.K, i));
    }
    double v[2] = {epi.dy2, epi.inter};
    block_store_partials<2>(v, d.part_dual);
}

// Adaptive step-size test (PDLP's rule; the paper uses eta without stating
// the rule).  eta_bar = (omega|dx|^2 + |dy|^2/omega) / (2|dy.K dx|).
__global__ __launch_bounds__(kBlock) void k_step_decide(Ctl *ctl, const double *pp, const double *pd, int np)
{
    if (ctl->done) {
        if (threadIdx.x == 0) ctl->mode = MODE_NONE;
        return;
    }
    double a[1], b[2];
    block_sum_partials<1>(pp, np, a);
    block_sum_partials<2>(pd, np, b);
    if (threadIdx.x != 0) return;
    step_decision(ctl, a[0], b[0], b[1]);
}

template <typename T, int NS, bool LONG>
__global__ __launch_bounds__(kBlock) void k_update(Dev<T> d, int vb_n, int vb_m)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done) return;
    const int c = ctl->cur;
    const T tau = (T)(ctl->eta / ctl->omega);
    double dx2 = 0.0;
    if (!ctl->accepted) {
        // rejected attempt: new primal trial from the same point with the smaller step
        for (int vb = blockIdx.x; vb < vb_n; vb += gridDim.x) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) primal_elem(d, c, tau, j, dx2);
        }
    } else {
        UpdateEpi<T> epi{pick(d.xb, c), d.cs, d.ls, d.us, pick(d.KTyb, c), d.xa, d.KTya, pick(d.xb, c ^ 1),
                         (T)ctl->avg_w, tau, ctl->mode == MODE_NONE, 0.0};
        const int total = vb_n + vb_m;
        for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
            if (vb < vb_n) {
                const int j = vb * kBlock + (int)threadIdx.x;
                T lt;
                const bool lng = long_row_total<LONG>(d.KT, vb, lt);
                if (j < d.n) epi(j, lng ? lt : sum_slices<NS>(d.KT, j));
            } else {
                const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
                if (i < d.m) average_row(d, i, c, epi.w);
            }
        }
        dx2 = epi.dx2;
    }
    double v[1] = {dx2};
    block_store_partials<1>(v, d.part_primal);
    if (ctl->mode == MODE_CHECK) {
        // a check follows this step: its sums come from here, not a separate pass
        double cs[kCheckSums];
        check_sums_pass(d, c, vb_n, vb_m, cs);
        block_store_partials<kCheckSums>(cs, d.part_check);
        double rs[kRaySums];
        ray_sums_pass(d, c, vb_n, vb_m, rs);
        block_store_partials<kRaySums>(rs, d.part_ray);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_check_reduce(Dev<T> d, int vb_n, int vb_m)
{
    const Ctl *ctl = d.ctl;
    if (ctl->mode == MODE_NONE || ctl->done) return;
    double s[kCheckSums];
    check_sums_pass(d, ctl->cur, vb_n, vb_m, s);
    block_store_partials<kCheckSums>(s, d.part_check);
    double r[kRaySums];
    ray_sums_pass(d, ctl->cur, vb_n, vb_m, r);
    block_store_partials<kRaySums>(r, d.part_ray);
}

__global__ __launch_bounds__(kBlock) void k_check_decide(Ctl *ctl, const double *part, const double *pray, int np,
                                                         double Nq, double Nc)
{
    if (ctl->mode == MODE_NONE || ctl->done) return;
    double S[kCheckSums], R[kRaySums];
    block_sum_partials<kCheckSums>(part, np, S);
    block_sum_partials<kRaySums>(pray, np, R);
    if (threadIdx.x != 0) return;
    check_decision(ctl, S, R, Nq, Nc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_check_apply(Dev<T> d, int vb_n, int vb_m)
{
    const Ctl *ctl = d.ctl;
    if (ctl->mode == MODE_NONE) return;
    const int c = ctl->cur, rt = ctl->restart_to, co = ctl->copy_out, sel = ctl->out_sel;
    const int np = ctl->need_primal;
    const T tau = (T)(ctl->eta / ctl->omega);
    double dx2 = 0.0;
    for (int vb = blockIdx.x; vb < vb_n + vb_m; vb += gridDim.x) {
        if (vb < vb_n) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) apply_col(d, j, c, rt, co, sel, np, tau, dx2);
        } else {
            const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
            if (i < d.m) apply_row(d, i, c, rt, co, sel);
        }
    }
    double v[1] = {dx2};
    block_store_partials<1>(v, d.part_primal);
}

// Mixed precision's FP64 re-check: out = K~ x with the FP64 scaled matrix
// in plain CSR and an iterate of either precision, a wavefront per row
// (lanes striding, FP64 accumulation, a butterfly combining them).
template <typename TX>
__global__ __launch_bounds__(kBlock) void k_csr64(const int *__restrict__ rp, const int *__restrict__ ci,
                                                  const double *__restrict__ v, const TX *__restrict__ x,
                                                  double *__restrict__ out, int rows)
{
    const int lane = (int)threadIdx.x & 63;
    const int nw = (int)(gridDim.x * kBlock) >> 6;
    for (int r = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6); r < rows; r += nw) {
        double acc = 0.0;
        const int e = rp[r + 1];
        for (int p = rp[r] + lane; p < e; p += 64) acc += v[p] * (double)x[ci[p]];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) out[r] = acc;
    }
}

// The 9 check sums of one iterate (same order as row_sums / col_sums) with
// FP64 products and the FP64 scaled data c~, l~, u~, q~ in place of their
// FP32 copies.
template <typename T>
__device__ __forceinline__ void conf_row(const Conf64 &cf, const double *Dr, int i, int m1, const T *y, const T *y0,
                                         const double *kx, double *s)
{
    const double k = kx[i], q = cf.qs[i];
    double r = k - q;
    if (i >= m1) {
        const double t = q - k;
        r = t > 0.0 ? t : 0.0;
    }
    const double ru = r * Dr[i];
    s[0] += ru * ru;
    s[1] += r * r;
    const double yi = (double)y[i];
    s[2] += q * yi;
    const double dd = yi - (double)y0[i];
    s[3] += dd * dd;
}

template <typename T>
__device__ __forceinline__ void conf_col(const Conf64 &cf, const double *Dc, int j, const T *x, const T *x0,
                                         const double *kty, double *s)
{
    const double cj = cf.cs[j], lj = cf.ls[j], uj = cf.us[j];
    const bool lf = isfinite(lj), uf = isfinite(uj);
    const double g = cj - kty[j];
    const double lam = proj_lambda(g, lf, uf);
    const double rd = g - lam;
    const double rdu = rd * Dc[j];
    s[4] += rdu * rdu;
    s[5] += rd * rd;
    const double xj = (double)x[j];
    s[6] += cj * xj;
    double b = 0.0;
    if (lf && lam > 0.0) b += lj * lam;
    if (uf && lam < 0.0) b += uj * lam;
    s[7] += b;
    const double dd = xj - (double)x0[j];
    s[8] += dd * dd;
}

// The 18 check sums of the current iterate (buffer cur) and the average,
// all in FP64 (products, data, accumulation) from the stored iterates.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_confirm_sums(Dev<T> d, Conf64 cf, int cur, int vb_n, int vb_m)
{
    const T *x = pick(d.xb, cur), *y = pick(d.yb, cur);
    double s[kCheckSums];
#pragma unroll
    for (int i = 0; i < kCheckSums; ++i) s[i] = 0.0;
    for (int vb = blockIdx.x; vb < vb_n + vb_m; vb += gridDim.x) {
        if (vb < vb_n) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) {
                conf_col(cf, d.Dc, j, x, (const T *)d.x0, cf.kty[0], s);
                conf_col(cf, d.Dc, j, (const T *)d.xa, (const T *)d.x0, cf.kty[1], s + 9);
            }
        } else {
            const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
            if (i < d.m) {
                conf_row(cf, d.Dr, i, d.m1, y, (const T *)d.y0, cf.kx[0], s);
                conf_row(cf, d.Dr, i, d.m1, (const T *)d.ya, (const T *)d.y0, cf.kx[1], s + 9);
            }
        }
    }
    block_store_partials<kCheckSums>(s, cf.part);
}

__global__ __launch_bounds__(kBlock) void k_confirm_decide(Ctl *ctl, const double *part, int np, double Nq, double Nc)
{
    double S[kCheckSums];
    block_sum_partials<kCheckSums>(part, np, S);
    if (threadIdx.x != 0) return;
    confirm_decision(ctl, S, Nq, Nc);
}

// ----------------------------------------------------------------------------
// the whole loop of a small LP in one workgroup
// ----------------------------------------------------------------------------

// Sum NV values over the kSmall threads of the workgroup in a fixed order
// (wavefront butterflies, then the wavefronts in index order); every thread
// gets the totals.  Every thread must call it.
template <int NV, int NT = kSmall>
__device__ __forceinline__ void small_sum(double (&v)[NV], double (*sh)[kCheckSums])
{
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double a = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        v[i] = a;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wave][i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = sh[0][i];
        for (int w = 1; w < NT / 64; ++w) t += sh[w][i];
        v[i] = t;
    }
    __syncthreads();
}

// small_sum with a single barrier: every thread gets the totals, and the
// caller must pass another barrier before the next small_sum or
// small_sum_once writes sh.
template <int NV, int NT>
__device__ __forceinline__ void small_sum_once(double (&v)[NV], double (*sh)[kCheckSums])
{
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double a = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        v[i] = a;
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wave][i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = sh[0][i];
        for (int w = 1; w < NT / 64; ++w) t += sh[w][i];
        v[i] = t;
    }
}

// The decisions outside the loop body's register allocation: inlined, their
// math calls would make the whole kernel spill.  Only thread 0 calls them.
__device__ __noinline__ void small_step_decision(Ctl *c, double dx2, double dy2, double inter)
{
    step_decision(c, dx2, dy2, inter);
}

__device__ __noinline__ void small_check_decision(Ctl *c, const double *S, const double *R, double Nq, double Nc)
{
    check_decision(c, S, R, Nq, Nc);
}

// row r of a plain CSR (rp, ci, v) against x, entries in order; eight at a
// time in straight-line phases so their loads overlap (slots past the row's
// end re-read its last entry and are masked out of the sum)
template <typename T, int U = 8>
__device__ __forceinline__ T small_row(const int *__restrict__ rp, const int *__restrict__ ci,
                                       const T *__restrict__ v, const T *__restrict__ x, int r)
{
    const int e = rp[r + 1];
    T acc = T(0);
    for (int p = rp[r]; p < e; p += U) {
        int c[U];
        T a[U], g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(p + u, e - 1);
            c[u] = ci[t];
            a[u] = v[t];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p + u < e) acc += a[u] * g[u];
    }
    return acc;
}

// Attempt slots of a small LP (both products one column slice, no long rows)
// run by one workgroup until the LP is done or max_slots slots have passed.
// Each slot is the multi-kernel slot's steps in order (K x' and the dual
// step, the step decision, K'y' with the averages and next primal trial or
// the new trial after a rejection, and at a check its sums, decision and
// restart / output bookkeeping), with workgroup barriers in place of kernel
// boundaries and the controller in LDS.  STAGE: K, K' and the vectors the
// products gather (the primal trial x', the dual trial y') are kept in LDS,
// so the products never leave the CU; every value written to a trial vector
// goes to its LDS copy too.  |x' - x|^2 of the pending trial is recomputed
// from the stored buffers at entry.
template <typename T, bool STAGE>
__global__ __launch_bounds__(kSmall) void k_small_loop(Dev<T> d, int max_slots, double Nq, double Nc)
{
    extern __shared__ double dyn[];
    __shared__ Ctl sc;
    __shared__ double sh[kSmall / 64][kCheckSums];
    const int tid = (int)threadIdx.x;
    const int nk = d.K.rp[d.m], nt = d.KT.rp[d.n];
    const int *krp = d.K.rp, *kci = d.K.ci, *trp = d.KT.rp, *tci = d.KT.ci;
    const T *kv = d.K.v, *tv = d.KT.v;
    T *sx = nullptr, *sy = nullptr;
    if constexpr (STAGE) {
        T *tb = reinterpret_cast<T *>(dyn);
        T *skv = tb, *stv = skv + nk;
        sx = stv + nt;
        sy = sx + d.n;
        int *ib = reinterpret_cast<int *>(sy + d.m);
        int *skrp = ib, *skci = skrp + d.m + 1, *strp = skci + nk, *stci = strp + d.n + 1;
        for (int t = tid; t < nk; t += kSmall) {
            skv[t] = kv[t];
            skci[t] = kci[t];
        }
        for (int t = tid; t < nt; t += kSmall) {
            stv[t] = tv[t];
            stci[t] = tci[t];
        }
        for (int t = tid; t <= d.m; t += kSmall) skrp[t] = krp[t];
        for (int t = tid; t <= d.n; t += kSmall) strp[t] = trp[t];
        krp = skrp; kci = skci; kv = skv;
        trp = strp; tci = stci; tv = stv;
    }
    if (tid == 0) sc = *d.ctl;
    __syncthreads();
    double dx2 = 0.0;
    {
        const T *x = pick(d.xb, sc.cur), *xt = pick(d.xb, sc.cur ^ 1);
        for (int j = tid; j < d.n; j += kSmall) {
            const T v = xt[j];
            if constexpr (STAGE) sx[j] = v;
            const double dd = (double)v - (double)x[j];
            dx2 += dd * dd;
        }
    }
    __syncthreads();
    for (int slot = 0; slot < max_slots; ++slot) {
        if (sc.done) break;   // the same LDS value for every thread
        {
            // K x' and the dual step (the arithmetic of DualEpi)
            const int c = sc.cur;
            const T *xg = STAGE ? (const T *)sx : (const T *)pick(d.xb, c ^ 1);
            const T *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
            T *yn = pick(d.yb, c ^ 1), *kxn = pick(d.Kxb, c ^ 1);
            const T sigma = (T)(sc.eta * sc.omega);
            double v[3] = {dx2, 0.0, 0.0};
            for (int i = tid; i < d.m; i += kSmall) {
                const T yo = y[i], ko = kx[i], qi = d.qs[i];
                const T s = small_row(krp, kci, kv, xg, i);
                T val = yo + sigma * (qi - T(2) * s + ko);
                if (i >= d.m1 && val < T(0)) val = T(0);
                yn[i] = val;
                kxn[i] = s;
                if constexpr (STAGE) sy[i] = val;
                const double dd = (double)val - (double)yo;
                v[1] += dd * dd;
                v[2] += dd * ((double)s - (double)ko);
            }
            small_sum<3>(v, sh);
            if (tid == 0) small_step_decision(&sc, v[0], v[1], v[2]);
            __syncthreads();
        }
        {
            const int c = sc.cur;
            const T tau = (T)(sc.eta / sc.omega);
            T *xn = pick(d.xb, c ^ 1);
            const T *x = pick(d.xb, c);
            dx2 = 0.0;
            if (!sc.accepted) {
                // a new primal trial from the same point with the smaller step
                for (int j = tid; j < d.n; j += kSmall) {
                    const T xj = x[j];
                    const T nv = clampv(xj - tau * (d.cs[j] - pick(d.KTyb, c)[j]), d.ls[j], d.us[j]);
                    xn[j] = nv;
                    if constexpr (STAGE) sx[j] = nv;
                    const double dd = (double)nv - (double)xj;
                    dx2 += dd * dd;
                }
            } else {
                // K'y', the averages and the next primal trial (the arithmetic of UpdateEpi)
                const T *yg = STAGE ? (const T *)sy : (const T *)pick(d.yb, c);
                T *kty = pick(d.KTyb, c);
                const T w = (T)sc.avg_w;
                const bool primal = sc.mode == MODE_NONE;
                for (int j = tid; j < d.n; j += kSmall) {
                    const T xj = x[j], a = d.xa[j], b = d.KTya[j];
                    const T s = small_row(trp, tci, tv, yg, j);
                    kty[j] = s;
                    d.xa[j] = a + w * (xj - a);
                    d.KTya[j] = b + w * (s - b);
                    if (primal) {
                        const T nv = clampv(xj - tau * (d.cs[j] - s), d.ls[j], d.us[j]);
                        xn[j] = nv;
                        if constexpr (STAGE) sx[j] = nv;
                        const double dd = (double)nv - (double)xj;
                        dx2 += dd * dd;
                    }
                }
                for (int i = tid; i < d.m; i += kSmall) average_row(d, i, c, w);
            }
            __syncthreads();
        }
        if (sc.mode != MODE_NONE) {
            const int c = sc.cur;
            double cs[kCheckSums], rs[kRaySums];
            const T *x = pick(d.xb, c), *kty = pick(d.KTyb, c), *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
#pragma unroll
            for (int k = 0; k < kCheckSums; ++k) cs[k] = 0.0;
#pragma unroll
            for (int k = 0; k < kRaySums; ++k) rs[k] = 0.0;
            for (int j = tid; j < d.n; j += kSmall) {
                col_sums(d, j, x, kty, cs);
                col_sums(d, j, (const T *)d.xa, (const T *)d.KTya, cs + 9);
                ray_col_sums(d, j, x, kty, rs);
            }
            for (int i = tid; i < d.m; i += kSmall) {
                row_sums(d, i, d.m1, y, kx, cs);
                row_sums(d, i, d.m1, (const T *)d.ya, (const T *)d.Kxa, cs + 9);
                ray_row_sums(d, i, d.m1, y, kx, rs);
            }
            small_sum<kCheckSums>(cs, sh);
            small_sum<kRaySums>(rs, sh);
            if (tid == 0) small_check_decision(&sc, cs, rs, Nq, Nc);
            __syncthreads();
            const int rt = sc.restart_to, co = sc.copy_out, sel = sc.out_sel, np = sc.need_primal;
            const T tau = (T)(sc.eta / sc.omega);
            dx2 = 0.0;
            for (int j = tid; j < d.n; j += kSmall) {
                apply_col(d, j, c, rt, co, sel, np, tau, dx2);
                // each thread re-reads only the trial entries it wrote itself
                if constexpr (STAGE) {
                    if (np) sx[j] = pick(d.xb, c ^ 1)[j];
                }
            }
            for (int i = tid; i < d.m; i += kSmall) apply_row(d, i, c, rt, co, sel);
            __syncthreads();
        }
    }
    if (tid == 0) *d.ctl = sc;
}

// The one-workgroup loop for LPs with at most R * kSmallReg rows and
// columns, K and K' staged in LDS as above: thread t owns columns and rows
// t + r kSmallReg (r < R), and every vector entry of them (current point,
// primal trial, K'y and K x, the averages, the data) stays in its registers
// for the whole launch; they are loaded at entry and stored back at exit in
// the layout of the multi-kernel path (the current buffer and the pending
// primal trial).  The anchor and the scaling factors, read only at checks,
// stay in memory.  Only the two trial vectors the products gather go
// through LDS.  The arithmetic is that of the element functions: the dual
// step of DualEpi, the averages and trial of UpdateEpi and primal_elem, the
// sums of row_sums_v / col_sums_v / ray_*_v, the bookkeeping of apply_col /
// apply_row.  The step rule's two factors for the accepted counts this
// launch can reach (at most max_slots of them) are tabulated in LDS at
// entry, so the per-slot step decision is plain arithmetic, which every
// thread takes for itself while thread 0 alone updates the controller.
// kSmallReg threads (fewer than the other forms) leave each thread enough
// registers to hold its R columns and rows without spilling.  The body is
// shared by the single-LP kernel and the batched one (a workgroup per LP).
template <typename T, int R>
__device__ __forceinline__ void small_reg_body(const Dev<T> &d, int max_slots, double Nq, double Nc)
{
    constexpr int NT = kSmallReg;
    extern __shared__ double dyn[];
    __shared__ Ctl sc;
    __shared__ double sh[NT / 64][kCheckSums];
    const int tid = (int)threadIdx.x;
    const int nk = d.K.rp[d.m], nt = d.KT.rp[d.n];
    T *skv = reinterpret_cast<T *>(dyn), *stv = skv + nk;
    T *sx = stv + nt, *sy = sx + d.n;
    int *skrp = reinterpret_cast<int *>(sy + d.m), *skci = skrp + d.m + 1, *strp = skci + nk, *stci = strp + d.n + 1;
    double *tab = dyn + (small_stage_bytes<T>(d.m, d.n, nk, nt) + 7) / 8;   // [max_slots][2]
    for (int t = tid; t < nk; t += NT) {
        skv[t] = d.K.v[t];
        skci[t] = d.K.ci[t];
    }
    for (int t = tid; t < nt; t += NT) {
        stv[t] = d.KT.v[t];
        stci[t] = d.KT.ci[t];
    }
    for (int t = tid; t <= d.m; t += NT) skrp[t] = d.K.rp[t];
    for (int t = tid; t <= d.n; t += NT) strp[t] = d.KT.rp[t];
    if (tid == 0) sc = *d.ctl;
    __syncthreads();
    const long long k0 = sc.k;
    const int sc_fixed = sc.fixed_step, sc_every = sc.check_every;   // fixed for the launch
    const long long sc_maxit = sc.max_iters;
    for (int t = tid; t < max_slots; t += NT) step_factors(k0 + t, tab[2 * t], tab[2 * t + 1]);
    // columns j = tid + r NT, rows i = tid + r NT
    T xc[R], xt[R], ktc[R], xa[R], kta[R], cj[R], lj[R], uj[R];
    T yc[R], kxc[R], ya[R], kxa[R], qi[R], yt[R], kxt[R];
    double dx2 = 0.0;
    {
        const int c = sc.cur;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = tid + r * NT, i = j;
            xc[r] = xt[r] = ktc[r] = xa[r] = kta[r] = cj[r] = lj[r] = uj[r] = T(0);
            yc[r] = kxc[r] = ya[r] = kxa[r] = qi[r] = yt[r] = kxt[r] = T(0);
            if (j < d.n) {
                xc[r] = pick(d.xb, c)[j];
                xt[r] = pick(d.xb, c ^ 1)[j];
                ktc[r] = pick(d.KTyb, c)[j];
                xa[r] = d.xa[j]; kta[r] = d.KTya[j];
                cj[r] = d.cs[j]; lj[r] = d.ls[j]; uj[r] = d.us[j];
                sx[j] = xt[r];
                const double dd = (double)xt[r] - (double)xc[r];
                dx2 += dd * dd;
            }
            if (i < d.m) {
                yc[r] = pick(d.yb, c)[i];
                kxc[r] = pick(d.Kxb, c)[i];
                ya[r] = d.ya[i]; kxa[r] = d.Kxa[i];
                qi[r] = d.qs[i];
            }
        }
    }
    __syncthreads();
    for (int slot = 0; slot < max_slots; ++slot) {
        if (sc.done) break;   // the same LDS value for every thread
        // the controller fields the step decision reads, taken before the
        // barrier after which thread 0 updates the controller
        const double eta = sc.eta, omega = sc.omega, W = sc.W;
        const long long kk = sc.k;
        int accepted, mode;
        double eta_next, avg_w = 0.0;
        {
            // K x' and the dual step
            const T sigma = (T)(eta * omega);
            double v[3] = {dx2, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = tid + r * NT;
                if (i < d.m) {
                    const T s = small_row<T, 4>(skrp, skci, skv, (const T *)sx, i);
                    T val = yc[r] + sigma * (qi[r] - T(2) * s + kxc[r]);
                    if (i >= d.m1 && val < T(0)) val = T(0);
                    yt[r] = val;
                    kxt[r] = s;
                    sy[i] = val;
                    const double dd = (double)val - (double)yc[r];
                    v[1] += dd * dd;
                    v[2] += dd * ((double)s - (double)kxc[r]);
                }
            }
            small_sum_once<3, NT>(v, sh);
            // every thread takes the step decision (the same arithmetic as
            // thread 0's update of the controller, so no barrier is needed
            // before the results are used)
            const int at = (int)(kk - k0);   // < max_slots: one accepted step per slot at most
            const int rule = step_rule(eta, omega, sc_fixed, v[0], v[1], v[2], tab[2 * at], tab[2 * at + 1], eta_next);
            accepted = rule == 1;
            mode = rule < 0 ? MODE_CHECK : (rule == 1 ? mode_after_accept(kk + 1, sc_every, sc_maxit) : MODE_NONE);
            if (rule < 0) eta_next = eta;
            if (rule == 1) avg_w = eta / (W + eta);
            if (tid == 0) step_decision_f(&sc, v[0], v[1], v[2], tab[2 * at], tab[2 * at + 1]);
        }
        {
            const T tau = (T)(eta_next / omega);
            dx2 = 0.0;
            if (!accepted) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int j = tid + r * NT;
                    if (j < d.n) {
                        const T nv = clampv(xc[r] - tau * (cj[r] - ktc[r]), lj[r], uj[r]);
                        xt[r] = nv;
                        sx[j] = nv;
                        const double dd = (double)nv - (double)xc[r];
                        dx2 += dd * dd;
                    }
                }
            } else {
                // the trials become the current point; K'y', averages, next trial
                const T w = (T)avg_w;
                const bool primal = mode == MODE_NONE;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = tid + r * NT, j = i;
                    if (i < d.m) {
                        yc[r] = yt[r];
                        kxc[r] = kxt[r];
                        ya[r] = ya[r] + w * (yc[r] - ya[r]);
                        kxa[r] = kxa[r] + w * (kxc[r] - kxa[r]);
                    }
                    if (j < d.n) {
                        xc[r] = xt[r];
                        const T s = small_row<T, 4>(strp, stci, stv, (const T *)sy, j);
                        ktc[r] = s;
                        xa[r] = xa[r] + w * (xc[r] - xa[r]);
                        kta[r] = kta[r] + w * (s - kta[r]);
                        if (primal) {
                            const T nv = clampv(xc[r] - tau * (cj[r] - s), lj[r], uj[r]);
                            xt[r] = nv;
                            sx[j] = nv;
                            const double dd = (double)nv - (double)xc[r];
                            dx2 += dd * dd;
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (sc.mode != MODE_NONE) {
            double cs[kCheckSums], rs[kRaySums];
#pragma unroll
            for (int k = 0; k < kCheckSums; ++k) cs[k] = 0.0;
#pragma unroll
            for (int k = 0; k < kRaySums; ++k) rs[k] = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = tid + r * NT, j = i;
                if (j < d.n) {
                    const double x0 = (double)d.x0[j], kt0 = (double)d.KTy0[j], Dcj = d.Dc[j];
                    col_sums_v((double)cj[r], (double)lj[r], (double)uj[r], Dcj, (double)ktc[r], (double)xc[r], x0,
                               cs);
                    col_sums_v((double)cj[r], (double)lj[r], (double)uj[r], Dcj, (double)kta[r], (double)xa[r], x0,
                               cs + 9);
                    ray_col_sums_v((double)cj[r], (double)lj[r], (double)uj[r], Dcj, (double)xc[r], x0,
                                   (double)ktc[r], kt0, rs);
                }
                if (i < d.m) {
                    const double y0 = (double)d.y0[i], kx0 = (double)d.Kx0[i], Dri = d.Dr[i];
                    const bool ineq = i >= d.m1;
                    row_sums_v((double)kxc[r], (double)qi[r], Dri, (double)yc[r], y0, ineq, cs);
                    row_sums_v((double)kxa[r], (double)qi[r], Dri, (double)ya[r], y0, ineq, cs + 9);
                    ray_row_sums_v((double)kxc[r], kx0, Dri, (double)yc[r], y0, (double)qi[r], ineq, rs);
                }
            }
            small_sum<kCheckSums, NT>(cs, sh);
            small_sum<kRaySums, NT>(rs, sh);
            if (tid == 0) small_check_decision(&sc, cs, rs, Nq, Nc);
            __syncthreads();
            const int rt = sc.restart_to, co = sc.copy_out, sel = sc.out_sel, np = sc.need_primal;
            const T tau = (T)(sc.eta / sc.omega);
            dx2 = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = tid + r * NT, j = i;
                if (j < d.n) {
                    if (co) {
                        if (sel == 2) {
                            d.xo[j] = xc[r] - d.x0[j];
                            d.KTyo[j] = cj[r] + (ktc[r] - d.KTy0[j]);
                        } else {
                            d.xo[j] = sel ? xa[r] : xc[r];
                            d.KTyo[j] = sel ? kta[r] : ktc[r];
                        }
                    }
                    if (rt == 2) {
                        xc[r] = xa[r];
                        ktc[r] = kta[r];
                        d.x0[j] = xa[r];
                        d.KTy0[j] = kta[r];
                    } else if (rt == 1) {
                        xa[r] = xc[r];
                        kta[r] = ktc[r];
                        d.x0[j] = xc[r];
                        d.KTy0[j] = ktc[r];
                    }
                    if (np) {
                        const T nv = clampv(xc[r] - tau * (cj[r] - ktc[r]), lj[r], uj[r]);
                        xt[r] = nv;
                        sx[j] = nv;
                        const double dd = (double)nv - (double)xc[r];
                        dx2 += dd * dd;
                    }
                }
                if (i < d.m) {
                    if (co) d.yo[i] = sel == 2 ? yc[r] - d.y0[i] : (sel ? ya[r] : yc[r]);
                    if (rt == 2) {
                        yc[r] = ya[r];
                        kxc[r] = kxa[r];
                        d.y0[i] = ya[r];
                        d.Kx0[i] = kxa[r];
                    } else if (rt == 1) {
                        ya[r] = yc[r];
                        kxa[r] = kxc[r];
                        d.y0[i] = yc[r];
                        d.Kx0[i] = kxc[r];
                    }
                }
            }
            __syncthreads();
        }
    }
    // back to the buffers of the multi-kernel path
    const int c = sc.cur;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = tid + r * NT, j = i;
        if (j < d.n) {
            pick(d.xb, c)[j] = xc[r];
            pick(d.xb, c ^ 1)[j] = xt[r];
            pick(d.KTyb, c)[j] = ktc[r];
            d.xa[j] = xa[r];
            d.KTya[j] = kta[r];
        }
        if (i < d.m) {
            pick(d.yb, c)[i] = yc[r];
            pick(d.Kxb, c)[i] = kxc[r];
            d.ya[i] = ya[r];
            d.Kxa[i] = kxa[r];
        }
    }
    if (tid == 0) *d.ctl = sc;
}

template <typename T, int R>
__global__ __launch_bounds__(kSmallReg) void k_small_reg(Dev<T> d, int max_slots, double Nq, double Nc)
{
    small_reg_body<T, R>(d, max_slots, Nq, Nc);
}

// Many small LPs, workgroup b on LP b: devs[b] is LP b's view of a batch
// (its vectors, its own plain CSR of K and K', its controller), nq / nc its
// norms; every LP runs until it is done or max_slots slots have passed.
template <typename T, int R>
__global__ __launch_bounds__(kSmallReg) void k_small_reg_batch(const Dev<T> *__restrict__ devs,
                                                               const double *__restrict__ nq,
                                                               const double *__restrict__ nc, int max_slots)
{
    small_reg_body<T, R>(devs[blockIdx.x], max_slots, nq[blockIdx.x], nc[blockIdx.x]);
}

// Gather-rate probe (a measurement helper, not a step of the method): the
// access pattern of a sliced product's gathers without its matrix.  Indices
// are slice-major, count / S per slice, local to the slice; workgroup b
// works on slice b % S (so a slice stays on the XCDs congruent to it, as in
// the products) and walks that slice's chunks of 2048 indices; each thread
// loads 8 indices, then makes their 8 gathers, then adds them, the same
// three phases as a row block.  One sum per thread is stored.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_probe(const int *__restrict__ idx, const T *__restrict__ x,
                                                         int64_t per_slice, int S, int64_t slice_len,
                                                         T *__restrict__ out)
{
    constexpr int U = kStreamNB / kBlock;
    const int s = (int)blockIdx.x % S;
    const int64_t chunks = (per_slice + kStreamNB - 1) / kStreamNB;
    const int *ix = idx + (size_t)s * per_slice;
    const T *xs = x + (size_t)s * slice_len;
    T acc = T(0);
    for (int64_t k = (int64_t)blockIdx.x / S; k < chunks; k += (int64_t)gridDim.x / S) {
        const int64_t b0 = k * kStreamNB;
        const int cnt = (int)(per_slice - b0 < kStreamNB ? per_slice - b0 : kStreamNB);
        int c[U];
        T g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = __builtin_nontemporal_load(ix + b0 + min((int)threadIdx.x + u * kBlock, cnt - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = xs[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if ((int)threadIdx.x + u * kBlock < cnt) acc += g[u];
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = acc;
}

template <typename T, bool LONG, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_partial_plain(Sliced<T> P, const T *__restrict__ x)
{
    sliced_partial<LONG, SPLIT>(P, x);
}

template <typename T, bool LONG>
__global__ __launch_bounds__(kBlock) void k_sum_slices(Sliced<T> P, T *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    T lt;
    const bool lng = long_row_total<LONG>(P, (int)blockIdx.x, lt);
    if (i < P.rows) out[i] = lng ? lt : sum_slices<0>(P, i);
}

// values into the sliced layout: dst[p] = src_vals[src_pos[p]]
template <typename T>
__global__ void k_gather_values(const double *__restrict__ src_vals, const int *__restrict__ src_pos,
                                T *__restrict__ dst, int64_t len)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) dst[i] = (T)src_vals[src_pos[i]];
}

// start point: x = proj_X(x_start * Dc), y = proj_Y(y_start * Dr) (0 when absent)
template <typename T>
__global__ void k_start(Dev<T> d, const double *xs, const double *ys, int c)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < d.n) {
        const double v0 = xs ? xs[i] * d.Dc[i] : 0.0;
        pick(d.xb, c)[i] = clampv((T)v0, d.ls[i], d.us[i]);
    }
    if (i < d.m) {
        double v0 = ys ? ys[i] * d.Dr[i] : 0.0;
        if (i >= d.m1 && v0 < 0.0) v0 = 0.0;
        pick(d.yb, c)[i] = (T)v0;
    }
}

// unscale the returned point; lam = proj_Lambda(c - K'y)
template <typename T>
__global__ void k_result(Dev<T> d, double *x, double *y, double *lam)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < d.n) {
        x[i] = (double)d.xo[i] / d.Dc[i];
        const double g = ((double)d.cs[i] - (double)d.KTyo[i]) * d.Dc[i];
        lam[i] = proj_lambda(g, isfinite((double)d.ls[i]), isfinite((double)d.us[i]));
    }
    if (i < d.m) y[i] = (double)d.yo[i] / d.Dr[i];
}

template <typename A, typename B>
__global__ void k_convert(const A *in, B *out, int64_t len)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < len) out[i] = (B)in[i];
}

// ----------------------------------------------------------------------------
// one-time scaling kernels (FP64, one wave64 per row)
// ----------------------------------------------------------------------------

// skip_long: rows longer than kLongRow are left at 0 (k_row_absmax_long
// then takes their maximum with many workgroups)
__global__ void k_row_absmax(const int *rp, const double *v, int nrows, int skip_long, double *out)
{
    const int row = blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    double a = 0.0;
    if (!(skip_long && rp[row + 1] - rp[row] > kLongRow))
        for (int j = rp[row] + lane; j < rp[row + 1]; j += 64) a = fmax(a, fabs(v[j]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a = fmax(a, __shfl_xor(a, off));
    if (lane == 0) out[row] = a;
}

__global__ void k_row_abspow_sum(const int *rp, const double *v, int nrows, double p, double *out)
{
    const int row = blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    double a = 0.0;
    for (int j = rp[row] + lane; j < rp[row + 1]; j += 64) {
        const double t = fabs(v[j]);
        a += p == 1.0 ? t : pow(t, p);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if (lane == 0) out[row] = a;
}

__global__ void k_finish_factor(double *f, int len)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < len) f[i] = f[i] > 0.0 ? sqrt(f[i]) : 1.0;
}

__global__ void k_rescale_rows(const int *rp, const int *ci, double *v, int nrows, int skip_long, const double *rowf,
                               const double *colf)
{
    const int row = blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    if (skip_long && rp[row + 1] - rp[row] > kLongRow) return;
    const double r = rowf[row];
    for (int j = rp[row] + lane; j < rp[row + 1]; j += 64) v[j] = v[j] / (r * colf[ci[j]]);
}

// The long rows listed in rows[0..nlong) (each more than kLongRow entries),
// spread over gridDim.x workgroups per row (blockIdx.y picks the row).  The
// maximum of |v| >= 0 is combined by an integer atomic max on the bit
// pattern, which orders non-negative doubles exactly, so the result does not
// depend on the order; the rescale is per entry, as in k_rescale_rows.
__global__ void k_row_absmax_long(const int *rp, const double *v, const int *rows, double *out)
{
    __shared__ double sh[kBlock / 64];
    const int r = rows[blockIdx.y];
    double a = 0.0;
    for (int j = rp[r] + (int)(blockIdx.x * kBlock + threadIdx.x); j < rp[r + 1]; j += (int)(gridDim.x * kBlock))
        a = fmax(a, fabs(v[j]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a = fmax(a, __shfl_xor(a, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double b = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        atomicMax(reinterpret_cast<unsigned long long *>(out + r), (unsigned long long)__double_as_longlong(b));
    }
}

__global__ void k_rescale_long(const int *rp, const int *ci, double *v, const int *rows, const double *rowf,
                               const double *colf)
{
    const int r = rows[blockIdx.y];
    const double f = rowf[r];
    for (int j = rp[r] + (int)(blockIdx.x * kBlock + threadIdx.x); j < rp[r + 1]; j += (int)(gridDim.x * kBlock))
        v[j] = v[j] / (f * colf[ci[j]]);
}

__global__ void k_mul_inplace(double *a, const double *f, int len)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < len) a[i] *= f[i];
}

__global__ void k_fill(double *a, double v, int len)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < len) a[i] = v;
}

__global__ void k_scale_vectors(const double *c, const double *l, const double *u, const double *q,
                                const double *Dc, const double *Dr, double *cs, double *ls, double *us,
                                double *qs, int n, int m)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < n) {
        cs[i] = c[i] / Dc[i];
        ls[i] = l[i] * Dc[i];
        us[i] = u[i] * Dc[i];
    }
    if (i < m) qs[i] = q[i] / Dr[i];
}

constexpr int kRedGrid = 1024;

__global__ void k_sumsq_part(const double *a, int64_t len, double *part)
{
    double s[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock)
        s[0] += a[i] * a[i];
    block_store_partials<1>(s, part);
}

__global__ void k_sum_final(const double *part, int np, double *out)
{
    double s[1];
    block_sum_partials<1>(part, np, s);
    if (threadIdx.x == 0) out[0] = s[0];
}

__global__ void k_absmax_part(const double *a, int64_t len, double *part)
{
    __shared__ double sh[kBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < len; i += (int64_t)gridDim.x * kBlock)
        s = fmax(s, fabs(a[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ void k_max_final(const double *part, int np, double *out)
{
    __shared__ double sh[kBlock / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < np; b += kBlock) s = fmax(s, part[b]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

static inline int blocks_for(int64_t len) { return (int)((len + kBlock - 1) / kBlock); }

template <typename T>
hipError_t launch_partial_K(const Dev<T> &d, hipStream_t s)
{
    const dim3 g(d.K.grid), t(kBlock);
    if (d.K.nlong) {
        if (d.K.split) hipLaunchKernelGGL((k_partial_K<T, true, true>), g, t, 0, s, d);
        else hipLaunchKernelGGL((k_partial_K<T, true, false>), g, t, 0, s, d);
    } else {
        if (d.K.split) hipLaunchKernelGGL((k_partial_K<T, false, true>), g, t, 0, s, d);
        else hipLaunchKernelGGL((k_partial_K<T, false, false>), g, t, 0, s, d);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_partial_KT(const Dev<T> &d, hipStream_t s)
{
    const dim3 g(d.KT.grid), t(kBlock);
    if (d.KT.nlong) {
        if (d.KT.split) hipLaunchKernelGGL((k_partial_KT<T, true, true>), g, t, 0, s, d);
        else hipLaunchKernelGGL((k_partial_KT<T, true, false>), g, t, 0, s, d);
    } else {
        if (d.KT.split) hipLaunchKernelGGL((k_partial_KT<T, false, true>), g, t, 0, s, d);
        else hipLaunchKernelGGL((k_partial_KT<T, false, false>), g, t, 0, s, d);
    }
    return hipGetLastError();
}

template <typename T, bool LONG>
void launch_dual_t(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    switch (d.K.S) {
    case 1: hipLaunchKernelGGL((k_dual<T, 1, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m); break;
    case 2: hipLaunchKernelGGL((k_dual<T, 2, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m); break;
    case 4: hipLaunchKernelGGL((k_dual<T, 4, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m); break;
    case 8: hipLaunchKernelGGL((k_dual<T, 8, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m); break;
    case 16: hipLaunchKernelGGL((k_dual<T, 16, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m); break;
    default: hipLaunchKernelGGL((k_dual<T, 0, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m); break;
    }
}

template <typename T>
hipError_t launch_dual(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    if (d.K.nlong) launch_dual_t<T, true>(d, g, s);
    else launch_dual_t<T, false>(d, g, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_decide(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_decide, dim3(1), dim3(kBlock), 0, s, d.ctl, (const double *)d.part_primal,
                       (const double *)d.part_dual, g.grid);
    return hipGetLastError();
}

template <typename T, bool LONG>
void launch_update_t(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    switch (d.KT.S) {
    case 1: hipLaunchKernelGGL((k_update<T, 1, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m); break;
    case 2: hipLaunchKernelGGL((k_update<T, 2, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m); break;
    case 4: hipLaunchKernelGGL((k_update<T, 4, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m); break;
    case 8: hipLaunchKernelGGL((k_update<T, 8, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m); break;
    case 16: hipLaunchKernelGGL((k_update<T, 16, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m);
        break;
    default: hipLaunchKernelGGL((k_update<T, 0, LONG>), dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m); break;
    }
}

template <typename T>
hipError_t launch_update(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    if (d.KT.nlong) launch_update_t<T, true>(d, g, s);
    else launch_update_t<T, false>(d, g, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_check_reduce(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_reduce<T>, dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_check_decide(const Dev<T> &d, const Geo &g, double Nq, double Nc, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_decide, dim3(1), dim3(kBlock), 0, s, d.ctl, (const double *)d.part_check,
                       (const double *)d.part_ray, g.grid, Nq, Nc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_check_apply(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_apply<T>, dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m);
    return hipGetLastError();
}

// The FP64 re-check of mixed precision's termination test: the four
// products of the current iterate (buffer cur, read from the controller by
// the host that stopped for the re-check) and the average, their check sums,
// and the decision.
template <typename T>
hipError_t launch_confirm(const Dev<T> &d, const Geo &g, const Conf64 &cf, int cur, double Nq, double Nc,
                          hipStream_t s)
{
    return launch_confirm_gather<T>(d, g, cf, cur, cur ? d.xb[1] : d.xb[0], d.xa, cur ? d.yb[1] : d.yb[0], d.ya, Nq,
                                    Nc, s);
}

template <typename T>
hipError_t launch_confirm_gather(const Dev<T> &d, const Geo &g, const Conf64 &cf, int cur, const T *gx,
                                 const T *gxa, const T *gy, const T *gya, double Nq, double Nc, hipStream_t s)
{
    auto waves = [](int rows) { return dim3((unsigned)std::max(1, std::min((rows + 3) / 4, 8192))); };
    if (d.m > 0) {
        hipLaunchKernelGGL(k_csr64<T>, waves(d.m), dim3(kBlock), 0, s, cf.rp, cf.ci, cf.kv, gx, cf.kx[0], d.m);
        hipLaunchKernelGGL(k_csr64<T>, waves(d.m), dim3(kBlock), 0, s, cf.rp, cf.ci, cf.kv, gxa, cf.kx[1], d.m);
    }
    if (d.n > 0) {
        hipLaunchKernelGGL(k_csr64<T>, waves(d.n), dim3(kBlock), 0, s, cf.tp, cf.ti, cf.tv, gy, cf.kty[0], d.n);
        hipLaunchKernelGGL(k_csr64<T>, waves(d.n), dim3(kBlock), 0, s, cf.tp, cf.ti, cf.tv, gya, cf.kty[1], d.n);
    }
    hipLaunchKernelGGL(k_confirm_sums<T>, dim3(g.grid), dim3(kBlock), 0, s, d, cf, cur, g.vb_n, g.vb_m);
    hipLaunchKernelGGL(k_confirm_decide, dim3(1), dim3(kBlock), 0, s, d.ctl, (const double *)cf.part, g.grid, Nq, Nc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_small_loop_batch(const Dev<T> *devs, const double *nq, const double *nc, int count, int R,
                                   size_t stage_bytes, int max_slots, hipStream_t s)
{
    static bool attr_set = false;   // the kernels' LDS limit raised once per process
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_small_reg_batch<T, 1>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallRegLds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_small_reg_batch<T, 2>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallRegLds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t bytes = ((stage_bytes + 7) / 8) * 8 + 16 * (size_t)max_slots;
    if (count <= 0 || max_slots <= 0 || bytes > kSmallRegLds || (R != 1 && R != 2)) return hipErrorInvalidValue;
    if (R == 1)
        hipLaunchKernelGGL((k_small_reg_batch<T, 1>), dim3(count), dim3(kSmallReg), bytes, s, devs, nq, nc, max_slots);
    else
        hipLaunchKernelGGL((k_small_reg_batch<T, 2>), dim3(count), dim3(kSmallReg), bytes, s, devs, nq, nc, max_slots);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_small_loop(const Dev<T> &d, int nnz_k, int nnz_t, int max_slots, double Nq, double Nc,
                             hipStream_t s)
{
    const size_t lds = small_stage_bytes<T>(d.m, d.n, nnz_k, nnz_t);
    if (lds <= kSmallStageMax) {
        static bool attr_set = false;   // the kernels' LDS limit raised once per process
        if (!attr_set) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_small_loop<T, true>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallStageMax);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_small_reg<T, 1>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallRegLds);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_small_reg<T, 2>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallRegLds);
            if (e != hipSuccess) return e;
            attr_set = true;
        }
        if (d.n <= 2 * kSmallReg && d.m <= 2 * kSmallReg && lds + 16 * 64 <= kSmallRegLds) {
            // as many slots as the factor table in the rest of the LDS holds
            const int tab = (int)std::min<size_t>((kSmallRegLds - ((lds + 7) / 8) * 8) / 16, (size_t)max_slots);
            const size_t bytes = ((lds + 7) / 8) * 8 + 16 * (size_t)tab;
            if (d.n <= kSmallReg && d.m <= kSmallReg)
                hipLaunchKernelGGL((k_small_reg<T, 1>), dim3(1), dim3(kSmallReg), bytes, s, d, tab, Nq, Nc);
            else
                hipLaunchKernelGGL((k_small_reg<T, 2>), dim3(1), dim3(kSmallReg), bytes, s, d, tab, Nq, Nc);
        } else
            hipLaunchKernelGGL((k_small_loop<T, true>), dim3(1), dim3(kSmall), lds, s, d, max_slots, Nq, Nc);
    } else {
        hipLaunchKernelGGL((k_small_loop<T, false>), dim3(1), dim3(kSmall), 0, s, d, max_slots, Nq, Nc);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_probe(const int *idx, const T *x, int64_t per_slice, int S, int64_t slice_len, T *out,
                               int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_probe<T>, dim3(grid), dim3(kBlock), 0, s, idx, x, per_slice, S, slice_len, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv(const Sliced<T> &P, const T *in, T *out, hipStream_t s)
{
    if (P.rows <= 0) return hipSuccess;
    if (P.nlong) {
        if (P.split) hipLaunchKernelGGL((k_partial_plain<T, true, true>), dim3(P.grid), dim3(kBlock), 0, s, P, in);
        else hipLaunchKernelGGL((k_partial_plain<T, true, false>), dim3(P.grid), dim3(kBlock), 0, s, P, in);
        hipLaunchKernelGGL((k_sum_slices<T, true>), dim3(blocks_for(P.rows)), dim3(kBlock), 0, s, P, out);
    } else {
        if (P.split) hipLaunchKernelGGL((k_partial_plain<T, false, true>), dim3(P.grid), dim3(kBlock), 0, s, P, in);
        else hipLaunchKernelGGL((k_partial_plain<T, false, false>), dim3(P.grid), dim3(kBlock), 0, s, P, in);
        hipLaunchKernelGGL((k_sum_slices<T, false>), dim3(blocks_for(P.rows)), dim3(kBlock), 0, s, P, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_values(const double *src_vals, const int *src_pos, T *dst, int64_t len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_values<T>, dim3(blocks_for(len)), dim3(kBlock), 0, s, src_vals, src_pos, dst, len);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_start(const Dev<T> &d, const double *xs, const double *ys, int cur, hipStream_t s)
{
    const int nb = blocks_for(d.n > d.m ? d.n : d.m);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_start<T>, dim3(nb), dim3(kBlock), 0, s, d, xs, ys, cur);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_result(const Dev<T> &d, double *x, double *y, double *lam, hipStream_t s)
{
    const int nb = blocks_for(d.n > d.m ? d.n : d.m);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_result<T>, dim3(nb), dim3(kBlock), 0, s, d, x, y, lam);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_to_double(const T *in, double *out, int64_t len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert<T, double>), dim3(blocks_for(len)), dim3(kBlock), 0, s, in, out, len);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_from_double(const double *in, T *out, int64_t len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert<double, T>), dim3(blocks_for(len)), dim3(kBlock), 0, s, in, out, len);
    return hipGetLastError();
}

hipError_t launch_row_absmax(const int *rp, const double *v, int nrows, double *out, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_absmax, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, v, nrows, 0, out);
    return hipGetLastError();
}

hipError_t launch_row_abspow_sum(const int *rp, const double *v, int nrows, double p, double *out, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_abspow_sum, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, v, nrows, p, out);
    return hipGetLastError();
}

hipError_t launch_finish_factor(double *f, int len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish_factor, dim3(blocks_for(len)), dim3(kBlock), 0, s, f, len);
    return hipGetLastError();
}

hipError_t launch_rescale_rows(const int *rp, const int *ci, double *v, int nrows, const double *rowf,
                               const double *colf, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rescale_rows, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, ci, v, nrows, 0, rowf, colf);
    return hipGetLastError();
}

hipError_t launch_mul_inplace(double *a, const double *f, int len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul_inplace, dim3(blocks_for(len)), dim3(kBlock), 0, s, a, f, len);
    return hipGetLastError();
}

hipError_t launch_fill(double *a, double v, int len, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(len)), dim3(kBlock), 0, s, a, v, len);
    return hipGetLastError();
}

hipError_t launch_scale_vectors(const double *c, const double *l, const double *u, const double *q,
                                const double *Dc, const double *Dr, double *cs, double *ls, double *us,
                                double *qs, int n, int m, hipStream_t s)
{
    const int nb = blocks_for(n > m ? n : m);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_vectors, dim3(nb), dim3(kBlock), 0, s, c, l, u, q, Dc, Dr, cs, ls, us, qs, n, m);
    return hipGetLastError();
}

hipError_t launch_sumsq(const double *a, int64_t len, double *part, double *out, hipStream_t s)
{
    int g = (int)((len + kBlock - 1) / kBlock);
    if (g > kRedGrid) g = kRedGrid;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_sumsq_part, dim3(g), dim3(kBlock), 0, s, a, len, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, g, out);
    return hipGetLastError();
}

hipError_t launch_absmax(const double *a, int64_t len, double *part, double *out, hipStream_t s)
{
    int g = (int)((len + kBlock - 1) / kBlock);
    if (g > kRedGrid) g = kRedGrid;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_absmax_part, dim3(g), dim3(kBlock), 0, s, a, len, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, g, out);
    return hipGetLastError();
}

// The diagonal scaling on the device: ruiz_iters Ruiz rounds (factors sqrt
// of the inf-norm of each row of K and of K', both from the same current
// matrix), then one Pock-Chambolle round with exponent alpha (skipped when
// alpha < 0).  Scales both CSR copies in place and accumulates Dr, Dc.
// One product's row maxima / rescale, its long rows (if listed) on their own grid.
static void row_absmax_split(const int *rp, const double *v, int nrows, const int *lrows, int nlong, double *out,
                             hipStream_t s)
{
    if (nrows <= 0) return;
    const int skip = lrows && nlong > 0 && nlong <= 65535;   // gridDim.y limit
    hipLaunchKernelGGL(k_row_absmax, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, v, nrows, skip, out);
    if (skip) hipLaunchKernelGGL(k_row_absmax_long, dim3(256, nlong), dim3(kBlock), 0, s, rp, v, lrows, out);
}

static void rescale_split(const int *rp, const int *ci, double *v, int nrows, const int *lrows, int nlong,
                          const double *rowf, const double *colf, hipStream_t s)
{
    if (nrows <= 0) return;
    const int skip = lrows && nlong > 0 && nlong <= 65535;   // gridDim.y limit
    hipLaunchKernelGGL(k_rescale_rows, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, ci, v, nrows, skip, rowf,
                       colf);
    if (skip) hipLaunchKernelGGL(k_rescale_long, dim3(256, nlong), dim3(kBlock), 0, s, rp, ci, v, lrows, rowf, colf);
}

hipError_t scale_csr_pair(const int *rp, const int *ci, double *kv, int m, const int *tp, const int *ti, double *tv,
                          int n, double *Dr, double *Dc, double *r, double *s, int ruiz_iters, double alpha,
                          hipStream_t st, const int *klong, int nklong, const int *tlong, int ntlong)
{
    hipError_t e;
    if ((e = launch_fill(Dr, 1.0, m, st)) != hipSuccess) return e;
    if ((e = launch_fill(Dc, 1.0, n, st)) != hipSuccess) return e;
    const int rounds = ruiz_iters + (alpha >= 0.0 ? 1 : 0);
    for (int it = 0; it < rounds; ++it) {
        const bool pc = it == ruiz_iters;
        if (!pc) {
            row_absmax_split(rp, kv, m, klong, nklong, r, st);
            row_absmax_split(tp, tv, n, tlong, ntlong, s, st);
        } else {
            (void)launch_row_abspow_sum(rp, kv, m, 2.0 - alpha, r, st);
            (void)launch_row_abspow_sum(tp, tv, n, alpha, s, st);
        }
        (void)launch_finish_factor(r, m, st);
        (void)launch_finish_factor(s, n, st);
        rescale_split(rp, ci, kv, m, klong, nklong, r, s, st);
        rescale_split(tp, ti, tv, n, tlong, ntlong, s, r, st);
        (void)launch_mul_inplace(Dr, r, m, st);
        if ((e = launch_mul_inplace(Dc, s, n, st)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

#define PDLP_INSTANTIATE(T)                                                                                        \
    template hipError_t launch_partial_K<T>(const Dev<T> &, hipStream_t);                                          \
    template hipError_t launch_partial_KT<T>(const Dev<T> &, hipStream_t);                                         \
    template hipError_t launch_dual<T>(const Dev<T> &, const Geo &, hipStream_t);                                  \
    template hipError_t launch_step_decide<T>(const Dev<T> &, const Geo &, hipStream_t);                           \
    template hipError_t launch_update<T>(const Dev<T> &, const Geo &, hipStream_t);                                \
    template hipError_t launch_check_reduce<T>(const Dev<T> &, const Geo &, hipStream_t);                          \
    template hipError_t launch_check_decide<T>(const Dev<T> &, const Geo &, double, double, hipStream_t);          \
    template hipError_t launch_check_apply<T>(const Dev<T> &, const Geo &, hipStream_t);                           \
    template hipError_t launch_spmv<T>(const Sliced<T> &, const T *, T *, hipStream_t);                            \
    template hipError_t launch_gather_probe<T>(const int *, const T *, int64_t, int, int64_t, T *, int, hipStream_t); \
    template hipError_t launch_small_loop<T>(const Dev<T> &, int, int, int, double, double, hipStream_t);        \
    template hipError_t launch_small_loop_batch<T>(const Dev<T> *, const double *, const double *, int, int,      \
                                                   size_t, int, hipStream_t);                                     \
    template hipError_t launch_confirm<T>(const Dev<T> &, const Geo &, const Conf64 &, int, double, double,       \
                                          hipStream_t);                                                           \
    template hipError_t launch_confirm_gather<T>(const Dev<T> &, const Geo &, const Conf64 &, int, const T *,     \
                                                 const T *, const T *, const T *, double, double, hipStream_t);   \
    template hipError_t launch_gather_values<T>(const double *, const int *, T *, int64_t, hipStream_t);           \
    template hipError_t launch_start<T>(const Dev<T> &, const double *, const double *, int, hipStream_t);         \
    template hipError_t launch_result<T>(const Dev<T> &, double *, double *, double *, hipStream_t);               \
    template hipError_t launch_to_double<T>(const T *, double *, int64_t, hipStream_t);                            \
    template hipError_t launch_from_double<T>(const double *, T *, int64_t, hipStream_t);

PDLP_INSTANTIATE(double)
PDLP_INSTANTIATE(float)

}  // namespace pdlp
