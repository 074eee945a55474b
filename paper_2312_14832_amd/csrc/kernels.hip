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
// coalesced streaming loads, then sums each row from LDS; the slice of x it
// gathers from stays resident in its XCD's L2.  The fused epilogue kernels
// add the slices' partial rows in a fixed order.
// Reductions are deterministic: each lane accumulates in FP64, wave64
// butterflies and a fixed-order LDS step give one partial per workgroup, and
// a single workgroup sums the partials in a fixed order.  No float atomics.
#include "internal.h"

#include <cmath>

namespace pdlp {

// ----------------------------------------------------------------------------
// small device helpers
// ----------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T clampv(T v, T lo, T hi)
{
    // projection onto [lo, hi]; NaN passes through
    return v < lo ? lo : (v > hi ? hi : v);
}

template <typename P>
__device__ __forceinline__ P pick(P const (&a)[2], int i)
{
    return i ? a[1] : a[0];
}

__device__ __forceinline__ double proj_lambda(double g, bool lf, bool uf)
{
    if (!lf && !uf) return 0.0;
    if (!lf) return g < 0.0 ? g : 0.0;
    if (!uf) return g > 0.0 ? g : 0.0;
    return g;
}

// One FP64 partial per workgroup and value: wave64 butterfly, then the four
// wave results added in a fixed order.
template <int NV>
__device__ __forceinline__ void block_store_partials(double (&v)[NV], double *out)
{
    __shared__ double sh[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    if (threadIdx.x < NV) {
        const int i = threadIdx.x;
        out[(size_t)blockIdx.x * NV + i] = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
    }
}

// Sum np partials of NV values each inside one workgroup; every thread gets
// the same (deterministic) totals.
template <int NV>
__device__ __forceinline__ void block_sum_partials(const double *part, int np, double (&out)[NV])
{
    __shared__ double sh[kBlock / 64][NV];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int b = threadIdx.x; b < np; b += kBlock) {
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += part[(size_t)b * NV + i];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off);
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wave][i] = acc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
    __syncthreads();
}

// ----------------------------------------------------------------------------
// column-sliced CSR-Stream partial products
// ----------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void sliced_partial(const Sliced<T> &P, const T *__restrict__ x)
{
    __shared__ T prod[kStreamNB];
    __shared__ double red[kBlock / 64];
    const int S = P.S;
    const int s = (int)blockIdx.x % S;
    const int chunk0 = (int)blockIdx.x / S, stride = (int)gridDim.x / S;
    const int *__restrict__ rp = P.rp + (size_t)s * (P.rows + 1);
    T *__restrict__ out = P.part + (size_t)s * P.rows;
    const int nblk = P.boff[s + 1] - P.boff[s];
    const int *__restrict__ bro = P.brow + P.boff[s] + s;
    const int *__restrict__ ci = P.ci;
    const T *__restrict__ v = P.v;
    for (int k = chunk0; k < nblk; k += stride) {
        const int r0 = bro[k], r1 = bro[k + 1];
        const int b = rp[r0], e = rp[r1];
        const int cnt = e - b;
        if (cnt <= kStreamNB) {
#pragma unroll 4
            for (int t = (int)threadIdx.x; t < cnt; t += kBlock) {
                const int c = __builtin_nontemporal_load(ci + b + t);
                const T a = __builtin_nontemporal_load(v + b + t);
                prod[t] = a * x[c];
            }
            __syncthreads();
            const int r = r0 + (int)threadIdx.x;   // r1 - r0 <= kStreamRB == kBlock
            if (r < r1) {
                T acc = T(0);
                const int je = rp[r + 1] - b;
                for (int j = rp[r] - b; j < je; ++j) acc += prod[j];
                out[r] = acc;
            }
            __syncthreads();
        } else {
            // one row with more than kStreamNB nonzeros in this slice
            T acc = T(0);
            for (int t = b + (int)threadIdx.x; t < e; t += kBlock) acc += v[t] * x[ci[t]];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (double)acc;
            __syncthreads();
            if (threadIdx.x == 0) out[r0] = (T)(((red[0] + red[1]) + red[2]) + red[3]);
            __syncthreads();
        }
    }
}

// row i of the product: the slices' partials added in slice order
template <typename T>
__device__ __forceinline__ T sum_slices(const Sliced<T> &P, int i)
{
    T a = P.part[i];
    for (int s = 1; s < P.S; ++s) a += P.part[(size_t)s * P.rows + i];
    return a;
}

// ----------------------------------------------------------------------------
// epilogues
// ----------------------------------------------------------------------------

// dual step on row i: y' = proj_Y(y + sigma (q - 2 Kx' + Kx)), y'_i >= 0 on G rows
template <typename T>
struct DualEpi {
    const T *__restrict__ y;
    const T *__restrict__ kx;
    const T *__restrict__ q;
    T *__restrict__ yn;
    T *__restrict__ kxn;
    int m1;
    T sigma;
    double dy2, inter;
    __device__ __forceinline__ void operator()(int i, T s)
    {
        const T yo = y[i], ko = kx[i];
        T val = yo + sigma * (q[i] - T(2) * s + ko);
        if (i >= m1 && val < T(0)) val = T(0);
        yn[i] = val;
        kxn[i] = s;
        const double d = (double)val - (double)yo;
        dy2 += d * d;
        inter += d * ((double)s - (double)ko);
    }
};

// after an accepted step, on column j: K'y' stored, averages moved, and the
// next primal trial x'' = proj_X(x' - tau (c - K'y'))
template <typename T>
struct UpdateEpi {
    const T *__restrict__ x;
    const T *__restrict__ cs;
    const T *__restrict__ ls;
    const T *__restrict__ us;
    T *__restrict__ kty;
    T *__restrict__ xa;
    T *__restrict__ ktya;
    T *__restrict__ xn;
    T w, tau;
    bool primal;
    double dx2;
    __device__ __forceinline__ void operator()(int j, T s)
    {
        kty[j] = s;
        const T xj = x[j];
        const T a = xa[j];
        xa[j] = a + w * (xj - a);
        const T b = ktya[j];
        ktya[j] = b + w * (s - b);
        if (primal) {
            const T nv = clampv(xj - tau * (cs[j] - s), ls[j], us[j]);
            xn[j] = nv;
            const double d = (double)nv - (double)xj;
            dx2 += d * d;
        }
    }
};

template <typename T>
__device__ __forceinline__ void primal_elem(const Dev<T> &d, int c, T tau, int j, double &dx2)
{
    const T *x = pick(d.xb, c);
    const T *kty = pick(d.KTyb, c);
    T *xn = pick(d.xb, c ^ 1);
    const T xj = x[j];
    const T nv = clampv(xj - tau * (d.cs[j] - kty[j]), d.ls[j], d.us[j]);
    xn[j] = nv;
    const double dd = (double)nv - (double)xj;
    dx2 += dd * dd;
}

// ----------------------------------------------------------------------------
// the iteration kernels
// ----------------------------------------------------------------------------

// K x' partial products (x' = the primal trial)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_partial_K(Dev<T> d)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done) return;
    sliced_partial(d.K, (const T *)pick(d.xb, ctl->cur ^ 1));
}

// K' y' partial products, only after an accepted step
template <typename T>
__global__ __launch_bounds__(kBlock) void k_partial_KT(Dev<T> d)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done || !ctl->accepted) return;
    sliced_partial(d.KT, (const T *)pick(d.yb, ctl->cur));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dual(Dev<T> d, int vb_m)
{
    const Ctl *ctl = d.ctl;
    if (ctl->done) return;
    const int c = ctl->cur;
    const T sigma = (T)(ctl->eta * ctl->omega);
    DualEpi<T> epi{pick(d.yb, c), pick(d.Kxb, c), d.qs, pick(d.yb, c ^ 1), pick(d.Kxb, c ^ 1), d.m1, sigma, 0.0, 0.0};
    for (int vb = blockIdx.x; vb < vb_m; vb += gridDim.x) {
        const int i = vb * kBlock + (int)threadIdx.x;
        if (i < d.m) epi(i, sum_slices(d.K, i));
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
    const double dx2 = a[0], dy2 = b[0], inter = b[1];
    const double eta = ctl->eta, omega = ctl->omega;
    double eta_new = eta;
    bool accept = true;
    ctl->attempts += 1;
    if (!ctl->fixed_step) {
        const double N = omega * dx2 + dy2 / omega;
        const double D = 2.0 * fabs(inter);
        if (isnan(N) || isnan(D)) {
            ctl->numerical = 1;
            ctl->accepted = 0;
            ctl->mode = MODE_CHECK;
            return;
        }
        const double eta_bar = D > 0.0 ? N / D : INFINITY;
        const double kk = (double)(ctl->k + 1) + 1.0;
        const double lo = (1.0 - pow(kk, -0.3)) * eta_bar;
        const double hi = (1.0 + pow(kk, -0.6)) * eta;
        eta_new = lo < hi ? lo : hi;
        accept = eta <= eta_bar;
    }
    if (accept) {
        ctl->W += eta;
        ctl->avg_w = eta / ctl->W;
        ctl->eta_last = eta;
        ctl->k += 1;
        ctl->t += 1;
        ctl->cur ^= 1;
        ctl->accepted = 1;
        ctl->mode = (ctl->k % ctl->check_every == 0 || ctl->k >= ctl->max_iters) ? MODE_CHECK : MODE_NONE;
    } else {
        ctl->accepted = 0;
        ctl->mode = MODE_NONE;
    }
    ctl->eta = eta_new;
}

template <typename T>
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
        const T *y = pick(d.yb, c);
        const T *kx = pick(d.Kxb, c);
        const int total = vb_n + vb_m;
        for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
            if (vb < vb_n) {
                const int j = vb * kBlock + (int)threadIdx.x;
                if (j < d.n) epi(j, sum_slices(d.KT, j));
            } else {
                const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
                if (i < d.m) {
                    const T w = epi.w;
                    const T a = d.ya[i];
                    d.ya[i] = a + w * (y[i] - a);
                    const T b = d.Kxa[i];
                    d.Kxa[i] = b + w * (kx[i] - b);
                }
            }
        }
        dx2 = epi.dx2;
    }
    double v[1] = {dx2};
    block_store_partials<1>(v, d.part_primal);
}

// the 9 check sums of one iterate; s[0..3] rows, s[4..8] columns:
// |r_p|^2 unscaled, |r_p|^2 scaled, q'y, |y-y0|^2,
// |r_d|^2 unscaled, |r_d|^2 scaled, c'x, l'lam+ - u'lam-, |x-x0|^2
template <typename T>
__device__ __forceinline__ void row_sums(const Dev<T> &d, int i, const T *y, const T *kx, double *s)
{
    const double k = (double)kx[i], q = (double)d.qs[i];
    double r = k - q;
    if (i >= d.m1) {
        const double t = q - k;
        r = t > 0.0 ? t : 0.0;
    }
    const double ru = r * d.Dr[i];
    s[0] += ru * ru;
    s[1] += r * r;
    const double yi = (double)y[i];
    s[2] += q * yi;
    const double dd = yi - (double)d.y0[i];
    s[3] += dd * dd;
}

template <typename T>
__device__ __forceinline__ void col_sums(const Dev<T> &d, int j, const T *x, const T *kty, double *s)
{
    const double cj = (double)d.cs[j], lj = (double)d.ls[j], uj = (double)d.us[j];
    const bool lf = isfinite(lj), uf = isfinite(uj);
    const double g = cj - (double)kty[j];
    const double lam = proj_lambda(g, lf, uf);
    const double rd = g - lam;
    const double rdu = rd * d.Dc[j];
    s[4] += rdu * rdu;
    s[5] += rd * rd;
    const double xj = (double)x[j];
    s[6] += cj * xj;
    double b = 0.0;
    if (lf && lam > 0.0) b += lj * lam;
    if (uf && lam < 0.0) b += uj * lam;
    s[7] += b;
    const double dd = xj - (double)d.x0[j];
    s[8] += dd * dd;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_check_reduce(Dev<T> d, int vb_n, int vb_m)
{
    const Ctl *ctl = d.ctl;
    if (ctl->mode == MODE_NONE || ctl->done) return;
    const int c = ctl->cur;
    const T *x = pick(d.xb, c), *kty = pick(d.KTyb, c), *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
    double s[kCheckSums];
#pragma unroll
    for (int i = 0; i < kCheckSums; ++i) s[i] = 0.0;
    for (int vb = blockIdx.x; vb < vb_n + vb_m; vb += gridDim.x) {
        if (vb < vb_n) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) {
                col_sums(d, j, x, kty, s);
                col_sums(d, j, d.xa, d.KTya, s + 9);
            }
        } else {
            const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
            if (i < d.m) {
                row_sums(d, i, y, kx, s);
                row_sums(d, i, d.ya, d.Kxa, s + 9);
            }
        }
    }
    block_store_partials<kCheckSums>(s, d.part_check);
}

// Termination (three relative criteria, unscaled), candidate choice and
// restart conditions 1-3 on KKT_omega (scaled), primal-weight update.
__global__ __launch_bounds__(kBlock) void k_check_decide(Ctl *ctl, const double *part, int np, double Nq, double Nc)
{
    if (ctl->mode == MODE_NONE || ctl->done) return;
    double S[kCheckSums];
    block_sum_partials<kCheckSums>(part, np, S);
    if (threadIdx.x != 0) return;
    const double wp = pow(ctl->omega, ctl->kkt_p);
    double rel[2], kkt[2];
    for (int z = 0; z < 2; ++z) {
        const double *e = S + 9 * z;
        const double pobj = e[6], dobj = e[2] + e[7], gap = dobj - pobj;
        const double rp = sqrt(e[0]) / (1.0 + Nq);
        const double rd = sqrt(e[4]) / (1.0 + Nc);
        const double rg = fabs(gap) / (1.0 + fabs(dobj) + fabs(pobj));
        double r = rp;
        if (rd > r) r = rd;
        if (rg > r) r = rg;
        if (isnan(rp) || isnan(rd) || isnan(rg)) r = NAN;
        rel[z] = r;
        kkt[z] = sqrt(wp * e[1] + e[5] / wp + gap * gap);
        ctl->rel_p[z] = rp;
        ctl->rel_d[z] = rd;
        ctl->rel_g[z] = rg;
        ctl->pobj[z] = pobj;
        ctl->dobj[z] = dobj;
        ctl->kkt[z] = kkt[z];
    }
    const int mode = ctl->mode;
    ctl->restart_to = 0;
    ctl->copy_out = 0;
    ctl->need_primal = 0;
    if (mode == MODE_INIT) {
        ctl->KKT0 = kkt[0];
        ctl->KKT_prev = INFINITY;
        ctl->need_primal = 1;
        return;
    }
    auto finish = [&](int status, int sel) {
        ctl->status = status;
        ctl->out_sel = sel;
        ctl->copy_out = 1;
        ctl->done = 1;
        ctl->out_rel_p = ctl->rel_p[sel];
        ctl->out_rel_d = ctl->rel_d[sel];
        ctl->out_rel_g = ctl->rel_g[sel];
        ctl->out_pobj = ctl->pobj[sel];
        ctl->out_dobj = ctl->dobj[sel];
    };
    if (ctl->numerical || isnan(rel[0]) || isnan(rel[1])) {
        finish(LP_NUMERICAL, 0);
        return;
    }
    const int use_avg = rel[1] < rel[0] ? 1 : 0;
    if (rel[0] <= ctl->tol || rel[1] <= ctl->tol) {
        finish(LP_OPTIMAL, use_avg);
        return;
    }
    int at_limit = 0;
    if (mode == MODE_FINAL) at_limit = ctl->final_status;
    else if (ctl->k >= ctl->max_iters) at_limit = LP_ITERATION_LIMIT;
    if (at_limit) finish(at_limit, use_avg);
    if (mode == MODE_CHECK && ctl->k % ctl->check_every == 0) {
        const int cand_cur = kkt[0] < kkt[1];
        const double kz = cand_cur ? kkt[0] : kkt[1];
        const double *ez = S + (cand_cur ? 0 : 9);
        int why = 0;
        if (kz <= 0.2 * ctl->KKT0) why = 1;
        else if (kz <= 0.8 * ctl->KKT0 && kz > ctl->KKT_prev) why = 2;
        else if ((double)ctl->t >= 0.36 * (double)ctl->k) why = 3;
        ctl->KKT_prev = kz;
        if (why) {
            const double dx = sqrt(ez[8]), dy = sqrt(ez[3]);
            double om = ctl->omega;
            if (dx > 1e-10 && dy > 1e-10) om = exp(0.5 * log(dy / dx) + 0.5 * log(om));
            ctl->omega = om;
            const double wp2 = pow(om, ctl->kkt_p);
            const double gz = (ez[2] + ez[7]) - ez[6];
            ctl->KKT0 = sqrt(wp2 * ez[1] + ez[5] / wp2 + gz * gz);
            ctl->KKT_prev = INFINITY;
            ctl->W = 0.0;
            ctl->t = 0;
            ctl->restarts += 1;
            ctl->restart_to = cand_cur ? 1 : 2;
        }
    }
    ctl->need_primal = ctl->done ? 0 : 1;
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
    T *x = pick(d.xb, c), *kty = pick(d.KTyb, c), *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
    for (int vb = blockIdx.x; vb < vb_n + vb_m; vb += gridDim.x) {
        if (vb < vb_n) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) {
                if (co) {
                    d.xo[j] = sel ? d.xa[j] : x[j];
                    d.KTyo[j] = sel ? d.KTya[j] : kty[j];
                }
                if (rt == 2) {
                    const T a = d.xa[j];
                    x[j] = a;
                    d.x0[j] = a;
                    kty[j] = d.KTya[j];
                } else if (rt == 1) {
                    const T a = x[j];
                    d.xa[j] = a;
                    d.x0[j] = a;
                    d.KTya[j] = kty[j];
                }
                if (np) primal_elem(d, c, tau, j, dx2);
            }
        } else {
            const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
            if (i < d.m) {
                if (co) d.yo[i] = sel ? d.ya[i] : y[i];
                if (rt == 2) {
                    const T a = d.ya[i];
                    y[i] = a;
                    d.y0[i] = a;
                    kx[i] = d.Kxa[i];
                } else if (rt == 1) {
                    const T a = y[i];
                    d.ya[i] = a;
                    d.y0[i] = a;
                    d.Kxa[i] = kx[i];
                }
            }
        }
    }
    double v[1] = {dx2};
    block_store_partials<1>(v, d.part_primal);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_partial_plain(Sliced<T> P, const T *__restrict__ x)
{
    sliced_partial(P, x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sum_slices(Sliced<T> P, T *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < P.rows) out[i] = sum_slices(P, i);
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

__global__ void k_row_absmax(const int *rp, const double *v, int nrows, double *out)
{
    const int row = blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    double a = 0.0;
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

__global__ void k_rescale_rows(const int *rp, const int *ci, double *v, int nrows, const double *rowf,
                               const double *colf)
{
    const int row = blockIdx.x * (kBlock / 64) + ((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= nrows) return;
    const double r = rowf[row];
    for (int j = rp[row] + lane; j < rp[row + 1]; j += 64) v[j] = v[j] / (r * colf[ci[j]]);
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
    hipLaunchKernelGGL(k_partial_K<T>, dim3(d.K.grid), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_partial_KT(const Dev<T> &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_partial_KT<T>, dim3(d.KT.grid), dim3(kBlock), 0, s, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dual(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_dual<T>, dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_m);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step_decide(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_decide, dim3(1), dim3(kBlock), 0, s, d.ctl, (const double *)d.part_primal,
                       (const double *)d.part_dual, g.grid);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_update<T>, dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m);
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
    hipLaunchKernelGGL(k_check_decide, dim3(1), dim3(kBlock), 0, s, d.ctl, (const double *)d.part_check, g.grid,
                       Nq, Nc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_check_apply(const Dev<T> &d, const Geo &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_apply<T>, dim3(g.grid), dim3(kBlock), 0, s, d, g.vb_n, g.vb_m);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spmv(const Sliced<T> &P, const T *in, T *out, hipStream_t s)
{
    if (P.rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_partial_plain<T>, dim3(P.grid), dim3(kBlock), 0, s, P, in);
    hipLaunchKernelGGL(k_sum_slices<T>, dim3(blocks_for(P.rows)), dim3(kBlock), 0, s, P, out);
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
    hipLaunchKernelGGL(k_row_absmax, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, v, nrows, out);
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
    hipLaunchKernelGGL(k_rescale_rows, dim3((nrows + 3) / 4), dim3(kBlock), 0, s, rp, ci, v, nrows, rowf, colf);
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
    template hipError_t launch_gather_values<T>(const double *, const int *, T *, int64_t, hipStream_t);           \
    template hipError_t launch_start<T>(const Dev<T> &, const double *, const double *, int, hipStream_t);         \
    template hipError_t launch_result<T>(const Dev<T> &, double *, double *, double *, hipStream_t);               \
    template hipError_t launch_to_double<T>(const T *, double *, int64_t, hipStream_t);                            \
    template hipError_t launch_from_double<T>(const double *, T *, int64_t, hipStream_t);

PDLP_INSTANTIATE(double)
PDLP_INSTANTIATE(float)

}  // namespace pdlp
