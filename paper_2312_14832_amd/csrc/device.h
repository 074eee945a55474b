// Device-side building blocks shared by the single-LP and the batched
// restarted-PDHG kernels: projections, deterministic reductions, the fused
// dual/primal/averaging element updates, the KKT check sums, the step-size
// and restart decisions, and the CSR-Stream row-block product.
#pragma once

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
__device__ __forceinline__ void block_store_partials(double (&v)[NV], double *out, int slot = -1)
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
        const size_t at = slot < 0 ? (size_t)blockIdx.x : (size_t)slot;
        out[at * NV + i] = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
    }
    if (slot >= 0) __syncthreads();   // the caller loops: sh is written again next round
}

// Sum np partials of NV values each inside one workgroup; every thread gets
// the same (deterministic) totals.  Partial idx starts at part[idx * stride * NV]
// (stride > 1: the partials of one instance among interleaved ones).
template <int NV>
__device__ __forceinline__ void block_sum_partials(const double *part, int np, double (&out)[NV], int stride = 1)
{
    __shared__ double sh[kBlock / 64][NV];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    // four strided partials per thread are loaded before any is added, so
    // their load latencies overlap
    constexpr int U = NV <= 2 ? 4 : 1;
    for (int b = threadIdx.x; b < np; b += U * kBlock) {
        double t[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = b + u * kBlock;
#pragma unroll
            for (int i = 0; i < NV; ++i) t[u][i] = idx < np ? part[(size_t)idx * stride * NV + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] += t[u][i];
        }
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

// Per-instance partials of a workgroup whose thread t always works for
// instance t % Bp (Bp a power of two <= kBlock; interleaved vectors of a
// shared-matrix batch): the values of the threads of one instance are added
// in a fixed order (a butterfly over the lanes of a wavefront, then the
// wavefronts in order) and stored at out[(blockIdx.x * Bp + b) * NV + k].
// With only_checking set, instance b's slot is written only while
// only_checking[b].mode != MODE_NONE.  Every thread must call it.
template <int NV>
__device__ __forceinline__ void store_inst_partials(const double (&v)[NV], int Bp, double *out,
                                                    const Ctl *only_checking = nullptr)
{
    __shared__ double sh[kBlock / 64][64];
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const int b = (int)threadIdx.x;
    const bool writer = b < Bp && (!only_checking || only_checking[b].mode != MODE_NONE);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = v[k];
        for (int off = 32; off >= Bp; off >>= 1) a += __shfl_xor(a, off);
        sh[wave][lane] = a;
        __syncthreads();
        if (writer) {
            double t = 0.0;
            if (Bp <= 64) {
                // every wavefront holds instance b's sum in lane b
                t = ((sh[0][b] + sh[1][b]) + sh[2][b]) + sh[3][b];
            } else {
                // wavefront w serves instances (64 w .. 64 w + 63) mod Bp
#pragma unroll
                for (int w = 0; w < kBlock / 64; ++w) {
                    const int base = (w * 64) & (Bp - 1);
                    if (b >= base && b < base + 64) t += sh[w][b - base];
                }
            }
            out[((size_t)blockIdx.x * Bp + b) * NV + k] = t;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// column-sliced CSR-Stream partial products
// ----------------------------------------------------------------------------

// row i of the product: the slices' partials added in slice order.  With
// the slice count NS known at compile time every load is issued before the
// first add; NS = 0 reads the count at run time.
template <int NS, typename T>
__device__ __forceinline__ T sum_slices(const Sliced<T> &P, int i)
{
    if constexpr (NS > 0) {
        T p[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) p[s] = P.part[(size_t)s * P.rows + i];
        T a = p[0];
#pragma unroll
        for (int s = 1; s < NS; ++s) a += p[s];
        return a;
    } else {
        T a = P.part[i];
        for (int s = 1; s < P.S; ++s) a += P.part[(size_t)s * P.rows + i];
        return a;
    }
}

// The total of every long row (more than kLongRow entries) inside rows
// [vb*kBlock, (vb+1)*kBlock): the whole workgroup adds the row's chunk dot
// products in a fixed order, and the thread of that row gets it in `val`
// (returns true for that thread only).  Every thread of the workgroup must
// call it with the same vb.  LONG = false (a product without long rows)
// compiles to nothing.
template <bool LONG, typename T>
__device__ __forceinline__ bool long_row_total(const Sliced<T> &P, int vb, T &val)
{
    if constexpr (!LONG) return false;
    if (P.nlong == 0) return false;
    __shared__ double sh[kBlock / 64];
    const int lo = vb * kBlock, hi = lo + kBlock;
    int a = 0, b = P.nlong;   // first long row >= lo
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (P.lrow[mid] < lo) a = mid + 1;
        else b = mid;
    }
    bool have = false;
    for (int k = a; k < P.nlong && P.lrow[k] < hi; ++k) {
        double acc = 0.0;
        for (int p = P.loff[k] + (int)threadIdx.x; p < P.loff[k + 1]; p += kBlock) acc += (double)P.lpart[p];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (P.lrow[k] - lo == (int)threadIdx.x) {
            val = (T)(((sh[0] + sh[1]) + sh[2]) + sh[3]);
            have = true;
        }
        __syncthreads();
    }
    return have;
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

// the 9 check sums of one iterate; s[0..3] rows, s[4..8] columns:
// |r_p|^2 unscaled, |r_p|^2 scaled, q'y, |y-y0|^2,
// |r_d|^2 unscaled, |r_d|^2 scaled, c'x, l'lam+ - u'lam-, |x-x0|^2.
// The *_v forms take the element's values (k = (K x)_i, g_kty = (K'y)_j);
// the array forms read them.
__device__ __forceinline__ void row_sums_v(double k, double q, double Dr, double yi, double y0i, bool ineq,
                                           double *s)
{
    double r = k - q;
    if (ineq) {
        const double t = q - k;
        r = t > 0.0 ? t : 0.0;
    }
    const double ru = r * Dr;
    s[0] += ru * ru;
    s[1] += r * r;
    s[2] += q * yi;
    const double dd = yi - y0i;
    s[3] += dd * dd;
}

__device__ __forceinline__ void col_sums_v(double cj, double lj, double uj, double Dc, double kty, double xj,
                                           double x0j, double *s)
{
    const bool lf = isfinite(lj), uf = isfinite(uj);
    const double g = cj - kty;
    const double lam = proj_lambda(g, lf, uf);
    const double rd = g - lam;
    const double rdu = rd * Dc;
    s[4] += rdu * rdu;
    s[5] += rd * rd;
    s[6] += cj * xj;
    double b = 0.0;
    if (lf && lam > 0.0) b += lj * lam;
    if (uf && lam < 0.0) b += uj * lam;
    s[7] += b;
    const double dd = xj - x0j;
    s[8] += dd * dd;
}

template <typename T>
__device__ __forceinline__ void row_sums(const Dev<T> &d, int i, int m1, const T *y, const T *kx, double *s)
{
    row_sums_v((double)kx[i], (double)d.qs[i], d.Dr[i], (double)y[i], (double)d.y0[i], i >= m1, s);
}

template <typename T>
__device__ __forceinline__ void col_sums(const Dev<T> &d, int j, const T *x, const T *kty, double *s)
{
    col_sums_v((double)d.cs[j], (double)d.ls[j], (double)d.us[j], d.Dc[j], (double)kty[j], (double)x[j],
               (double)d.x0[j], s);
}

// The 4 ray sums of the current iterate (difference from the anchor, taken
// as a Farkas ray on the unscaled problem; scalings cancel in the
// objectives): s[0] c'd, s[1] |(A d, max(-G d, 0), bound-cone violation)|^2,
// s[2] q'w + l'lam+ - u'lam- with lam = proj_Lambda(-K'w),
// s[3] |(-K'w - lam, min(w_G, 0))|^2; d = (x - x0)/Dc, w = (y - y0)/Dr.
__device__ __forceinline__ void ray_row_sums_v(double kx, double kx0, double Dr, double yi, double y0i, double q,
                                               bool ineq, double *s)
{
    const double kd = (kx - kx0) * Dr;
    double r = kd;
    if (ineq) r = -kd > 0.0 ? -kd : 0.0;
    s[1] += r * r;
    const double dy = yi - y0i;
    s[2] += q * dy;
    if (ineq) {
        const double w = dy / Dr;
        if (w < 0.0) s[3] += w * w;
    }
}

__device__ __forceinline__ void ray_col_sums_v(double cj, double lj, double uj, double Dc, double xj, double x0j,
                                               double kty, double kty0, double *s)
{
    const bool lf = isfinite(lj), uf = isfinite(uj);
    const double dx = xj - x0j;
    s[0] += cj * dx;
    const double dj = dx / Dc;
    if ((lf && dj < 0.0) || (uf && dj > 0.0)) s[1] += dj * dj;
    const double g = kty0 - kty;
    const double lam = proj_lambda(g, lf, uf);
    const double r = (g - lam) * Dc;
    s[3] += r * r;
    if (lf && lam > 0.0) s[2] += lj * lam;
    if (uf && lam < 0.0) s[2] += uj * lam;
}

template <typename T>
__device__ __forceinline__ void ray_row_sums(const Dev<T> &d, int i, int m1, const T *y, const T *kx, double *s)
{
    ray_row_sums_v((double)kx[i], (double)d.Kx0[i], d.Dr[i], (double)y[i], (double)d.y0[i], (double)d.qs[i],
                   i >= m1, s);
}

template <typename T>
__device__ __forceinline__ void ray_col_sums(const Dev<T> &d, int j, const T *x, const T *kty, double *s)
{
    ray_col_sums_v((double)d.cs[j], (double)d.ls[j], (double)d.us[j], d.Dc[j], (double)x[j], (double)d.x0[j],
                   (double)kty[j], (double)d.KTy0[j], s);
}

// Adaptive step-size test (PDLP's rule; the paper uses eta without stating
// the rule): eta_bar = (omega|dx|^2 + |dy|^2/omega) / (2|dy.K dx|),
// eta' = min((1-kk^-0.3) eta_bar, (1+kk^-0.6) eta) with kk counting from 2;
// accept iff eta <= eta_bar.  Called by one thread per LP.
// The two factors of the step rule at accepted count k: 1 - kk^-0.3 and
// 1 + kk^-0.6 with kk = k + 2.
__device__ inline void step_factors(long long k, double &f_lo, double &f_hi)
{
    const double kk = (double)(k + 1) + 1.0;
    f_lo = 1.0 - pow(kk, -0.3);
    f_hi = 1.0 + pow(kk, -0.6);
}

// The adaptive step rule of one attempt with step size eta (the factors of
// the current accepted count given, step_factors): 1 accept, 0 reject, -1 a
// NaN in the test; eta_new is the next step size (eta itself on a NaN or
// with a fixed step).
__device__ inline int step_rule(double eta, double omega, int fixed_step, double dx2, double dy2, double inter,
                                double f_lo, double f_hi, double &eta_new)
{
    eta_new = eta;
    if (fixed_step) return 1;
    const double N = omega * dx2 + dy2 / omega;
    const double D = 2.0 * fabs(inter);
    if (isnan(N) || isnan(D)) return -1;
    const double eta_bar = D > 0.0 ? N / D : INFINITY;
    const double lo = f_lo * eta_bar;
    const double hi = f_hi * eta;
    eta_new = lo < hi ? lo : hi;
    return eta <= eta_bar ? 1 : 0;
}

// The check mode after an accepted step that brings the accepted count to k
__device__ inline int mode_after_accept(long long k, int check_every, long long max_iters)
{
    return (k % check_every == 0 || k >= max_iters) ? MODE_CHECK : MODE_NONE;
}

// The step decision with the factors of the current accepted count given
// (step_factors), for callers that tabulate them ahead.
__device__ inline void step_decision_f(Ctl *ctl, double dx2, double dy2, double inter, double f_lo, double f_hi)
{
    const double eta = ctl->eta;
    double eta_new;
    ctl->attempts += 1;
    const int rule = step_rule(eta, ctl->omega, ctl->fixed_step, dx2, dy2, inter, f_lo, f_hi, eta_new);
    if (rule < 0) {
        ctl->numerical = 1;
        ctl->accepted = 0;
        ctl->mode = MODE_CHECK;
        return;
    }
    const bool accept = rule == 1;
    if (accept) {
        ctl->W += eta;
        ctl->avg_w = eta / ctl->W;
        ctl->eta_last = eta;
        ctl->k += 1;
        ctl->t += 1;
        ctl->cur ^= 1;
        ctl->accepted = 1;
        ctl->mode = mode_after_accept(ctl->k, ctl->check_every, ctl->max_iters);
    } else {
        ctl->accepted = 0;
        ctl->mode = MODE_NONE;
    }
    ctl->eta = eta_new;
}

__device__ inline void step_decision(Ctl *ctl, double dx2, double dy2, double inter)
{
    double f_lo = 0.0, f_hi = 0.0;
    if (!ctl->fixed_step) step_factors(ctl->k, f_lo, f_hi);
    step_decision_f(ctl, dx2, dy2, inter, f_lo, f_hi);
}

// The termination quantities (unscaled) and KKT_omega (scaled) of the
// current (z = 0) and the averaged (z = 1) iterate from their 9 check sums
// each, stored in the controller; rel[z] is the relative KKT error (NaN if
// any part is NaN).
__device__ inline void check_quantities(Ctl *ctl, const double *S, double Nq, double Nc, double (&rel)[2],
                                        double (&kkt)[2])
{
    const double wp = pow(ctl->omega, ctl->kkt_p);
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
}

// End the solve with `status`, returning iterate `sel` (0 current, 1 average).
__device__ inline void finish_ctl(Ctl *ctl, int status, int sel)
{
    ctl->status = status;
    ctl->out_sel = sel;
    ctl->copy_out = 1;
    ctl->done = 1;
    ctl->out_rel_p = ctl->rel_p[sel];
    ctl->out_rel_d = ctl->rel_d[sel];
    ctl->out_rel_g = ctl->rel_g[sel];
    ctl->out_pobj = ctl->pobj[sel];
    ctl->out_dobj = ctl->dobj[sel];
}

// Termination (the three relative criteria on the unscaled problem), then
// the ray certificates of infeasibility, candidate choice and restart
// conditions 1-3 on KKT_omega (scaled problem), primal-weight update.  S
// holds the 9 check sums of the current iterate then the 9 of the average,
// R the 4 ray sums.  With confirm_on (mixed precision) a passed termination
// test only stops the loop with `confirm` set: the host redoes the sums with
// FP64 products (confirm_decision) and either ends the solve or runs this
// decision again with `veto`, which skips the termination test once.
// Called by one thread per LP.
__device__ inline void check_decision(Ctl *ctl, const double *S, const double *R, double Nq, double Nc)
{
    double rel[2], kkt[2];
    check_quantities(ctl, S, Nq, Nc, rel, kkt);
    const int mode = ctl->mode;
    const int veto = ctl->veto;
    ctl->veto = 0;
    ctl->restart_to = 0;
    ctl->copy_out = 0;
    ctl->need_primal = 0;
    if (mode == MODE_INIT) {
        ctl->KKT0 = kkt[0];
        ctl->KKT_prev = INFINITY;
        ctl->need_primal = 1;
        return;
    }
    if (ctl->numerical || isnan(rel[0]) || isnan(rel[1])) {
        finish_ctl(ctl, LP_NUMERICAL, 0);
        return;
    }
    const int use_avg = rel[1] < rel[0] ? 1 : 0;
    if ((rel[0] <= ctl->tol || rel[1] <= ctl->tol) && !veto) {
        if (ctl->confirm_on) {
            ctl->confirm = 1;
            ctl->conf_mode = mode;
            ctl->done = 1;
            return;
        }
        finish_ctl(ctl, LP_OPTIMAL, use_avg);
        return;
    }
    if (ctl->infeas_tol > 0.0) {
        const double *r = R;
        int st = 0;
        if (r[2] > 0.0 && sqrt(r[3]) <= ctl->infeas_tol * r[2]) st = LP_PRIMAL_INFEASIBLE;
        else if (r[0] < 0.0 && sqrt(r[1]) <= ctl->infeas_tol * -r[0]) st = LP_DUAL_INFEASIBLE;
        if (st) {
            finish_ctl(ctl, st, 0);
            ctl->out_sel = 2;   // the rays
            ctl->out_pobj = r[0];
            ctl->out_dobj = r[2];
            return;
        }
    }
    int at_limit = 0;
    if (mode == MODE_FINAL) at_limit = ctl->final_status;
    else if (ctl->k >= ctl->max_iters) at_limit = LP_ITERATION_LIMIT;
    if (at_limit) finish_ctl(ctl, at_limit, use_avg);
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

// Mixed precision: the FP64 re-check of a passed termination test.  S holds
// the 9 check sums of the current iterate and of the average computed with
// FP64 products of the FP64 scaled matrix.  If either iterate meets the
// criteria the solve ends OPTIMAL with the FP64 quantities; otherwise the
// loop resumes and the check decision runs again without its termination
// test (veto).  Called by one thread.
__device__ inline void confirm_decision(Ctl *ctl, const double *S, double Nq, double Nc)
{
    double rel[2], kkt[2];
    check_quantities(ctl, S, Nq, Nc, rel, kkt);
    ctl->confirm = 0;
    ctl->confirms += 1;
    ctl->mode = ctl->conf_mode;
    const int use_avg = rel[1] < rel[0] ? 1 : 0;
    if (!isnan(rel[0]) && !isnan(rel[1]) && (rel[0] <= ctl->tol || rel[1] <= ctl->tol)) {
        finish_ctl(ctl, LP_OPTIMAL, use_avg);
        return;
    }
    ctl->done = 0;
    ctl->veto = 1;
}

// restart / output bookkeeping on column j (current buffer c):
// rt = 2 restart to the average, 1 restart to the current point (the anchor
// and its product follow); co copies the chosen point (sel: 0 current,
// 1 average, 2 the rays: differences from the anchor, with K'yo set so that
// the result's lam is proj_Lambda(-K'w)) to the output buffers; np computes
// the next primal trial with step tau
template <typename T>
__device__ __forceinline__ void apply_col(const Dev<T> &d, int j, int c, int rt, int co, int sel, int np, T tau,
                                          double &dx2)
{
    T *x = pick(d.xb, c), *kty = pick(d.KTyb, c);
    if (co) {
        if (sel == 2) {
            d.xo[j] = x[j] - d.x0[j];
            d.KTyo[j] = d.cs[j] + (kty[j] - d.KTy0[j]);
        } else {
            d.xo[j] = sel ? d.xa[j] : x[j];
            d.KTyo[j] = sel ? d.KTya[j] : kty[j];
        }
    }
    if (rt == 2) {
        const T a = d.xa[j], b = d.KTya[j];
        x[j] = a;
        d.x0[j] = a;
        kty[j] = b;
        d.KTy0[j] = b;
    } else if (rt == 1) {
        const T a = x[j], b = kty[j];
        d.xa[j] = a;
        d.x0[j] = a;
        d.KTya[j] = b;
        d.KTy0[j] = b;
    }
    if (np) primal_elem(d, c, tau, j, dx2);
}

template <typename T>
__device__ __forceinline__ void apply_row(const Dev<T> &d, int i, int c, int rt, int co, int sel)
{
    T *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
    if (co) d.yo[i] = sel == 2 ? y[i] - d.y0[i] : (sel ? d.ya[i] : y[i]);
    if (rt == 2) {
        const T a = d.ya[i], b = d.Kxa[i];
        y[i] = a;
        d.y0[i] = a;
        kx[i] = b;
        d.Kx0[i] = b;
    } else if (rt == 1) {
        const T a = y[i], b = kx[i];
        d.ya[i] = a;
        d.y0[i] = a;
        d.Kxa[i] = b;
        d.Kx0[i] = b;
    }
}

// averaging of row i after an accepted step (weight w)
template <typename T>
__device__ __forceinline__ void average_row(const Dev<T> &d, int i, int c, T w)
{
    const T *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
    const T a = d.ya[i];
    d.ya[i] = a + w * (y[i] - a);
    const T b = d.Kxa[i];
    d.Kxa[i] = b + w * (kx[i] - b);
}

// Row extents for stream_block, of row r of a block holding rows [r0, r1)
// and entries [b, e).  RowsPlain: a CSR's own row pointers.  RowsRel: each
// row's start relative to its block's first entry in 16 bits (the end of the
// block's last row is e); every load stays inside rows [r0, r1).
struct RowsPlain {
    const int *__restrict__ rp;
    __device__ __forceinline__ int start(int r, int) const { return rp[r]; }
    __device__ __forceinline__ int end(int r, int, int, int) const { return rp[r + 1]; }
};
struct RowsRel {
    const unsigned short *__restrict__ ro;
    __device__ __forceinline__ int start(int r, int b) const { return b + (int)ro[r]; }
    __device__ __forceinline__ int end(int r, int r1, int b, int e) const
    {
        const int nx = b + (int)ro[min(r + 1, r1 - 1)];
        return r + 1 < r1 ? nx : e;
    }
};

// LDS of the split row sums of a block of short rows (stream_block, SPLIT).
// Thread t walks the products of chunk t, entries [8t, 8t + 8) of the block.
template <typename T>
struct SplitLds {
    unsigned short rend[kStreamRB];   // each row's end, relative to the block's first entry
    unsigned short head[kBlock];      // the row holding each chunk's first entry
    unsigned short crow[kBlock];      // the row a chunk's walk leaves open (kNoRow: none)
    T cval[kBlock];                   // that row's sum over the chunk
};
constexpr unsigned short kNoRow = 0xFFFF;

// The split sums of stream_block (SPLIT, a block of short rows, rows
// [r0, r1) with entries [b, b + cnt)), after the products, row ends and chunk
// heads are in LDS and a barrier; rs, re hold the extents of the thread's
// rows r0 + t + kBlock j, which it stores to out at the end.  See
// stream_block.
template <int U, int RU, typename T>
__device__ __forceinline__ void split_row_sums(const int (&rs)[RU], const int (&re)[RU], int r0, int r1, int b,
                                               int cnt, T *__restrict__ out, T *prod, SplitLds<T> *L)
{
    const int t = (int)threadIdx.x, c0 = t * U, c1 = min(c0 + U, cnt);
    int prow = -1;   // the crossing row this thread finishes, if any
    T pval = T(0);
    if (c0 < cnt) {
        int i = L->head[t];
        int is = i ? (int)L->rend[i - 1] : 0, ie = L->rend[i];
        const bool crossing = is < c0;
        bool first = true;
        T acc = T(0);
        for (int p = c0; p < c1; ++p) {
            if (p >= ie) {   // row i ended before entry p
                if (first && crossing) {
                    prow = i;
                    pval = acc;
                } else {
                    prod[is] = acc;
                }
                first = false;
                acc = T(0);
                do {   // on to the row holding p (past empty rows)
                    ++i;
                    is = ie;
                    ie = L->rend[i];
                } while (ie <= p);
            }
            acc += prod[p];
        }
        if (ie == c1) {   // the last row ends with the chunk
            if (first && crossing) {
                prow = i;
                pval = acc;
            } else {
                prod[is] = acc;
            }
            L->crow[t] = kNoRow;
        } else {
            L->crow[t] = (unsigned short)i;
            L->cval[t] = acc;
        }
    } else {
        L->crow[t] = kNoRow;
    }
    __syncthreads();
    if (prow >= 0) {   // the open parts of the chunks before this one, nearest first
        T tot = pval;
        for (int u = t - 1; u >= 0 && (int)L->crow[u] == prow; --u) tot = L->cval[u] + tot;
        prod[prow ? (int)L->rend[prow - 1] : 0] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RU; ++j) {
        const int r = r0 + t + j * kBlock;
        if (r < r1) out[r] = rs[j] == re[j] ? T(0) : prod[rs[j] - b];
    }
}

// CSR-Stream sums of one row block: rows [r0, r1) whose entries are [b, e),
// row extents from rows (RowsPlain or RowsRel).  Products are staged in LDS.
// In a block of short rows (at most kStreamRB) each thread sums every
// kBlock-th row in index order; with SPLIT the sums are split by entries
// instead, so that a few long rows among short ones do not hold up their
// wavefront: thread t adds up the products of chunk t (8 entries) row by
// row, a row that lies wholly in the chunk is finished there, and a row that
// crosses chunks is finished by the thread holding its last entry, which adds
// the open parts of the chunks before its own in a fixed order.  Every
// finished sum is parked in the LDS slot of its row's first product (a slot
// the chunk's own walk has already read, or, for a crossing row, after a
// barrier), then every thread stores its rows as before.  In a block of long
// rows (wave set, at most kBlock/64) each wavefront sums one row, lanes
// striding and a butterfly combining them.  A block of one row longer than
// kStreamNB is summed by the whole workgroup.  Every thread of the workgroup
// must call it.
template <bool SPLIT = false, typename T, typename ROWS>
__device__ __forceinline__ void stream_block(const ROWS &rows, const int *__restrict__ ci,
                                             const T *__restrict__ v, const T *__restrict__ x, int r0, int r1,
                                             bool wave, int b, int e, T *__restrict__ out, T *prod, double *red,
                                             SplitLds<T> *L = nullptr)
{
    const int cnt = e - b;
    // a multi-row block never exceeds kStreamNB nonzeros, only a single row can
    if (cnt <= kStreamNB) {
        // Straight-line phases so that a thread's loads overlap: every value,
        // column and row pointer it owns, then every gather, then the
        // products.  Slots past the block's end re-read its last entry or row
        // (same cache line) rather than branch, which would serialise them.
        constexpr int U = kStreamNB / kBlock, RU = kStreamRB / kBlock;
        int col[U], rs[RU], re[RU];
        T a[U], g[U];
        if (cnt > 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = min((int)threadIdx.x + u * kBlock, cnt - 1);
                col[u] = __builtin_nontemporal_load(ci + b + t);
                a[u] = __builtin_nontemporal_load(v + b + t);
            }
        }
#pragma unroll
        for (int j = 0; j < RU; ++j) {
            const int r = min(r0 + (int)threadIdx.x + j * kBlock, r1 - 1);
            rs[j] = rows.start(r, b);
            re[j] = rows.end(r, r1, b, e);
        }
        if (cnt > 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) g[u] = x[col[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = (int)threadIdx.x + u * kBlock;
                if (t < cnt) prod[t] = a[u] * g[u];
            }
        }
        if constexpr (SPLIT) {
            if (!wave) {   // row ends, and the row of each chunk's first entry
#pragma unroll
                for (int j = 0; j < RU; ++j) {
                    const int r = (int)threadIdx.x + j * kBlock;
                    if (r0 + r < r1) {
                        const int s = rs[j] - b, f = re[j] - b;
                        L->rend[r] = (unsigned short)f;
                        for (int k = (s + U - 1) / U; k * U < f; ++k) L->head[k] = (unsigned short)r;
                    }
                }
            }
        }
        __syncthreads();
        if (SPLIT && !wave) {
            split_row_sums<U>(rs, re, r0, r1, b, cnt, out, prod, L);
        } else if (!wave) {
#pragma unroll
            for (int j = 0; j < RU; ++j) {
                const int r = r0 + (int)threadIdx.x + j * kBlock;
                if (r < r1) {
                    T acc = T(0);
                    for (int p = rs[j] - b; p < re[j] - b; ++p) acc += prod[p];
                    out[r] = acc;
                }
            }
        } else {
            const int r = r0 + ((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
            if (r < r1) {   // uniform over the wavefront
                const int p1 = rows.end(r, r1, b, e) - b;
                T acc = T(0);
                for (int p = rows.start(r, b) - b + lane; p < p1; p += 64) acc += prod[p];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
                if (lane == 0) out[r] = acc;
            }
        }
        __syncthreads();
    } else {
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

// Dot product of entries [b, e) of one slice (1 <= e - b <= kStreamNB): a
// chunk of a long row.  Same load / gather / product phases as stream_block,
// products added in registers, then across the workgroup in a fixed order;
// every thread gets the result.  Every thread of the workgroup must call it.
template <typename T>
__device__ __forceinline__ T chunk_dot(const int *__restrict__ ci, const T *__restrict__ v, const T *__restrict__ x,
                                       int b, int e, double *red)
{
    constexpr int U = kStreamNB / kBlock;
    const int cnt = e - b;
    int col[U];
    T a[U], g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = min((int)threadIdx.x + u * kBlock, cnt - 1);
        col[u] = __builtin_nontemporal_load(ci + b + t);
        a[u] = __builtin_nontemporal_load(v + b + t);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = x[col[u]];
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
        if ((int)threadIdx.x + u * kBlock < cnt) acc += a[u] * g[u];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (double)acc;
    __syncthreads();
    const T r = (T)(((red[0] + red[1]) + red[2]) + red[3]);
    __syncthreads();
    return r;
}

// The 18 check sums of the current and the averaged iterate over the
// elements this workgroup owns in a grid-stride walk of the n-chunks then the
// m-chunks (the same walk as the elementwise solver kernels, so a thread
// only reads entries it wrote itself earlier in the same kernel).
template <typename T>
__device__ __forceinline__ void check_sums_pass(const Dev<T> &d, int c, int vb_n, int vb_m, double (&s)[kCheckSums])
{
#pragma unroll
    for (int i = 0; i < kCheckSums; ++i) s[i] = 0.0;
    const T *x = pick(d.xb, c), *kty = pick(d.KTyb, c), *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
    for (int vb = blockIdx.x; vb < vb_n + vb_m; vb += gridDim.x) {
        if (vb < vb_n) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) {
                col_sums(d, j, x, kty, s);
                col_sums(d, j, (const T *)d.xa, (const T *)d.KTya, s + 9);
            }
        } else {
            const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
            if (i < d.m) {
                row_sums(d, i, d.m1, y, kx, s);
                row_sums(d, i, d.m1, (const T *)d.ya, (const T *)d.Kxa, s + 9);
            }
        }
    }
}

// The 4 ray sums over the same walk, after the check sums are stored.
template <typename T>
__device__ __forceinline__ void ray_sums_pass(const Dev<T> &d, int c, int vb_n, int vb_m, double (&s)[kRaySums])
{
#pragma unroll
    for (int i = 0; i < kRaySums; ++i) s[i] = 0.0;
    const T *x = pick(d.xb, c), *kty = pick(d.KTyb, c), *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
    for (int vb = blockIdx.x; vb < vb_n + vb_m; vb += gridDim.x) {
        if (vb < vb_n) {
            const int j = vb * kBlock + (int)threadIdx.x;
            if (j < d.n) ray_col_sums(d, j, x, kty, s);
        } else {
            const int i = (vb - vb_n) * kBlock + (int)threadIdx.x;
            if (i < d.m) ray_row_sums(d, i, d.m1, y, kx, s);
        }
    }
}

// One column slice's partial products (see Sliced): workgroup b takes slice
// b % S and walks that slice's row blocks with stride gridDim / S.  LONG:
// the product has long rows, so some blocks are chunks of one.
template <bool LONG, bool SPLIT = false, typename T>
__device__ __forceinline__ void sliced_partial(const Sliced<T> &P, const T *__restrict__ x)
{
    __shared__ T prod[kStreamNB];
    __shared__ double red[kBlock / 64];
    SplitLds<T> *split = nullptr;
    if constexpr (SPLIT) {
        __shared__ SplitLds<T> split_lds;
        split = &split_lds;
    }
    const int S = P.S;
    const int s = (int)blockIdx.x % S;
    const int chunk0 = (int)blockIdx.x / S, stride = (int)gridDim.x / S;
    const RowsRel rows{P.ro + (size_t)s * P.rows};
    T *out = P.part + (size_t)s * P.rows;
    const int nblk = P.boff[s + 1] - P.boff[s];
    const int4 *bd = P.blk + P.boff[s];
    for (int k = chunk0; k < nblk; k += stride) {
        const int4 q = bd[k];
        if constexpr (LONG) {
            if (q.x < 0) {   // a chunk of a long row
                const T r = chunk_dot(P.ci, P.v, x, q.z, q.w, red);
                if (threadIdx.x == 0) P.lpart[~q.x] = r;
                continue;
            }
        }
        const bool wave = q.y < 0;
        stream_block<SPLIT>(rows, P.ci, P.v, x, q.x, wave ? ~q.y : q.y, wave, q.z, q.w, out, prod, red, split);
    }
}

}  // namespace pdlp
