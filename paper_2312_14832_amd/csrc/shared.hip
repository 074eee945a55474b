// Batched restarted PDHG over one shared matrix (a parametric family: K
// fixed, c, q, l, u per instance).  The slot structure is the single-LP
// solver's, with one difference that matters for memory traffic: each sparse
// product is an SpMM over the interleaved iterates, so K is read once per
// product for all instances, and the gather of x[j][0..Bp) for a nonzero
// K_ij is a contiguous run of Bp values rather than one value per instance.
// Every per-instance quantity (step size, primal weight, restarts,
// termination) lives in the instance's own controller; a lane's instance is
// fixed for the whole kernel (thread t always serves instance t % Bp), so
// per-instance partial sums need no atomics.
#include "device.h"

#include <algorithm>

namespace pdlp {

// One row of the SpMM for instance b: sum over the row's entries [rs, re)
// of v[p] x[ci[p]][b], in entry order.  Eight entries at a time in three
// straight-line phases (indices and values, then the eight gathers, then the
// products), so eight gathers of the row are in flight at once; slots past
// the row's end re-read its last entry and are masked out of the sum.
template <typename T>
__device__ __forceinline__ T spmm_row(const int *__restrict__ ci, const T *__restrict__ v, const T *__restrict__ x,
                                      int rs, int re, int lgB, int b)
{
    constexpr int U = 8;
    T acc = T(0);
    for (int p = rs; p < re; p += U) {
        int c[U];
        T a[U], g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = min(p + u, re - 1);
            c[u] = ci[t];
            a[u] = v[t];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = x[((size_t)c[u] << lgB) + b];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p + u < re) acc += a[u] * g[u];
    }
    return acc;
}

// K~ x' for every instance fused with the dual step: element e = i * Bp + b.
// The step's own operands are loaded before the row's product so their
// latency overlaps the gathers.  Workgroup 0 lowers the check gate (this
// slot's step decisions raise it).
template <typename T>
__global__ __launch_bounds__(kBlock) void sk_dual(SDev<T> S)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *S.gate = 0;
    const int b = (int)threadIdx.x & (S.Bp - 1);
    const Ctl *ctl = S.ctl + b;
    const Dev<T> &d = S.d;
    double v[2] = {0.0, 0.0};
    if (!ctl->done) {
        const int c = ctl->cur;
        const T *x = pick(d.xb, c ^ 1);
        const T *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
        T *yn = pick(d.yb, c ^ 1), *kxn = pick(d.Kxb, c ^ 1);
        const T sigma = (T)(ctl->eta * ctl->omega);
        const int total = S.m << S.lgB;
        for (int e = (int)(blockIdx.x * kBlock + threadIdx.x); e < total; e += (int)(gridDim.x * kBlock)) {
            const int i = e >> S.lgB;
            const T yo = y[e], ko = kx[e], qi = d.qs[e];
            const T s = spmm_row(S.kci, S.kv, x, S.krp[i], S.krp[i + 1], S.lgB, b);
            // the dual step of DualEpi
            T val = yo + sigma * (qi - T(2) * s + ko);
            if (e >= d.m1 && val < T(0)) val = T(0);
            yn[e] = val;
            kxn[e] = s;
            const double dd = (double)val - (double)yo;
            v[0] += dd * dd;
            v[1] += dd * ((double)s - (double)ko);
        }
    }
    store_inst_partials<2>(v, S.Bp, d.part_dual);
}

// one workgroup per instance
template <typename T>
__global__ __launch_bounds__(kBlock) void sk_step_decide(SDev<T> S)
{
    const int b = (int)blockIdx.x;
    Ctl *ctl = S.ctl + b;
    if (ctl->done) {
        if (threadIdx.x == 0) ctl->mode = MODE_NONE;
        return;
    }
    double a[1], c2[2];
    block_sum_partials<1>(S.d.part_primal + b, S.grid, a, S.Bp);
    block_sum_partials<2>(S.d.part_dual + 2 * (size_t)b, S.grid_m, c2, S.Bp);
    if (threadIdx.x == 0) {
        step_decision(ctl, a[0], c2[0], c2[1]);
        if (ctl->mode != MODE_NONE) atomicExch(S.gate, 1);
    }
}

// K~' y' for every accepted instance fused with the averages and the next
// primal trial (or, after a rejection, the new trial from the same point);
// the m-side averages follow in the same walk.
template <typename T>
__global__ __launch_bounds__(kBlock) void sk_update(SDev<T> S)
{
    const int b = (int)threadIdx.x & (S.Bp - 1);
    const Ctl *ctl = S.ctl + b;
    const Dev<T> &d = S.d;
    double v[1] = {0.0};
    if (!ctl->done) {
        const int c = ctl->cur;
        const T tau = (T)(ctl->eta / ctl->omega);
        const int nt = S.n << S.lgB, mt = S.m << S.lgB;
        const int e0 = (int)(blockIdx.x * kBlock + threadIdx.x), stride = (int)(gridDim.x * kBlock);
        if (!ctl->accepted) {
            for (int e = e0; e < nt; e += stride) primal_elem(d, c, tau, e, v[0]);
        } else {
            const T *x = pick(d.xb, c), *y = pick(d.yb, c);
            T *kty = pick(d.KTyb, c), *xn = pick(d.xb, c ^ 1);
            const T w = (T)ctl->avg_w;
            const bool primal = ctl->mode == MODE_NONE;
            for (int e = e0; e < nt; e += stride) {
                const int j = e >> S.lgB;
                const T xj = x[e], a = d.xa[e], bb = d.KTya[e];
                const T cj = d.cs[e], lj = d.ls[e], uj = d.us[e];
                const T s = spmm_row(S.tci, S.tv, y, S.trp[j], S.trp[j + 1], S.lgB, b);
                // the averages and next primal trial of UpdateEpi
                kty[e] = s;
                d.xa[e] = a + w * (xj - a);
                d.KTya[e] = bb + w * (s - bb);
                if (primal) {
                    const T nv = clampv(xj - tau * (cj - s), lj, uj);
                    xn[e] = nv;
                    const double dd = (double)nv - (double)xj;
                    v[0] += dd * dd;
                }
            }
            for (int e = e0; e < mt; e += stride) average_row(d, e, c, w);
        }
    }
    store_inst_partials<1>(v, S.Bp, d.part_primal);
}

// The 18 check sums and 4 ray sums of every instance in a check, over the
// same walk as sk_update.  Gated inside the solve loop.
template <typename T>
__global__ __launch_bounds__(kBlock) void sk_check_reduce(SDev<T> S, int gated)
{
    if (gated && *S.gate == 0) return;
    const int b = (int)threadIdx.x & (S.Bp - 1);
    const Ctl *ctl = S.ctl + b;
    const Dev<T> &d = S.d;
    double s[kCheckSums], r[kRaySums];
#pragma unroll
    for (int k = 0; k < kCheckSums; ++k) s[k] = 0.0;
#pragma unroll
    for (int k = 0; k < kRaySums; ++k) r[k] = 0.0;
    if (ctl->mode != MODE_NONE && !ctl->done) {
        const int c = ctl->cur;
        const T *x = pick(d.xb, c), *kty = pick(d.KTyb, c), *y = pick(d.yb, c), *kx = pick(d.Kxb, c);
        const int nt = S.n << S.lgB, mt = S.m << S.lgB;
        const int e0 = (int)(blockIdx.x * kBlock + threadIdx.x), stride = (int)(gridDim.x * kBlock);
        for (int e = e0; e < nt; e += stride) {
            col_sums(d, e, x, kty, s);
            col_sums(d, e, (const T *)d.xa, (const T *)d.KTya, s + 9);
            ray_col_sums(d, e, x, kty, r);
        }
        for (int e = e0; e < mt; e += stride) {
            row_sums(d, e, d.m1, y, kx, s);
            row_sums(d, e, d.m1, (const T *)d.ya, (const T *)d.Kxa, s + 9);
            ray_row_sums(d, e, d.m1, y, kx, r);
        }
    }
    store_inst_partials<kCheckSums>(s, S.Bp, d.part_check);
    store_inst_partials<kRaySums>(r, S.Bp, d.part_ray);
}

// one workgroup per instance
template <typename T>
__global__ __launch_bounds__(kBlock) void sk_check_decide(SDev<T> S, int gated)
{
    if (gated && *S.gate == 0) return;
    const int b = (int)blockIdx.x;
    Ctl *ctl = S.ctl + b;
    if (ctl->mode == MODE_NONE || ctl->done) return;
    double Sm[kCheckSums], R[kRaySums];
    block_sum_partials<kCheckSums>(S.d.part_check + (size_t)kCheckSums * b, S.grid, Sm, S.Bp);
    block_sum_partials<kRaySums>(S.d.part_ray + (size_t)kRaySums * b, S.grid, R, S.Bp);
    if (threadIdx.x == 0) check_decision(ctl, Sm, R, S.Nq[b], S.Nc[b]);
}

// restart copies, output copy and next primal trial of every instance in a
// check; its |x'' - x|^2 partial replaces the one sk_update left for it
template <typename T>
__global__ __launch_bounds__(kBlock) void sk_check_apply(SDev<T> S, int gated)
{
    if (gated && *S.gate == 0) return;
    const int b = (int)threadIdx.x & (S.Bp - 1);
    const Ctl *ctl = S.ctl + b;
    const Dev<T> &d = S.d;
    double v[1] = {0.0};
    if (ctl->mode != MODE_NONE) {
        const int c = ctl->cur, rt = ctl->restart_to, co = ctl->copy_out, sel = ctl->out_sel;
        const int np = ctl->need_primal;
        const T tau = (T)(ctl->eta / ctl->omega);
        const int nt = S.n << S.lgB, mt = S.m << S.lgB;
        const int e0 = (int)(blockIdx.x * kBlock + threadIdx.x), stride = (int)(gridDim.x * kBlock);
        for (int e = e0; e < nt; e += stride) apply_col(d, e, c, rt, co, sel, np, tau, v[0]);
        for (int e = e0; e < mt; e += stride) apply_row(d, e, c, rt, co, sel);
    }
    store_inst_partials<1>(v, S.Bp, d.part_primal, S.ctl);
}

// a plain product for every instance (start, resume and the anchor's products)
template <typename T, int WHICH>
__global__ __launch_bounds__(kBlock) void sk_product(SDev<T> S, const T *__restrict__ in, T *__restrict__ out)
{
    const int *rp = WHICH ? S.trp : S.krp, *ci = WHICH ? S.tci : S.kci;
    const T *v = WHICH ? S.tv : S.kv;
    const int total = (WHICH ? S.n : S.m) << S.lgB;
    const int b = (int)threadIdx.x & (S.Bp - 1);
    for (int e = (int)(blockIdx.x * kBlock + threadIdx.x); e < total; e += (int)(gridDim.x * kBlock))
        out[e] = spmm_row(ci, v, in, rp[e >> S.lgB], rp[(e >> S.lgB) + 1], S.lgB, b);
}

template <typename T>
__global__ void sk_extract(const T *src, int lgB, int b, double *dst, int rows)
{
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (i < rows) dst[i] = (double)src[((size_t)i << lgB) + b];
}

template <typename T>
__global__ void sk_insert(const double *src, int lgB, int b, T *dst, int rows)
{
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (i < rows) dst[((size_t)i << lgB) + b] = (T)src[i];
}

__global__ void sk_set_final(Ctl *ctl, int Bp, int status)
{
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (i < Bp && !ctl[i].done) {
        ctl[i].mode = MODE_FINAL;
        ctl[i].final_status = status;
    }
}

// ----------------------------------------------------------------------------

namespace {
inline dim3 nblocks(int64_t len) { return dim3((unsigned)((len + kBlock - 1) / kBlock > 0 ? (len + kBlock - 1) / kBlock : 1)); }
}  // namespace

template <typename T>
hipError_t launch_shared_check(const SDev<T> &S, int gated, hipStream_t s)
{
    hipLaunchKernelGGL(sk_check_reduce<T>, dim3(S.grid), dim3(kBlock), 0, s, S, gated);
    hipLaunchKernelGGL(sk_check_decide<T>, dim3(S.Bp), dim3(kBlock), 0, s, S, gated);
    hipLaunchKernelGGL(sk_check_apply<T>, dim3(S.grid), dim3(kBlock), 0, s, S, gated);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_shared_apply(const SDev<T> &S, hipStream_t s)
{
    hipLaunchKernelGGL(sk_check_apply<T>, dim3(S.grid), dim3(kBlock), 0, s, S, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_shared_slot(const SDev<T> &S, hipStream_t s)
{
    hipLaunchKernelGGL(sk_dual<T>, dim3(S.grid_m), dim3(kBlock), 0, s, S);
    hipLaunchKernelGGL(sk_step_decide<T>, dim3(S.Bp), dim3(kBlock), 0, s, S);
    hipLaunchKernelGGL(sk_update<T>, dim3(S.grid), dim3(kBlock), 0, s, S);
    return launch_shared_check<T>(S, 1, s);
}

template <typename T>
hipError_t launch_shared_product(const SDev<T> &S, int which, const T *in, T *out, hipStream_t s)
{
    const int64_t total = (int64_t)(which ? S.n : S.m) << S.lgB;
    if (total <= 0) return hipSuccess;
    const dim3 g((unsigned)std::min<int64_t>((total + kBlock - 1) / kBlock, 8192));
    if (which == 0) hipLaunchKernelGGL((sk_product<T, 0>), g, dim3(kBlock), 0, s, S, in, out);
    else hipLaunchKernelGGL((sk_product<T, 1>), g, dim3(kBlock), 0, s, S, in, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_shared_extract(const T *src, int lgB, int b, double *dst, int rows, hipStream_t s)
{
    if (rows > 0) hipLaunchKernelGGL(sk_extract<T>, nblocks(rows), dim3(kBlock), 0, s, src, lgB, b, dst, rows);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_shared_insert(const double *src, int lgB, int b, T *dst, int rows, hipStream_t s)
{
    if (rows > 0) hipLaunchKernelGGL(sk_insert<T>, nblocks(rows), dim3(kBlock), 0, s, src, lgB, b, dst, rows);
    return hipGetLastError();
}

hipError_t launch_shared_set_final(Ctl *ctl, int Bp, int status, hipStream_t s)
{
    hipLaunchKernelGGL(sk_set_final, nblocks(Bp), dim3(kBlock), 0, s, ctl, Bp, status);
    return hipGetLastError();
}

#define PDLP_SHARED_INSTANTIATE(T)                                                                                 \
    template hipError_t launch_shared_slot<T>(const SDev<T> &, hipStream_t);                                       \
    template hipError_t launch_shared_check<T>(const SDev<T> &, int, hipStream_t);                                 \
    template hipError_t launch_shared_apply<T>(const SDev<T> &, hipStream_t);                                      \
    template hipError_t launch_shared_product<T>(const SDev<T> &, int, const T *, T *, hipStream_t);               \
    template hipError_t launch_shared_extract<T>(const T *, int, int, double *, int, hipStream_t);                 \
    template hipError_t launch_shared_insert<T>(const double *, int, int, T *, int, hipStream_t);

PDLP_SHARED_INSTANTIATE(double)
PDLP_SHARED_INSTANTIATE(float)

}  // namespace pdlp
