// Batched restarted PDHG: many independent LPs advanced together by one set
// of kernels per attempt slot (the same slot structure as the single-LP
// solver, replayed as one captured hipGraph window).  Each LP keeps its own
// controller block, so step acceptance, restarts, primal weight and
// termination are per instance; a finished instance drops out of every
// kernel.  The block-diagonal products need no column slicing: every row
// block belongs to one instance and instances are dealt to XCDs, so an
// instance's gathered vector is fetched into a single L2.
#include "device.h"

namespace pdlp {

// row block blk of a batch product (end row complemented for long rows)
template <bool SPLIT, typename T>
__device__ __forceinline__ void batch_block(const int *rp, const int *ci, const T *v, const T *x, const BlockList &L,
                                            int blk, T *out, T *prod, double *red, SplitLds<T> *sl)
{
    const int r0 = L.r0[blk], r1e = L.r1[blk];
    const bool wave = r1e < 0;
    const int r1 = wave ? ~r1e : r1e;
    stream_block<SPLIT>(RowsPlain{rp}, ci, v, x, r0, r1, wave, rp[r0], rp[r1], out, prod, red, sl);
}

// SPLIT (here and below): short-row blocks summed split by entries (BlockList::split)
template <typename T, int WHICH, bool SPLIT>
__global__ __launch_bounds__(kBlock) void bk_product(BDev<T> b)
{
    __shared__ T prod[kStreamNB];
    __shared__ double red[kBlock / 64];
    SplitLds<T> *sl = nullptr;
    if constexpr (SPLIT) {
        __shared__ SplitLds<T> split_lds;
        sl = &split_lds;
    }
    const BlockList &L = WHICH ? b.LT : b.LK;
    const int xcd = (int)blockIdx.x % kXcds;
    const int per = (int)gridDim.x / kXcds;
    for (int k = L.xoff[xcd] + (int)blockIdx.x / kXcds; k < L.xoff[xcd + 1]; k += per) {
        const int blk = L.order[k];
        const Ctl *c = b.ctl + L.inst[blk];
        if (c->done || (WHICH == 1 && !c->accepted)) continue;
        if (WHICH == 0)
            batch_block<SPLIT>(b.krp, b.kci, b.kv, (const T *)pick(b.d.xb, c->cur ^ 1), L, blk, b.prodK, prod, red,
                               sl);
        else
            batch_block<SPLIT>(b.trp, b.tci, b.tv, (const T *)pick(b.d.yb, c->cur), L, blk, b.prodKT, prod, red, sl);
    }
}

template <typename T, int WHICH, bool SPLIT>
__global__ __launch_bounds__(kBlock) void bk_product_plain(BDev<T> b, const T *__restrict__ in, T *__restrict__ out)
{
    __shared__ T prod[kStreamNB];
    __shared__ double red[kBlock / 64];
    SplitLds<T> *sl = nullptr;
    if constexpr (SPLIT) {
        __shared__ SplitLds<T> split_lds;
        sl = &split_lds;
    }
    const BlockList &L = WHICH ? b.LT : b.LK;
    const int xcd = (int)blockIdx.x % kXcds;
    const int per = (int)gridDim.x / kXcds;
    for (int k = L.xoff[xcd] + (int)blockIdx.x / kXcds; k < L.xoff[xcd + 1]; k += per) {
        const int blk = L.order[k];
        if (WHICH == 0) batch_block<SPLIT>(b.krp, b.kci, b.kv, in, L, blk, out, prod, red, sl);
        else batch_block<SPLIT>(b.trp, b.tci, b.tv, in, L, blk, out, prod, red, sl);
    }
}

// one workgroup per m-chunk; workgroup 0 also lowers the check gate, which
// the step decisions of this slot raise again if an instance checks
template <typename T>
__global__ __launch_bounds__(kBlock) void bk_dual(BDev<T> b)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *b.gate = 0;
    if ((int)blockIdx.x >= b.acm) return;
    const int chunk = b.act_cm ? b.act_cm[blockIdx.x] : (int)blockIdx.x;
    const int inst = b.cinst_m[chunk];
    const Ctl *ctl = b.ctl + inst;
    if (ctl->done) return;
    const Dev<T> &d = b.d;
    const int c = ctl->cur;
    DualEpi<T> epi{pick(d.yb, c), pick(d.Kxb, c), d.qs, pick(d.yb, c ^ 1), pick(d.Kxb, c ^ 1), b.m1g[inst],
                   (T)(ctl->eta * ctl->omega), 0.0, 0.0};
    const int i = chunk * kBlock + (int)threadIdx.x;
    epi(i, b.prodK[i]);
    double v[2] = {epi.dy2, epi.inter};
    block_store_partials<2>(v, d.part_dual, chunk);
}

// one workgroup per instance
template <typename T>
__global__ __launch_bounds__(kBlock) void bk_step_decide(BDev<T> b)
{
    if ((int)blockIdx.x >= b.aci) return;
    const int inst = b.act_i ? b.act_i[blockIdx.x] : (int)blockIdx.x;
    Ctl *ctl = b.ctl + inst;
    if (ctl->done) {
        if (threadIdx.x == 0) ctl->mode = MODE_NONE;
        return;
    }
    double a[1], c2[2];
    block_sum_partials<1>(b.d.part_primal + b.nc0[inst], b.ncc[inst], a);
    block_sum_partials<2>(b.d.part_dual + 2 * (size_t)b.mc0[inst], b.mcc[inst], c2);
    if (threadIdx.x == 0) {
        step_decision(ctl, a[0], c2[0], c2[1]);
        if (ctl->mode != MODE_NONE) atomicExch(b.gate, 1);
    }
}

// one workgroup per n-chunk, then one per m-chunk
template <typename T>
__global__ __launch_bounds__(kBlock) void bk_update(BDev<T> b)
{
    const bool nside = (int)blockIdx.x < b.acn;
    const int at = nside ? (int)blockIdx.x : (int)blockIdx.x - b.acn;
    const int chunk = nside ? (b.act_cn ? b.act_cn[at] : at) : (b.act_cm ? b.act_cm[at] : at);
    const int inst = nside ? b.cinst_n[chunk] : b.cinst_m[chunk];
    const Ctl *ctl = b.ctl + inst;
    if (ctl->done) return;
    const Dev<T> &d = b.d;
    const int c = ctl->cur;
    const T tau = (T)(ctl->eta / ctl->omega);
    const int e = chunk * kBlock + (int)threadIdx.x;
    double dx2 = 0.0;
    if (!ctl->accepted) {
        if (nside) primal_elem(d, c, tau, e, dx2);
    } else if (nside) {
        UpdateEpi<T> epi{pick(d.xb, c), d.cs, d.ls, d.us, pick(d.KTyb, c), d.xa, d.KTya, pick(d.xb, c ^ 1),
                         (T)ctl->avg_w, tau, ctl->mode == MODE_NONE, 0.0};
        epi(e, b.prodKT[e]);
        dx2 = epi.dx2;
    } else {
        average_row(d, e, c, (T)ctl->avg_w);
    }
    if (nside) {
        double v[1] = {dx2};
        block_store_partials<1>(v, d.part_primal, chunk);
    }
}

// The check kernels walk 256-element chunks (each inside one instance) with
// a grid stride, each chunk's partial in its own slot.  Inside the solve
// loop (gated) they return at once unless this slot's step decisions put
// some instance into a check; the host-driven start, resume and final checks
// run ungated.
template <typename T>
__global__ __launch_bounds__(kBlock) void bk_check_reduce(BDev<T> b, int gated)
{
    if (gated && *b.gate == 0) return;
    for (int t = blockIdx.x; t < b.acn + b.acm; t += gridDim.x) {
        const bool nside = t < b.acn;
        const int at = nside ? t : t - b.acn;
        const int chunk = nside ? (b.act_cn ? b.act_cn[at] : at) : (b.act_cm ? b.act_cm[at] : at);
        const int ch = nside ? chunk : b.ncn + chunk;   // the chunk's partial slot
        const int inst = nside ? b.cinst_n[chunk] : b.cinst_m[chunk];
        const Ctl *ctl = b.ctl + inst;
        if (ctl->mode == MODE_NONE || ctl->done) continue;
        const Dev<T> &d = b.d;
        const int c = ctl->cur;
        const int e = chunk * kBlock + (int)threadIdx.x;
        double s[kCheckSums];
#pragma unroll
        for (int i = 0; i < kCheckSums; ++i) s[i] = 0.0;
        if (nside) {
            col_sums(d, e, (const T *)pick(d.xb, c), (const T *)pick(d.KTyb, c), s);
            col_sums(d, e, (const T *)d.xa, (const T *)d.KTya, s + 9);
        } else {
            row_sums(d, e, b.m1g[inst], (const T *)pick(d.yb, c), (const T *)pick(d.Kxb, c), s);
            row_sums(d, e, b.m1g[inst], (const T *)d.ya, (const T *)d.Kxa, s + 9);
        }
        block_store_partials<kCheckSums>(s, d.part_check, ch);
        double r[kRaySums] = {0.0, 0.0, 0.0, 0.0};
        if (nside) ray_col_sums(d, e, (const T *)pick(d.xb, c), (const T *)pick(d.KTyb, c), r);
        else ray_row_sums(d, e, b.m1g[inst], (const T *)pick(d.yb, c), (const T *)pick(d.Kxb, c), r);
        block_store_partials<kRaySums>(r, d.part_ray, ch);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bk_check_decide(BDev<T> b, int gated)
{
    if (gated && *b.gate == 0) return;
    if ((int)blockIdx.x >= b.aci) return;
    const int inst = b.act_i ? b.act_i[blockIdx.x] : (int)blockIdx.x;
    Ctl *ctl = b.ctl + inst;
    if (ctl->mode == MODE_NONE || ctl->done) return;
    double Sn[kCheckSums], Sm[kCheckSums], Rn[kRaySums], Rm[kRaySums];
    block_sum_partials<kCheckSums>(b.d.part_check + (size_t)kCheckSums * b.nc0[inst], b.ncc[inst], Sn);
    block_sum_partials<kCheckSums>(b.d.part_check + (size_t)kCheckSums * (b.ncn + b.mc0[inst]), b.mcc[inst], Sm);
    block_sum_partials<kRaySums>(b.d.part_ray + (size_t)kRaySums * b.nc0[inst], b.ncc[inst], Rn);
    block_sum_partials<kRaySums>(b.d.part_ray + (size_t)kRaySums * (b.ncn + b.mc0[inst]), b.mcc[inst], Rm);
    if (threadIdx.x != 0) return;
    double S[kCheckSums], R[kRaySums];
    for (int i = 0; i < kCheckSums; ++i) S[i] = Sn[i] + Sm[i];
    for (int i = 0; i < kRaySums; ++i) R[i] = Rn[i] + Rm[i];
    check_decision(ctl, S, R, b.Nq[inst], b.Nc[inst]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void bk_check_apply(BDev<T> b, int gated)
{
    if (gated && *b.gate == 0) return;
    for (int t = blockIdx.x; t < b.acn + b.acm; t += gridDim.x) {
        const bool nside = t < b.acn;
        const int at = nside ? t : t - b.acn;
        const int chunk = nside ? (b.act_cn ? b.act_cn[at] : at) : (b.act_cm ? b.act_cm[at] : at);
        const int inst = nside ? b.cinst_n[chunk] : b.cinst_m[chunk];
        const Ctl *ctl = b.ctl + inst;
        if (ctl->mode == MODE_NONE) continue;
        const Dev<T> &d = b.d;
        const int c = ctl->cur, rt = ctl->restart_to, co = ctl->copy_out, sel = ctl->out_sel;
        const int np = ctl->need_primal;
        const int e = chunk * kBlock + (int)threadIdx.x;
        double dx2 = 0.0;
        if (nside) {
            apply_col(d, e, c, rt, co, sel, np, (T)(ctl->eta / ctl->omega), dx2);
            double v[1] = {dx2};
            block_store_partials<1>(v, d.part_primal, chunk);
        } else {
            apply_row(d, e, c, rt, co, sel);
        }
    }
}

// cold start of every instance: x = proj_X(0), y = 0 (buffer 0)
template <typename T>
__global__ void bk_start(BDev<T> b)
{
    const int e = blockIdx.x * kBlock + (int)threadIdx.x;
    const Dev<T> &d = b.d;
    if (e < d.n) d.xb[0][e] = clampv(T(0), d.ls[e], d.us[e]);
    if (e < d.m) d.yb[0][e] = T(0);
}

__global__ void bk_set_final(Ctl *ctl, int B, int status)
{
    const int i = blockIdx.x * kBlock + (int)threadIdx.x;
    if (i < B && !ctl[i].done) {
        ctl[i].mode = MODE_FINAL;
        ctl[i].final_status = status;
    }
}

// per-segment sum of squares / max |.|: one workgroup per segment [off[i], off[i+1])
__global__ void k_seg_sumsq(const double *a, const int64_t *off, double *out)
{
    double s[1] = {0.0};
    for (int64_t i = off[blockIdx.x] + threadIdx.x; i < off[blockIdx.x + 1]; i += kBlock) s[0] += a[i] * a[i];
    double t[1];
    __shared__ double tmp[kBlock];
    tmp[threadIdx.x] = s[0];
    __syncthreads();
    block_sum_partials<1>(tmp, kBlock, t);
    if (threadIdx.x == 0) out[blockIdx.x] = t[0];
}

__global__ void k_seg_absmax(const double *a, const int64_t *off, double *out)
{
    __shared__ double sh[kBlock / 64];
    double s = 0.0;
    for (int64_t i = off[blockIdx.x] + threadIdx.x; i < off[blockIdx.x + 1]; i += kBlock) s = fmax(s, fabs(a[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// ----------------------------------------------------------------------------

// workgroups of a chunk-striding batch kernel: every chunk, at most 4096
inline int chunk_grid(int chunks) { return chunks < 1 ? 1 : (chunks < 4096 ? chunks : 4096); }

template <typename T>
hipError_t launch_batch_product(const BDev<T> &b, int which, hipStream_t s)
{
    const BlockList &L = which ? b.LT : b.LK;
    const dim3 g(L.grid), t(kBlock);
    if (which == 0) {
        if (L.split) hipLaunchKernelGGL((bk_product<T, 0, true>), g, t, 0, s, b);
        else hipLaunchKernelGGL((bk_product<T, 0, false>), g, t, 0, s, b);
    } else {
        if (L.split) hipLaunchKernelGGL((bk_product<T, 1, true>), g, t, 0, s, b);
        else hipLaunchKernelGGL((bk_product<T, 1, false>), g, t, 0, s, b);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_product_plain(const BDev<T> &b, int which, const T *in, T *out, hipStream_t s)
{
    const BlockList &L = which ? b.LT : b.LK;
    const dim3 g(L.grid), t(kBlock);
    if (which == 0) {
        if (L.split) hipLaunchKernelGGL((bk_product_plain<T, 0, true>), g, t, 0, s, b, in, out);
        else hipLaunchKernelGGL((bk_product_plain<T, 0, false>), g, t, 0, s, b, in, out);
    } else {
        if (L.split) hipLaunchKernelGGL((bk_product_plain<T, 1, true>), g, t, 0, s, b, in, out);
        else hipLaunchKernelGGL((bk_product_plain<T, 1, false>), g, t, 0, s, b, in, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_dual(const BDev<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL(bk_dual<T>, dim3(b.acm > 0 ? b.acm : 1), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_step_decide(const BDev<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL(bk_step_decide<T>, dim3(b.aci > 0 ? b.aci : 1), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_update(const BDev<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL(bk_update<T>, dim3(b.acn + b.acm > 0 ? b.acn + b.acm : 1), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_check(const BDev<T> &b, int gated, hipStream_t s)
{
    hipLaunchKernelGGL(bk_check_reduce<T>, dim3(chunk_grid(b.acn + b.acm)), dim3(kBlock), 0, s, b, gated);
    hipLaunchKernelGGL(bk_check_decide<T>, dim3(b.aci > 0 ? b.aci : 1), dim3(kBlock), 0, s, b, gated);
    hipLaunchKernelGGL(bk_check_apply<T>, dim3(chunk_grid(b.acn + b.acm)), dim3(kBlock), 0, s, b, gated);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_apply(const BDev<T> &b, hipStream_t s)
{
    hipLaunchKernelGGL(bk_check_apply<T>, dim3(chunk_grid(b.ncn + b.ncm)), dim3(kBlock), 0, s, b, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_start(const BDev<T> &b, hipStream_t s)
{
    const int nb = (b.d.n > b.d.m ? b.d.n : b.d.m) / kBlock;
    if (nb > 0) hipLaunchKernelGGL(bk_start<T>, dim3(nb), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_set_final(Ctl *ctl, int B, int status, hipStream_t s)
{
    hipLaunchKernelGGL(bk_set_final, dim3((B + kBlock - 1) / kBlock), dim3(kBlock), 0, s, ctl, B, status);
    return hipGetLastError();
}

hipError_t launch_seg_sumsq(const double *a, const int64_t *off, int B, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_seg_sumsq, dim3(B), dim3(kBlock), 0, s, a, off, out);
    return hipGetLastError();
}

hipError_t launch_seg_absmax(const double *a, const int64_t *off, int B, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_seg_absmax, dim3(B), dim3(kBlock), 0, s, a, off, out);
    return hipGetLastError();
}

#define PDLP_BATCH_INSTANTIATE(T)                                                                                  \
    template hipError_t launch_batch_product<T>(const BDev<T> &, int, hipStream_t);                                \
    template hipError_t launch_batch_product_plain<T>(const BDev<T> &, int, const T *, T *, hipStream_t);          \
    template hipError_t launch_batch_dual<T>(const BDev<T> &, hipStream_t);                                        \
    template hipError_t launch_batch_step_decide<T>(const BDev<T> &, hipStream_t);                                 \
    template hipError_t launch_batch_update<T>(const BDev<T> &, hipStream_t);                                      \
    template hipError_t launch_batch_check<T>(const BDev<T> &, int, hipStream_t);                                  \
    template hipError_t launch_batch_apply<T>(const BDev<T> &, hipStream_t);                                       \
    template hipError_t launch_batch_start<T>(const BDev<T> &, hipStream_t);

PDLP_BATCH_INSTANTIATE(double)
PDLP_BATCH_INSTANTIATE(float)

}  // namespace pdlp
