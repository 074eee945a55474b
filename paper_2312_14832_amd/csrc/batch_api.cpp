// Host side of the batched solver (lp_batch_* in include/lp.h).
//
// lp_batch_load concatenates the instances block-diagonally (each one's
// vectors padded to whole 256-element chunks), scales the whole
// block-diagonal matrix at once (row and column scaling never mixes blocks,
// so every instance gets exactly its own scaling), cuts the rows of K and K'
// into CSR-Stream row blocks that never straddle instances, and deals the
// instances to the 8 XCDs by a longest-processing-time rule on their
// nonzeros.  lp_batch_solve replays a captured window of attempt slots until
// every instance is done.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "host_util.h"
#include "internal.h"

using namespace pdlp;

namespace {
constexpr int kNScalars = 16;

int64_t pad256(int64_t v) { return (v + kBlock - 1) / kBlock * kBlock; }
}  // namespace

struct lp_batch {
    int B = 0;
    lp_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool mixed = false;
    std::vector<int64_t> n, m, m1, noff, moff;
    int64_t Ntot = 0, Mtot = 0;
    std::vector<double> Nq, Nc, omega0, eta0;
    Arena arena;
    BDev<double> b64{};
    BDev<float> b32{};
    Ctl *hctl = nullptr;   // pinned mirror, B entries
    double *stage_n0 = nullptr, *stage_n1 = nullptr, *stage_m = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_window = 0;
    bool has_result = false;
    std::vector<char> state_set;
    std::vector<double> finish_s;   // per instance: seconds into the last solve when it finished
    // Narrowed launches once most instances have finished (see compact_active):
    // the owners of every chunk, host copies of the full block lists, and
    // device room for the narrowed chunk and block lists
    std::vector<int> cin, cim;
    std::vector<int> lorder[2], linst[2];
    BlockList full[2]{};
    int *act_cn = nullptr, *act_cm = nullptr, *act_i = nullptr, *act_order[2] = {nullptr, nullptr};
    int active = -1;   // unfinished instances the lists were narrowed to (-1: full lists)
    // The one-workgroup loop per instance (set up at load when every instance
    // fits its register form): per-instance views (Dev<T>, device array), the
    // instances' norms, the form (1 or 2 columns and rows per thread, 0: not
    // set up), the largest LDS stage and the slots per launch
    // Mixed precision's FP64 re-check of a passed termination test (as
    // lp_solve's): the FP64 scaled matrices and vectors kept from the load,
    // the batch's CSR pair, and scratch for one instance at a time
    const double *kv64 = nullptr, *tv64 = nullptr, *cs64 = nullptr, *ls64 = nullptr, *us64 = nullptr,
                 *qs64 = nullptr;
    const int *g_rp = nullptr, *g_ci = nullptr, *g_tp = nullptr, *g_ti = nullptr;
    double *ckx[2] = {nullptr, nullptr}, *ckty[2] = {nullptr, nullptr}, *cpart = nullptr;
    void *small_devs = nullptr;
    double *small_nq = nullptr, *small_nc = nullptr;
    int small_R = 0, small_slots = 0;
    size_t small_stage = 0;
    int shape[2][2] = {{kStreamNB, kStreamRB}, {kStreamNB, kStreamRB}};   // K, K': most nonzeros, rows per block
    double seconds = 0;
    std::string err;

    template <typename T> BDev<T> &dev();
    ~lp_batch()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (hctl) (void)hipHostFree(hctl);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

template <> BDev<double> &lp_batch::dev<double>() { return b64; }
template <> BDev<float> &lp_batch::dev<float>() { return b32; }

namespace {

void bsync(lp_batch *P) { HIPT(hipStreamSynchronize(P->stream)); }

void release_blocks(lp_batch *P, const BlockList &L)
{
    for (const void *p : {(const void *)L.r0, (const void *)L.r1, (const void *)L.inst, (const void *)L.order})
        P->arena.release(const_cast<void *>(p));
}

int fail(lp_batch *P, const HipError &h)
{
    char buf[512];
    snprintf(buf, sizeof(buf), "%s failed: %s", h.what, hipGetErrorString(h.e));
    if (P) P->err = buf;
    return h.e == hipErrorOutOfMemory ? LP_ERR_NOMEM : LP_ERR_HIP;
}

// Instance i's view of the batch's vectors and controller (its own indices
// 0 .. n_i, 0 .. m_i); the products are left unset.
template <typename T>
Dev<T> view_of(lp_batch *P, int i)
{
    const BDev<T> &b = P->dev<T>();
    const Dev<T> &d = b.d;
    const int64_t mo = P->moff[i], no = P->noff[i];
    Dev<T> v{};
    v.m = (int)P->m[i];
    v.n = (int)P->n[i];
    v.m1 = (int)P->m1[i];
    v.cs = d.cs + no; v.ls = d.ls + no; v.us = d.us + no; v.qs = d.qs + mo;
    v.Dr = d.Dr + mo; v.Dc = d.Dc + no;
    for (int k = 0; k < 2; ++k) {
        v.xb[k] = d.xb[k] + no; v.yb[k] = d.yb[k] + mo; v.Kxb[k] = d.Kxb[k] + mo; v.KTyb[k] = d.KTyb[k] + no;
    }
    v.xa = d.xa + no; v.ya = d.ya + mo; v.Kxa = d.Kxa + mo; v.KTya = d.KTya + no;
    v.x0 = d.x0 + no; v.y0 = d.y0 + mo; v.Kx0 = d.Kx0 + mo; v.KTy0 = d.KTy0 + no;
    v.xo = d.xo + no; v.yo = d.yo + mo; v.KTyo = d.KTyo + no;
    v.ctl = b.ctl + i;
    return v;
}

// The one-workgroup loop for a batch of small LPs: when every instance has
// rows and columns for the register form (at most 2 kSmallReg each, at least
// one) and its stage fits the LDS, each gets a view of the batch (its
// vectors, its controller, and a plain CSR of its own K and K' with row
// pointers from 0 and indices inside the instance, sharing the batch's
// scaled values), and the solve runs one workgroup per instance.
template <typename T>
void setup_small(lp_batch *P, const std::vector<int> &rp, const std::vector<int> &ci, const std::vector<int> &tp,
                 const std::vector<int> &ti)
{
    const int B = P->B;
    BDev<T> &b = P->dev<T>();
    size_t stage = 0;
    int R = 1;
    for (int i = 0; i < B; ++i) {
        const int64_t m = P->m[i], n = P->n[i];
        if (m < 1 || n < 1 || m > 2 * kSmallReg || n > 2 * kSmallReg) return;
        if (m > kSmallReg || n > kSmallReg) R = 2;
        const int64_t nk = rp[P->moff[i] + m] - rp[P->moff[i]], nt = tp[P->noff[i] + n] - tp[P->noff[i]];
        stage = std::max(stage, small_stage_bytes<T>((int)m, (int)n, (int)nk, (int)nt));
    }
    const size_t lds = (stage + 7) / 8 * 8;
    if (B < 1 || lds + 16 * 64 > kSmallRegLds) return;
    std::vector<int> lrp, ltp, lci(ci.size()), lti(ti.size());
    std::vector<int64_t> krow(B), trow(B);
    for (int i = 0; i < B; ++i) {
        const int64_t mo = P->moff[i], no = P->noff[i], m = P->m[i], n = P->n[i];
        const int e0 = rp[mo], t0 = tp[no];
        krow[i] = (int64_t)lrp.size();
        for (int64_t r = 0; r <= m; ++r) lrp.push_back(rp[mo + r] - e0);
        for (int p = e0; p < rp[mo + m]; ++p) lci[p] = ci[p] - (int)no;
        trow[i] = (int64_t)ltp.size();
        for (int64_t r = 0; r <= n; ++r) ltp.push_back(tp[no + r] - t0);
        for (int p = t0; p < tp[no + n]; ++p) lti[p] = ti[p] - (int)mo;
    }
    Arena &A = P->arena;
    hipStream_t st = P->stream;
    int *d_lrp = A.make<int>((int64_t)lrp.size()), *d_ltp = A.make<int>((int64_t)ltp.size());
    int *d_lci = A.make<int>((int64_t)lci.size()), *d_lti = A.make<int>((int64_t)lti.size());
    h2d(st, d_lrp, lrp.data(), (int64_t)lrp.size());
    h2d(st, d_ltp, ltp.data(), (int64_t)ltp.size());
    h2d(st, d_lci, lci.data(), (int64_t)lci.size());
    h2d(st, d_lti, lti.data(), (int64_t)lti.size());
    std::vector<Dev<T>> views((size_t)B);
    for (int i = 0; i < B; ++i) {
        const int64_t mo = P->moff[i], no = P->noff[i];
        Dev<T> v = view_of<T>(P, i);
        v.K.S = 1;
        v.K.rows = v.m;
        v.K.rp = d_lrp + krow[i];
        v.K.ci = d_lci + rp[mo];
        v.K.v = b.kv + rp[mo];
        v.KT.S = 1;
        v.KT.rows = v.n;
        v.KT.rp = d_ltp + trow[i];
        v.KT.ci = d_lti + tp[no];
        v.KT.v = b.tv + tp[no];
        views[(size_t)i] = v;
    }
    Dev<T> *d_views = (Dev<T> *)A.alloc(sizeof(Dev<T>) * (size_t)B);
    h2d(st, d_views, views.data(), B);
    P->small_nq = A.make<double>(B);
    P->small_nc = A.make<double>(B);
    h2d(st, P->small_nq, P->Nq.data(), B);
    h2d(st, P->small_nc, P->Nc.data(), B);
    bsync(P);
    P->small_devs = d_views;
    P->small_R = R;
    P->small_stage = stage;
    P->small_slots = (int)std::min<size_t>((kSmallRegLds - lds) / 16, (size_t)64 * std::max(1, P->opt.window));
}

// row blocks (at most nb nonzeros and rb rows) of every instance's padded
// row range, dealt to XCDs
BlockList make_blocks(lp_batch *P, const std::vector<int> &rp, const std::vector<int64_t> &off,
                      const std::vector<int64_t> &len_pad, const std::vector<int> &xcd_of, int nb = kStreamNB,
                      int rb = kStreamRB)
{
    const int B = P->B;
    std::vector<int> r0, r1, inst;
    for (int i = 0; i < B; ++i) {
        std::vector<int> ends;
        std::vector<char> wave;
        row_blocks(rp.data(), (int)off[i], (int)(off[i] + len_pad[i]), ends, wave, nb, rb);
        int start = (int)off[i];
        for (size_t k = 0; k < ends.size(); ++k) {
            r0.push_back(start);
            r1.push_back(wave[k] ? ~ends[k] : ends[k]);
            inst.push_back(i);
            start = ends[k];
        }
    }
    BlockList L{};
    L.nblk = (int)r0.size();
    std::vector<int> order;
    int maxper = 1;
    for (int x = 0; x < kXcds; ++x) {
        L.xoff[x] = (int)order.size();
        for (int k = 0; k < L.nblk; ++k)
            if (xcd_of[inst[k]] == x) order.push_back(k);
        maxper = std::max(maxper, (int)order.size() - L.xoff[x]);
    }
    L.xoff[kXcds] = (int)order.size();
    L.grid = kXcds * std::min(maxper, 512);
    L.split = P->opt.split_sums == 1;   // by rows unless asked: no faster on the batched workloads
    int *d_r0 = P->arena.make<int>(L.nblk), *d_r1 = P->arena.make<int>(L.nblk);
    int *d_inst = P->arena.make<int>(L.nblk), *d_order = P->arena.make<int>(L.nblk);
    h2d(P->stream, d_r0, r0.data(), L.nblk);
    h2d(P->stream, d_r1, r1.data(), L.nblk);
    h2d(P->stream, d_inst, inst.data(), L.nblk);
    h2d(P->stream, d_order, order.data(), L.nblk);
    bsync(P);
    L.r0 = d_r0; L.r1 = d_r1; L.inst = d_inst; L.order = d_order;
    return L;
}

int do_batch_load(lp_batch *P, const lp_csr *K, const double *const *c, const double *const *q,
                  const double *const *l, const double *const *u)
{
    const int B = P->B;
    hipStream_t st = P->stream;
    // offsets of the padded concatenation
    P->noff.assign(B + 1, 0);
    P->moff.assign(B + 1, 0);
    std::vector<int64_t> npad(B), mpad(B);
    for (int i = 0; i < B; ++i) {
        npad[i] = pad256(P->n[i]);
        mpad[i] = pad256(P->m[i]);
        P->noff[i + 1] = P->noff[i] + npad[i];
        P->moff[i + 1] = P->moff[i] + mpad[i];
    }
    P->Ntot = P->noff[B];
    P->Mtot = P->moff[B];
    if (P->Ntot >= (int64_t(1) << 31) || P->Mtot >= (int64_t(1) << 31)) return LP_ERR_TOO_LARGE;
    // block-diagonal K (padding rows empty) and its transpose
    std::vector<int> rp, ci, tp, ti;
    std::vector<double> kv, tv;
    rp.push_back(0);
    for (int i = 0; i < B; ++i) {
        append_sorted_rows(&K[i], (int)P->noff[i], rp, ci, kv);
        for (int64_t r = P->m[i]; r < mpad[i]; ++r) rp.push_back((int)ci.size());
    }
    if ((int64_t)ci.size() >= (int64_t(1) << 31)) return LP_ERR_TOO_LARGE;
    const int64_t nnz = (int64_t)ci.size();
    transpose_csr((int)P->Mtot, (int)P->Ntot, rp, ci, kv, tp, ti, tv);
    // vectors; padding entries: zero data, bounds [0,0]
    std::vector<double> hc(P->Ntot, 0.0), hl(P->Ntot, 0.0), hu(P->Ntot, 0.0), hq(P->Mtot, 0.0);
    std::vector<int> m1g(B);
    for (int i = 0; i < B; ++i) {
        std::copy(c[i], c[i] + P->n[i], hc.begin() + P->noff[i]);
        std::copy(l[i], l[i] + P->n[i], hl.begin() + P->noff[i]);
        std::copy(u[i], u[i] + P->n[i], hu.begin() + P->noff[i]);
        std::copy(q[i], q[i] + P->m[i], hq.begin() + P->moff[i]);
        m1g[i] = (int)(P->moff[i] + P->m1[i]);
    }
    const int N = (int)P->Ntot, M = (int)P->Mtot;
    Arena &A = P->arena;
    // test hook: PDLP_DEBUG_FILL_BYTE=<0..255> fills every device allocation of
    // the batch with that byte, so a read of memory the load never sets shows
    if (const char *fb = std::getenv("PDLP_DEBUG_FILL_BYTE")) A.fill = std::atoi(fb) & 255;
    int *d_rp = A.make<int>(M + 1), *d_ci = A.make<int>(nnz), *d_tp = A.make<int>(N + 1), *d_ti = A.make<int>(nnz);
    double *d_kv = A.make<double>(nnz), *d_tv = A.make<double>(nnz);
    double *d_c = A.make<double>(N), *d_l = A.make<double>(N), *d_u = A.make<double>(N), *d_q = A.make<double>(M);
    double *Dr = A.make<double>(M), *Dc = A.make<double>(N), *r = A.make<double>(M), *s = A.make<double>(N);
    double *cs = A.make<double>(N), *ls = A.make<double>(N), *us = A.make<double>(N), *qs = A.make<double>(M);
    P->stage_n0 = A.make<double>(N);
    P->stage_n1 = A.make<double>(N);
    P->stage_m = A.make<double>(M);
    h2d(st, d_rp, rp.data(), M + 1);
    h2d(st, d_ci, ci.data(), nnz);
    h2d(st, d_kv, kv.data(), nnz);
    h2d(st, d_tp, tp.data(), N + 1);
    h2d(st, d_ti, ti.data(), nnz);
    h2d(st, d_tv, tv.data(), nnz);
    h2d(st, d_c, hc.data(), N);
    h2d(st, d_l, hl.data(), N);
    h2d(st, d_u, hu.data(), N);
    h2d(st, d_q, hq.data(), M);
    HIPT(scale_csr_pair(d_rp, d_ci, d_kv, M, d_tp, d_ti, d_tv, N, Dr, Dc, r, s, P->opt.ruiz_iters, P->opt.pc_alpha, st));
    HIPT(launch_scale_vectors(d_c, d_l, d_u, d_q, Dc, Dr, cs, ls, us, qs, N, M, st));
    // per-instance norms: |q|, |c| (unscaled), |q~|, |c~|, max |K~|
    std::vector<int64_t> on(B + 1), om(B + 1), oz(B + 1);
    for (int i = 0; i <= B; ++i) {
        on[i] = P->noff[i];
        om[i] = P->moff[i];
        oz[i] = rp[P->moff[i]];
    }
    int64_t *d_on = A.make<int64_t>(B + 1), *d_om = A.make<int64_t>(B + 1), *d_oz = A.make<int64_t>(B + 1);
    double *d_norms = A.make<double>(5 * (int64_t)B);
    h2d(st, d_on, on.data(), B + 1);
    h2d(st, d_om, om.data(), B + 1);
    h2d(st, d_oz, oz.data(), B + 1);
    HIPT(launch_seg_sumsq(d_q, d_om, B, d_norms + 0 * B, st));
    HIPT(launch_seg_sumsq(d_c, d_on, B, d_norms + 1 * B, st));
    HIPT(launch_seg_sumsq(qs, d_om, B, d_norms + 2 * B, st));
    HIPT(launch_seg_sumsq(cs, d_on, B, d_norms + 3 * B, st));
    HIPT(launch_seg_absmax(d_kv, d_oz, B, d_norms + 4 * B, st));
    std::vector<double> h(5 * (size_t)B);
    d2h(st, h.data(), d_norms, 5 * (int64_t)B);
    bsync(P);
    P->Nq.resize(B); P->Nc.resize(B); P->omega0.resize(B); P->eta0.resize(B);
    for (int i = 0; i < B; ++i) {
        P->Nq[i] = std::sqrt(h[i]);
        P->Nc[i] = std::sqrt(h[B + i]);
        const double nq = std::sqrt(h[2 * B + i]), nc = std::sqrt(h[3 * B + i]);
        P->omega0[i] = (nc > 1e-10 && nq > 1e-10) ? nc / nq : 1.0;
        P->eta0[i] = h[4 * B + i] > 0.0 ? 1.0 / h[4 * B + i] : 1.0;
        if (P->opt.fixed_step) P->eta0[i] = P->opt.fixed_eta;
    }
    // instances to XCDs: longest processing time first on nonzeros
    std::vector<int> idx(B), xcd_of(B, 0);
    std::iota(idx.begin(), idx.end(), 0);
    std::vector<int64_t> work(B);
    for (int i = 0; i < B; ++i) work[i] = rp[P->moff[i + 1]] - rp[P->moff[i]] + npad[i] + mpad[i];
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work[a] > work[b]; });
    int64_t load[kXcds] = {0};
    for (int i : idx) {
        int best = 0;
        for (int x = 1; x < kXcds; ++x)
            if (load[x] < load[best]) best = x;
        xcd_of[i] = best;
        load[best] += work[i];
    }
    // chunk tables
    std::vector<int> cin((size_t)(N / kBlock)), cim((size_t)(M / kBlock)), nc0(B), ncc(B), mc0(B), mcc(B);
    for (int i = 0; i < B; ++i) {
        nc0[i] = (int)(P->noff[i] / kBlock);
        ncc[i] = (int)(npad[i] / kBlock);
        mc0[i] = (int)(P->moff[i] / kBlock);
        mcc[i] = (int)(mpad[i] / kBlock);
        for (int k = 0; k < ncc[i]; ++k) cin[nc0[i] + k] = i;
        for (int k = 0; k < mcc[i]; ++k) cim[mc0[i] + k] = i;
    }

    auto setup = [&](auto tag) {
        using T = decltype(tag);
        BDev<T> &b = P->dev<T>();
        Dev<T> &d = b.d;
        d.n = N;
        d.m = M;
        d.m1 = 0;
        d.Dr = Dr;
        d.Dc = Dc;
        b.B = B;
        b.ncn = N / kBlock;
        b.ncm = M / kBlock;
        b.act_cn = b.act_cm = b.act_i = nullptr;
        b.acn = b.ncn;
        b.acm = b.ncm;
        b.aci = B;
        b.krp = d_rp; b.kci = d_ci; b.trp = d_tp; b.tci = d_ti;
        if (std::is_same<T, double>::value) {
            b.kv = (const T *)d_kv; b.tv = (const T *)d_tv;
            d.cs = (const T *)cs; d.ls = (const T *)ls; d.us = (const T *)us; d.qs = (const T *)qs;
        } else {
            T *kvT = A.make<T>(nnz), *tvT = A.make<T>(nnz);
            T *csT = A.make<T>(N), *lsT = A.make<T>(N), *usT = A.make<T>(N), *qsT = A.make<T>(M);
            HIPT(launch_from_double<T>(d_kv, kvT, nnz, st));
            HIPT(launch_from_double<T>(d_tv, tvT, nnz, st));
            HIPT(launch_from_double<T>(cs, csT, N, st));
            HIPT(launch_from_double<T>(ls, lsT, N, st));
            HIPT(launch_from_double<T>(us, usT, N, st));
            HIPT(launch_from_double<T>(qs, qsT, M, st));
            b.kv = kvT; b.tv = tvT;
            d.cs = csT; d.ls = lsT; d.us = usT; d.qs = qsT;
        }
        for (int k = 0; k < 2; ++k) {
            d.xb[k] = A.make<T>(N); d.yb[k] = A.make<T>(M); d.Kxb[k] = A.make<T>(M); d.KTyb[k] = A.make<T>(N);
        }
        d.xa = A.make<T>(N); d.ya = A.make<T>(M); d.Kxa = A.make<T>(M); d.KTya = A.make<T>(N);
        d.x0 = A.make<T>(N); d.y0 = A.make<T>(M); d.Kx0 = A.make<T>(M); d.KTy0 = A.make<T>(N);
        d.xo = A.make<T>(N); d.yo = A.make<T>(M); d.KTyo = A.make<T>(N);
        b.prodK = A.make<T>(M);
        b.prodKT = A.make<T>(N);
        // Zero every iterate vector: lp_batch_set_state writes only each
        // instance's own entries, and the chunk padding must read as the
        // inert zeros a cold start writes (a resume's first primal trial
        // sums |x' - x|^2 over whole chunks, padding included).
        for (int k = 0; k < 2; ++k)
            for (auto pv : {std::make_pair((void *)d.xb[k], N), std::make_pair((void *)d.yb[k], M),
                            std::make_pair((void *)d.Kxb[k], M), std::make_pair((void *)d.KTyb[k], N)})
                HIPT(hipMemsetAsync(pv.first, 0, sizeof(T) * (size_t)std::max<int64_t>(pv.second, 1), st));
        for (auto pv : {std::make_pair((void *)d.xa, N), std::make_pair((void *)d.ya, M), std::make_pair((void *)d.Kxa, M),
                        std::make_pair((void *)d.KTya, N), std::make_pair((void *)d.x0, N), std::make_pair((void *)d.y0, M),
                        std::make_pair((void *)d.Kx0, M), std::make_pair((void *)d.KTy0, N), std::make_pair((void *)d.xo, N),
                        std::make_pair((void *)d.yo, M), std::make_pair((void *)d.KTyo, N),
                        std::make_pair((void *)b.prodK, M), std::make_pair((void *)b.prodKT, N)})
            HIPT(hipMemsetAsync(pv.first, 0, sizeof(T) * (size_t)std::max<int64_t>(pv.second, 1), st));
        d.part_primal = A.make<double>(b.ncn);
        d.part_dual = A.make<double>(2 * (int64_t)b.ncm);
        d.part_check = A.make<double>((int64_t)kCheckSums * (b.ncn + b.ncm));
        d.part_ray = A.make<double>((int64_t)kRaySums * (b.ncn + b.ncm));
        b.ctl = A.make<Ctl>(B);
        d.ctl = b.ctl;
        b.gate = A.make<int>(1);
        HIPT(hipMemsetAsync(b.gate, 0, sizeof(int), st));
        int *d_cin = A.make<int>(b.ncn), *d_cim = A.make<int>(b.ncm);
        int *d_nc0 = A.make<int>(B), *d_ncc = A.make<int>(B), *d_mc0 = A.make<int>(B), *d_mcc = A.make<int>(B);
        int *d_m1g = A.make<int>(B);
        double *d_Nq = A.make<double>(B), *d_Nc = A.make<double>(B);
        h2d(st, d_cin, cin.data(), b.ncn);
        h2d(st, d_cim, cim.data(), b.ncm);
        h2d(st, d_nc0, nc0.data(), B);
        h2d(st, d_ncc, ncc.data(), B);
        h2d(st, d_mc0, mc0.data(), B);
        h2d(st, d_mcc, mcc.data(), B);
        h2d(st, d_m1g, m1g.data(), B);
        h2d(st, d_Nq, P->Nq.data(), B);
        h2d(st, d_Nc, P->Nc.data(), B);
        b.cinst_n = d_cin; b.cinst_m = d_cim;
        b.nc0 = d_nc0; b.ncc = d_ncc; b.mc0 = d_mc0; b.mcc = d_mcc;
        b.m1g = d_m1g; b.Nq = d_Nq; b.Nc = d_Nc;
        b.LK = make_blocks(P, rp, P->moff, mpad, xcd_of);
        b.LT = make_blocks(P, tp, P->noff, npad, xcd_of);
        bsync(P);
        if (P->opt.autotune) {
            // row-block shapes timed on the actual block-diagonal matrix, per
            // product: the default and smaller nonzero and row limits
            const int cand[][2] = {{kStreamNB, kStreamRB}, {kStreamNB / 2, kStreamRB}, {kStreamNB, 256},
                                   {kStreamNB / 2, 256}};
            // vectors of ones in the trial buffers (overwritten by every solve's start)
            HIPT(launch_fill(P->stage_n0, 1.0, N, st));
            HIPT(launch_fill(P->stage_m, 1.0, M, st));
            HIPT(launch_from_double<T>(P->stage_n0, d.xb[1], N, st));
            HIPT(launch_from_double<T>(P->stage_m, d.yb[1], M, st));
            EventPair ev;
            for (int which = 0; which < 2; ++which) {
                BlockList &cur = which ? b.LT : b.LK;
                float best_ms = 0;
                int best = 0;
                for (int k = 0; k < 4; ++k) {
                    const BlockList L = k == 0 ? cur
                                               : make_blocks(P, which ? tp : rp, which ? P->noff : P->moff,
                                                             which ? npad : mpad, xcd_of, cand[k][0], cand[k][1]);
                    BDev<T> t = b;
                    (which ? t.LT : t.LK) = L;
                    const T *in = which ? d.yb[1] : d.xb[1];
                    T *out = which ? b.prodKT : b.prodK;
                    for (int r = 0; r < 2; ++r) HIPT(launch_batch_product_plain<T>(t, which, in, out, st));
                    HIPT(hipEventRecord(ev.a, st));
                    for (int r = 0; r < 5; ++r) HIPT(launch_batch_product_plain<T>(t, which, in, out, st));
                    HIPT(hipEventRecord(ev.b, st));
                    HIPT(hipEventSynchronize(ev.b));
                    const float ms = ev.ms();
                    if (P->opt.verbose)
                        fprintf(stderr, "[lp_batch] product %d: blocks of <= %d nonzeros, <= %d rows: %.3f ms\n",
                                which, cand[k][0], cand[k][1], ms / 5);
                    if (k == 0 || ms < 0.97f * best_ms) {   // 3% margin: near-ties keep the default shape
                        if (k > 0) release_blocks(P, cur);
                        cur = L;
                        best_ms = ms;
                        best = k;
                    } else {
                        release_blocks(P, L);
                    }
                }
                P->shape[which][0] = cand[best][0];
                P->shape[which][1] = cand[best][1];
            }
            // the trial vectors and products back to the zeros every iterate
            // vector holds after the load
            for (auto pv : {std::make_pair((void *)d.xb[1], N), std::make_pair((void *)d.yb[1], M),
                            std::make_pair((void *)b.prodK, M), std::make_pair((void *)b.prodKT, N)})
                HIPT(hipMemsetAsync(pv.first, 0, sizeof(T) * (size_t)std::max<int64_t>(pv.second, 1), st));
        }
    };
    if (P->mixed) setup(float{});
    else setup(double{});
    if (P->opt.persistent != 0) {
        if (P->mixed) setup_small<float>(P, rp, ci, tp, ti);
        else setup_small<double>(P, rp, ci, tp, ti);
    }
    P->cin = std::move(cin);
    P->cim = std::move(cim);
    // controller blocks start zeroed (buffer 0 current)
    HIPT(hipMemcpyAsync(P->mixed ? P->b32.ctl : P->b64.ctl, P->hctl, sizeof(Ctl) * (size_t)B, hipMemcpyHostToDevice,
                        st));
    bsync(P);
    for (void *pp : {(void *)r, (void *)s, (void *)d_c, (void *)d_l, (void *)d_u, (void *)d_q}) A.release(pp);
    if (P->mixed) {
        // kept for the FP64 re-check of termination tests passed on FP32 products
        P->kv64 = d_kv; P->tv64 = d_tv; P->cs64 = cs; P->ls64 = ls; P->us64 = us; P->qs64 = qs;
        P->g_rp = d_rp; P->g_ci = d_ci; P->g_tp = d_tp; P->g_ti = d_ti;
        int64_t mmax = 1, nmax = 1;
        for (int i = 0; i < B; ++i) {
            mmax = std::max(mmax, P->m[i]);
            nmax = std::max(nmax, P->n[i]);
        }
        for (int k = 0; k < 2; ++k) {
            P->ckx[k] = A.make<double>(mmax);
            P->ckty[k] = A.make<double>(nmax);
        }
        P->cpart = A.make<double>((int64_t)kMaxGrid * kCheckSums);
    }
    return LP_OK;
}

// Launch only for unfinished instances: the elementwise and check kernels
// get the chunks of the instances with live[i] set, the decision kernels
// those instances, the products their row blocks (each XCD's list keeps its
// order).  Finished instances would otherwise still cost a workgroup per
// chunk in every launch (the kernels skip them, but they are dispatched).
// Each chunk's partial keeps its slot, so the sums are those of the full
// launches.  live = nullptr restores the full lists.  The caller captures
// the window again afterwards.
template <typename T>
void compact_active(lp_batch *P, const std::vector<char> *live)
{
    BDev<T> &b = P->dev<T>();
    hipStream_t st = P->stream;
    if (P->active < 0) {   // the full lists are current: keep them, with host copies
        for (int w = 0; w < 2; ++w) {
            const BlockList &L = w ? b.LT : b.LK;
            P->full[w] = L;
            P->lorder[w].resize((size_t)std::max(L.nblk, 1));
            P->linst[w].resize((size_t)std::max(L.nblk, 1));
            if (L.nblk > 0) {
                HIPT(hipMemcpyAsync(P->lorder[w].data(), L.order, sizeof(int) * (size_t)L.nblk,
                                    hipMemcpyDeviceToHost, st));
                HIPT(hipMemcpyAsync(P->linst[w].data(), L.inst, sizeof(int) * (size_t)L.nblk,
                                    hipMemcpyDeviceToHost, st));
            }
            if (!P->act_order[w]) P->act_order[w] = P->arena.make<int>(L.nblk);
        }
        if (!P->act_cn) P->act_cn = P->arena.make<int>(b.ncn);
        if (!P->act_cm) P->act_cm = P->arena.make<int>(b.ncm);
        if (!P->act_i) P->act_i = P->arena.make<int>(b.B);
        bsync(P);
    }
    if (!live) {
        b.LK = P->full[0];
        b.LT = P->full[1];
        b.act_cn = b.act_cm = b.act_i = nullptr;
        b.acn = b.ncn;
        b.acm = b.ncm;
        b.aci = b.B;
        P->active = -1;
        return;
    }
    const std::vector<char> &on = *live;
    for (int w = 0; w < 2; ++w) {
        const BlockList &F = P->full[w];
        BlockList L = F;
        std::vector<int> ord;
        int maxper = 1;
        for (int x = 0; x < kXcds; ++x) {
            L.xoff[x] = (int)ord.size();
            for (int k = F.xoff[x]; k < F.xoff[x + 1]; ++k) {
                const int blk = P->lorder[w][(size_t)k];
                if (on[(size_t)P->linst[w][(size_t)blk]]) ord.push_back(blk);
            }
            maxper = std::max(maxper, (int)ord.size() - L.xoff[x]);
        }
        L.xoff[kXcds] = (int)ord.size();
        L.grid = kXcds * std::min(maxper, 512);
        L.order = P->act_order[w];
        h2d(st, P->act_order[w], ord.data(), (int64_t)ord.size());
        bsync(P);   // ord is a local
        (w ? b.LT : b.LK) = L;
    }
    std::vector<int> cn, cm, ins;
    for (int c = 0; c < b.ncn; ++c)
        if (on[(size_t)P->cin[(size_t)c]]) cn.push_back(c);
    for (int c = 0; c < b.ncm; ++c)
        if (on[(size_t)P->cim[(size_t)c]]) cm.push_back(c);
    for (int i = 0; i < b.B; ++i)
        if (on[(size_t)i]) ins.push_back(i);
    h2d(st, P->act_cn, cn.data(), (int64_t)cn.size());
    h2d(st, P->act_cm, cm.data(), (int64_t)cm.size());
    h2d(st, P->act_i, ins.data(), (int64_t)ins.size());
    bsync(P);
    b.act_cn = P->act_cn;
    b.act_cm = P->act_cm;
    b.act_i = P->act_i;
    b.acn = (int)cn.size();
    b.acm = (int)cm.size();
    b.aci = (int)ins.size();
    P->active = b.aci;
}

template <typename T>
void batch_slot(lp_batch *P)
{
    BDev<T> &b = P->dev<T>();
    hipStream_t st = P->stream;
    HIPT(launch_batch_product<T>(b, 0, st));
    HIPT(launch_batch_dual<T>(b, st));
    HIPT(launch_batch_step_decide<T>(b, st));
    HIPT(launch_batch_product<T>(b, 1, st));
    HIPT(launch_batch_update<T>(b, st));
    HIPT(launch_batch_check<T>(b, 1, st));
}

void put_ctls(lp_batch *P, Ctl *d)
{
    HIPT(hipMemcpyAsync(d, P->hctl, sizeof(Ctl) * (size_t)P->B, hipMemcpyHostToDevice, P->stream));
    bsync(P);
}

void get_ctls(lp_batch *P, const Ctl *d)
{
    HIPT(hipMemcpyAsync(P->hctl, d, sizeof(Ctl) * (size_t)P->B, hipMemcpyDeviceToHost, P->stream));
    bsync(P);
}

Ctl fresh_ctl(const lp_batch *P, int i, double tol, int64_t max_iters)
{
    Ctl c{};
    c.eta = P->eta0[i];
    c.omega = P->omega0[i];
    c.KKT_prev = INFINITY;
    c.tol = tol;
    c.infeas_tol = P->opt.infeas_tol;
    c.kkt_p = P->opt.kkt_omega_power;
    c.fixed_eta = P->opt.fixed_eta;
    c.max_iters = max_iters;
    c.check_every = P->opt.check_every;
    c.fixed_step = P->opt.fixed_step;
    c.final_status = LP_ITERATION_LIMIT;
    c.confirm_on = P->mixed ? 1 : 0;
    return c;
}

// Mixed precision: instances whose termination test passed on FP32 products
// stopped with `confirm` set.  Each is re-checked with FP64 products of the
// FP64 scaled matrix (its rows of the batch's CSR pair, gathering from the
// batch's vectors): confirmed, it ends OPTIMAL with the FP64 quantities;
// otherwise its check decision runs again without the termination test
// (restart logic, next primal trial) and it resumes in the next window.
// Returns whether any instance was re-checked (the host controllers are then
// current again).
template <typename T>
bool resolve_batch_confirms(lp_batch *P)
{
    if (!P->mixed) return false;
    BDev<T> &b = P->dev<T>();
    const Dev<T> &d = b.d;
    hipStream_t st = P->stream;
    bool any = false;
    for (int i = 0; i < P->B; ++i) {
        const Ctl &c = P->hctl[i];
        if (!c.confirm) continue;
        any = true;
        const int64_t mo = P->moff[i], no = P->noff[i];
        const Dev<T> v = view_of<T>(P, i);
        Conf64 cf{};
        cf.rp = P->g_rp + mo; cf.ci = P->g_ci; cf.kv = P->kv64;
        cf.tp = P->g_tp + no; cf.ti = P->g_ti; cf.tv = P->tv64;
        cf.cs = P->cs64 + no; cf.ls = P->ls64 + no; cf.us = P->us64 + no; cf.qs = P->qs64 + mo;
        for (int k = 0; k < 2; ++k) {
            cf.kx[k] = P->ckx[k];
            cf.kty[k] = P->ckty[k];
        }
        cf.part = P->cpart;
        Geo g{};
        g.vb_n = (int)((v.n + kBlock - 1) / kBlock);
        g.vb_m = (int)((v.m + kBlock - 1) / kBlock);
        g.grid = std::max(1, std::min(kMaxGrid, g.vb_n + g.vb_m));
        const int cur = c.cur;
        HIPT(launch_confirm_gather<T>(v, g, cf, cur, (const T *)d.xb[cur], (const T *)d.xa, (const T *)d.yb[cur],
                                      (const T *)d.ya, P->Nq[i], P->Nc[i], st));
    }
    if (!any) return false;
    // the vetoed instances' check decisions (the confirmed ones only copy
    // out); every other instance is kept out of these check kernels (an
    // instance whose last slot was a check still has that check's mode; its
    // next step decision sets the mode afresh)
    std::vector<char> conf((size_t)P->B);
    for (int i = 0; i < P->B; ++i) conf[(size_t)i] = P->hctl[i].confirm ? 1 : 0;
    get_ctls(P, b.ctl);
    for (int i = 0; i < P->B; ++i)
        if (!conf[(size_t)i]) P->hctl[i].mode = MODE_NONE;
    put_ctls(P, b.ctl);
    HIPT(launch_batch_check<T>(b, 0, st));
    get_ctls(P, b.ctl);
    return true;
}

template <typename T>
int do_batch_solve(lp_batch *P, double tol, int64_t max_iters, double time_limit)
{
    BDev<T> &b = P->dev<T>();
    Dev<T> &d = b.d;
    hipStream_t st = P->stream;
    const int B = P->B;
    const int64_t N = P->Ntot, M = P->Mtot;
    auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    // a solve starts with every instance's chunks and blocks in the lists
    // (the start products below need all of them)
    const bool narrowed = P->active >= 0;
    if (narrowed) compact_active<T>(P, nullptr);
    const bool resume = std::all_of(P->state_set.begin(), P->state_set.end(), [](char v) { return v != 0; }) && B > 0;
    if (!resume) {
        HIPT(launch_batch_start<T>(b, st));
        for (int i = 0; i < B; ++i) {
            P->hctl[i] = fresh_ctl(P, i, tol, max_iters);
            P->hctl[i].mode = MODE_INIT;
        }
        put_ctls(P, b.ctl);
        HIPT(launch_batch_product_plain<T>(b, 0, d.xb[0], d.Kxb[0], st));
        HIPT(launch_batch_product_plain<T>(b, 1, d.yb[0], d.KTyb[0], st));
        d2d(st, d.xa, (const T *)d.xb[0], N);
        d2d(st, d.x0, (const T *)d.xb[0], N);
        d2d(st, d.KTya, (const T *)d.KTyb[0], N);
        d2d(st, d.ya, (const T *)d.yb[0], M);
        d2d(st, d.y0, (const T *)d.yb[0], M);
        d2d(st, d.Kxa, (const T *)d.Kxb[0], M);
        d2d(st, d.Kx0, (const T *)d.Kxb[0], M);
        d2d(st, d.KTy0, (const T *)d.KTyb[0], N);
        HIPT(launch_batch_check<T>(b, 0, st));
    } else {
        for (int i = 0; i < B; ++i) {
            Ctl &c = P->hctl[i];
            c.mode = MODE_RESUME;
            c.done = 0;
            c.status = LP_NOT_SOLVED;
            c.numerical = 0;
            c.restart_to = 0;
            c.copy_out = 0;
            c.need_primal = 1;
            c.tol = tol;
            c.infeas_tol = P->opt.infeas_tol;
            c.max_iters = max_iters;
            c.kkt_p = P->opt.kkt_omega_power;
            c.check_every = P->opt.check_every;
            c.fixed_step = P->opt.fixed_step;
            c.fixed_eta = P->opt.fixed_eta;
            c.confirm_on = P->mixed ? 1 : 0;
            c.confirm = 0;
            c.veto = 0;
        }
        put_ctls(P, b.ctl);
        // the anchor's products (the state holds the anchor, not its products)
        HIPT(launch_batch_product_plain<T>(b, 0, d.x0, d.Kx0, st));
        HIPT(launch_batch_product_plain<T>(b, 1, d.y0, d.KTy0, st));
        // resume only needs the first primal trial: the apply step alone
        HIPT(launch_batch_apply<T>(b, st));
    }
    std::fill(P->state_set.begin(), P->state_set.end(), 0);
    get_ctls(P, b.ctl);
    bool any_at_limit = false;
    for (int i = 0; i < B; ++i)
        if (!P->hctl[i].done && P->hctl[i].k >= max_iters) any_at_limit = true;
    if (any_at_limit) {
        HIPT(launch_batch_set_final(b.ctl, B, LP_ITERATION_LIMIT, st));
        HIPT(launch_batch_check<T>(b, 0, st));
        get_ctls(P, b.ctl);
        resolve_batch_confirms<T>(P);
    }
    P->finish_s.assign(B, -1.0);
    const int W = std::max(1, P->opt.window);
    if (P->small_R > 0) {
        // a workgroup per instance runs its whole loop (up to small_slots
        // attempt slots per launch); the host polls between launches
        auto progress = [&] {
            long long s = 0;
            for (int i = 0; i < B; ++i) s += P->hctl[i].k + P->hctl[i].attempts;
            return s;
        };
        int left = 0;
        const double now0 = elapsed();
        for (int i = 0; i < B; ++i) {
            if (P->hctl[i].done && P->finish_s[i] < 0) P->finish_s[i] = now0;
            if (!P->hctl[i].done) ++left;
        }
        while (left > 0) {
            const long long before = progress();
            HIPT(launch_small_loop_batch<T>((const Dev<T> *)P->small_devs, P->small_nq, P->small_nc, B, P->small_R,
                                            P->small_stage, P->small_slots, st));
            get_ctls(P, b.ctl);
            resolve_batch_confirms<T>(P);
            left = 0;
            const double now = elapsed();
            for (int i = 0; i < B; ++i) {
                if (P->hctl[i].done && P->finish_s[i] < 0) P->finish_s[i] = now;
                if (!P->hctl[i].done) ++left;
            }
            if (left > 0 && progress() == before) {
                P->err = "no step decision in a whole launch (controller stalled)";
                return LP_ERR_HIP;
            }
            if (left > 0 && time_limit > 0.0 && now > time_limit) {
                HIPT(launch_batch_set_final(b.ctl, B, LP_TIME_LIMIT, st));
                HIPT(launch_batch_check<T>(b, 0, st));
                get_ctls(P, b.ctl);
                resolve_batch_confirms<T>(P);
                break;
            }
        }
        bsync(P);
        P->seconds = elapsed();
        P->has_result = true;
        return LP_OK;
    }
    auto capture = [&] {
        if (P->graph) {
            (void)hipGraphExecDestroy(P->graph);
            P->graph = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPT(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        for (int s = 0; s < W; ++s) batch_slot<T>(P);
        HIPT(hipStreamEndCapture(st, &g));
        HIPT(hipGraphInstantiate(&P->graph, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        P->graph_window = W;
    };
    if (P->opt.use_graph && (!P->graph || P->graph_window != W || narrowed)) capture();
    auto note_finished = [&] {
        int left = 0;
        const double now = elapsed();
        for (int i = 0; i < B; ++i) {
            if (P->hctl[i].done && P->finish_s[i] < 0) P->finish_s[i] = now;
            if (!P->hctl[i].done) ++left;
        }
        return left;
    };
    int left = note_finished();
    while (left > 0) {
        if (P->opt.use_graph) HIPT(hipGraphLaunch(P->graph, st));
        else
            for (int s = 0; s < W; ++s) batch_slot<T>(P);
        get_ctls(P, b.ctl);
        resolve_batch_confirms<T>(P);
        left = note_finished();
        // narrow the launches to the unfinished instances each time their
        // count has halved
        if (left > 0 && 2 * left <= (P->active < 0 ? B : P->active)) {
            std::vector<char> live((size_t)B);
            for (int i = 0; i < B; ++i) live[(size_t)i] = P->hctl[i].done ? 0 : 1;
            compact_active<T>(P, &live);
            if (P->opt.use_graph) capture();
        }
        if (left > 0 && time_limit > 0.0 && elapsed() > time_limit) {
            HIPT(launch_batch_set_final(b.ctl, B, LP_TIME_LIMIT, st));
            HIPT(launch_batch_check<T>(b, 0, st));
            get_ctls(P, b.ctl);
            resolve_batch_confirms<T>(P);
            left = note_finished();
            break;
        }
    }
    bsync(P);
    P->seconds = elapsed();
    P->has_result = true;
    return LP_OK;
}

template <typename T>
int do_batch_result(lp_batch *P, int i, double *x, double *y, double *lam, lp_info *info)
{
    BDev<T> &b = P->dev<T>();
    if (x || y || lam) {
        HIPT(launch_result<T>(b.d, P->stage_n0, P->stage_m, P->stage_n1, P->stream));
        if (x) d2h(P->stream, x, (const double *)P->stage_n0 + P->noff[i], P->n[i]);
        if (lam) d2h(P->stream, lam, (const double *)P->stage_n1 + P->noff[i], P->n[i]);
        if (y) d2h(P->stream, y, (const double *)P->stage_m + P->moff[i], P->m[i]);
        bsync(P);
    }
    if (info) {
        Ctl c;
        HIPT(hipMemcpyAsync(&c, b.ctl + i, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
        bsync(P);
        info->status = c.status;
        info->pobj = c.out_pobj;
        info->dobj = c.out_dobj;
        info->rel_primal = c.out_rel_p;
        info->rel_dual = c.out_rel_d;
        info->rel_gap = c.out_rel_g;
        info->iterations = c.k;
        info->attempts = c.attempts;
        info->restarts = c.restarts;
        info->omega = c.omega;
        info->eta = c.eta;
        info->seconds = P->finish_s.empty() ? 0.0 : P->finish_s[i];
    }
    return LP_OK;
}

template <typename T>
void state_vecs(lp_batch *P, int cur, T *(&v)[10], bool (&is_n)[10])
{
    Dev<T> &d = P->dev<T>().d;
    T *list[10] = {d.xb[cur], d.yb[cur], d.Kxb[cur], d.KTyb[cur], d.xa, d.ya, d.Kxa, d.KTya, d.x0, d.y0};
    const bool nn[10] = {true, false, false, true, true, false, false, true, true, false};
    for (int k = 0; k < 10; ++k) {
        v[k] = list[k];
        is_n[k] = nn[k];
    }
}

template <typename T>
int do_batch_get_state(lp_batch *P, int i, double *buf)
{
    BDev<T> &b = P->dev<T>();
    Ctl c;
    HIPT(hipMemcpyAsync(&c, b.ctl + i, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
    bsync(P);
    std::fill(buf, buf + kNScalars, 0.0);
    buf[0] = c.eta; buf[1] = c.omega; buf[2] = c.W; buf[3] = c.KKT0; buf[4] = c.KKT_prev;
    buf[5] = (double)c.k; buf[6] = (double)c.t; buf[7] = (double)c.attempts; buf[8] = (double)c.restarts;
    buf[9] = c.status; buf[10] = c.eta_last;
    T *v[10];
    bool is_n[10];
    state_vecs<T>(P, c.cur, v, is_n);
    double *p = buf + kNScalars;
    for (int k = 0; k < 10; ++k) {
        const int64_t len = is_n[k] ? P->n[i] : P->m[i];
        const int64_t off = is_n[k] ? P->noff[i] : P->moff[i];
        double *stage = is_n[k] ? P->stage_n0 : P->stage_m;
        HIPT(launch_to_double<T>(v[k] + off, stage, len, P->stream));
        d2h(P->stream, p, (const double *)stage, len);
        bsync(P);
        p += len;
    }
    return LP_OK;
}

template <typename T>
int do_batch_set_state(lp_batch *P, int i, const double *buf)
{
    BDev<T> &b = P->dev<T>();
    Ctl c{};
    HIPT(hipMemcpyAsync(&c, b.ctl + i, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
    bsync(P);
    const int old_cur = c.cur;
    c.eta = buf[0]; c.omega = buf[1]; c.W = buf[2]; c.KKT0 = buf[3]; c.KKT_prev = buf[4];
    c.k = (long long)buf[5]; c.t = (long long)buf[6]; c.attempts = (long long)buf[7];
    c.restarts = (long long)buf[8]; c.eta_last = buf[10];
    // the state goes to the instance's current buffers
    c.cur = old_cur;
    T *v[10];
    bool is_n[10];
    state_vecs<T>(P, c.cur, v, is_n);
    const double *p = buf + kNScalars;
    for (int k = 0; k < 10; ++k) {
        const int64_t len = is_n[k] ? P->n[i] : P->m[i];
        const int64_t off = is_n[k] ? P->noff[i] : P->moff[i];
        double *stage = is_n[k] ? P->stage_n0 : P->stage_m;
        h2d(P->stream, stage, p, len);
        HIPT(launch_from_double<T>(stage, v[k] + off, len, P->stream));
        bsync(P);
        p += len;
    }
    P->hctl[i] = c;
    HIPT(hipMemcpyAsync(b.ctl + i, &P->hctl[i], sizeof(Ctl), hipMemcpyHostToDevice, P->stream));
    bsync(P);
    P->state_set[i] = 1;
    return LP_OK;
}

}  // namespace

extern "C" {

int lp_batch_load(lp_batch **out, int32_t count, const lp_csr *K, const double *const *c, const double *const *q,
                  const double *const *l, const double *const *u, const int64_t *m1, const lp_options *opt)
{
    if (!out) return LP_ERR_ARG;
    *out = nullptr;
    if (count <= 0 || !K || !c || !q || !l || !u || !m1) return LP_ERR_ARG;
    if (opt && (opt->ptr_kind != LP_HOST || opt->workspace || opt->presolve)) return LP_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const int rc = validate_lp(&K[i], c[i], q[i], l[i], u[i], m1[i]);
        if (rc != LP_OK) return rc;
    }
    lp_options o;
    if (opt) o = *opt;
    else lp_default_options(&o);
    if ((o.precision != LP_FP64 && o.precision != LP_MIXED) || o.check_every <= 0 || o.ruiz_iters < 0 ||
        (o.fixed_step && !(o.fixed_eta > 0.0)) || o.window <= 0 || !(o.infeas_tol >= 0.0) ||
        std::isinf(o.infeas_tol) || o.split_sums < -1 || o.split_sums > 1)
        return LP_ERR_ARG;
    std::unique_ptr<lp_batch> P(new lp_batch());
    P->B = count;
    P->opt = o;
    P->mixed = o.precision == LP_MIXED;
    P->stream = (hipStream_t)o.stream;
    for (int i = 0; i < count; ++i) {
        P->n.push_back(K[i].n);
        P->m.push_back(K[i].m);
        P->m1.push_back(m1[i]);
    }
    P->state_set.assign(count, 0);
    int rc;
    try {
        if (!P->stream) {
            HIPT(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
            P->own_stream = true;
        }
        HIPT(hipHostMalloc((void **)&P->hctl, sizeof(Ctl) * (size_t)count, hipHostMallocDefault));
        std::memset(P->hctl, 0, sizeof(Ctl) * (size_t)count);
        rc = do_batch_load(P.get(), K, c, q, l, u);
    } catch (const HipError &h) {
        rc = fail(P.get(), h);
    } catch (const std::bad_alloc &) {
        rc = LP_ERR_NOMEM;
    }
    if (rc != LP_OK) return rc;
    *out = P.release();
    return LP_OK;
}

int lp_batch_solve(lp_batch *P, double tol, int64_t max_iters, double time_limit_s)
{
    if (!P || max_iters < 0 || std::isnan(tol)) return LP_ERR_ARG;
    try {
        return P->mixed ? do_batch_solve<float>(P, tol, max_iters, time_limit_s)
                        : do_batch_solve<double>(P, tol, max_iters, time_limit_s);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_batch_result(const lp_batch *Pc, int32_t i, double *x, double *y, double *lambda, lp_info *info)
{
    lp_batch *P = const_cast<lp_batch *>(Pc);
    if (!P || i < 0 || i >= P->B) return LP_ERR_ARG;
    if (!P->has_result) return LP_ERR_STATE;
    try {
        return P->mixed ? do_batch_result<float>(P, i, x, y, lambda, info)
                        : do_batch_result<double>(P, i, x, y, lambda, info);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_batch_get_state(const lp_batch *Pc, int32_t i, double *buf, int64_t *len)
{
    lp_batch *P = const_cast<lp_batch *>(Pc);
    if (!P || !len || i < 0 || i >= P->B) return LP_ERR_ARG;
    *len = kNScalars + 5 * P->n[i] + 5 * P->m[i];
    if (!buf) return LP_OK;
    try {
        return P->mixed ? do_batch_get_state<float>(P, i, buf) : do_batch_get_state<double>(P, i, buf);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_batch_set_state(lp_batch *P, int32_t i, const double *buf, int64_t len)
{
    if (!P || !buf || i < 0 || i >= P->B) return LP_ERR_ARG;
    if (len != kNScalars + 5 * P->n[i] + 5 * P->m[i]) return LP_ERR_STATE;
    try {
        return P->mixed ? do_batch_set_state<float>(P, i, buf) : do_batch_set_state<double>(P, i, buf);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_batch_layout_blocks(const lp_batch *P, int which, int *nnz_per_block, int *rows_per_block)
{
    if (!P || (which != 0 && which != 1)) return LP_ERR_ARG;
    if (nnz_per_block) *nnz_per_block = P->shape[which][0];
    if (rows_per_block) *rows_per_block = P->shape[which][1];
    return LP_OK;
}

int lp_batch_loop_form(const lp_batch *P, int *form)
{
    if (!P || !form) return LP_ERR_ARG;
    *form = P->small_R > 0 ? 1 : 0;
    return LP_OK;
}

int lp_batch_device_bytes(const lp_batch *P, int64_t *bytes)
{
    if (!P || !bytes) return LP_ERR_ARG;
    *bytes = P->arena.bytes;
    return LP_OK;
}

void lp_batch_free(lp_batch *P)
{
    if (!P) return;
    (void)hipStreamSynchronize(P->stream);
    delete P;
}

const char *lp_batch_last_error(const lp_batch *P) { return P ? P->err.c_str() : ""; }

}  // extern "C"
