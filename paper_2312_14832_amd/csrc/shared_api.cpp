// Host side of the shared-matrix batch (lp_shared_*): many LPs of one
// family (the same K, their own c, q, l, u) solved together.  K and K' are
// stored once; the iterates of all instances are interleaved so that every
// sparse product is one pass over K for all of them (an SpMM).  The method
// per instance is exactly the single-LP one: the same scaling (it depends on
// K alone, so every instance gets the same factors), the same start, step
// rule, checks and restarts, each with its own controller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "host_util.h"
#include "internal.h"

using namespace pdlp;

namespace {
constexpr int kNScalars = 16;
constexpr int kMaxShared = kBlock;   // instances per handle (the interleave width is at most one workgroup)
}  // namespace

struct lp_shared {
    int B = 0, Bp = 1, lgB = 0;
    int64_t n = 0, m = 0, m1 = 0, nnz = 0;
    lp_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool mixed = false;
    std::vector<double> Nq, Nc, omega0;
    double eta0 = 1.0;
    std::vector<double> Dr, Dc;               // host copies of the scaling (for the start norms)
    Arena arena;
    SDev<double> s64{};
    SDev<float> s32{};
    Ctl *hctl = nullptr;                      // pinned mirror, Bp entries
    double *stage_n0 = nullptr, *stage_n1 = nullptr, *stage_m = nullptr;   // interleaved FP64 staging
    double *pick_n = nullptr, *pick_m = nullptr;                           // one instance's vector
    double *start_x = nullptr, *start_y = nullptr;                         // interleaved start (unscaled)
    std::vector<char> has_start;
    std::vector<double> omega_start;
    // Mixed precision's FP64 re-check of a passed termination test (as
    // lp_solve's): the FP64 scaled matrices and interleaved vectors kept from
    // the load, the scaling as plain vectors, and one instance's FP64 copies
    const double *kv64 = nullptr, *tv64 = nullptr, *cs64 = nullptr, *ls64 = nullptr, *us64 = nullptr,
                 *qs64 = nullptr;
    double *cDr = nullptr, *cDc = nullptr, *cvec[10] = {}, *ckx[2] = {}, *ckty[2] = {}, *cpart = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_window = 0;
    bool has_result = false, result_ready = false;
    std::vector<char> state_set;
    std::vector<double> finish_s;
    double seconds = 0;
    std::string err;

    template <typename T> SDev<T> &dev();
    ~lp_shared()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (hctl) (void)hipHostFree(hctl);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

template <> SDev<double> &lp_shared::dev<double>() { return s64; }
template <> SDev<float> &lp_shared::dev<float>() { return s32; }

namespace {

void ssync(lp_shared *P) { HIPT(hipStreamSynchronize(P->stream)); }

int fail(lp_shared *P, const HipError &h)
{
    char buf[512];
    snprintf(buf, sizeof(buf), "%s failed: %s", h.what, hipGetErrorString(h.e));
    if (P) P->err = buf;
    return h.e == hipErrorOutOfMemory ? LP_ERR_NOMEM : LP_ERR_HIP;
}

// The per-instance vector rules of lp_load (K is validated once).
int validate_vectors(int64_t n, int64_t m, const double *c, const double *q, const double *l, const double *u)
{
    if ((n > 0 && (!c || !l || !u)) || (m > 0 && !q)) return LP_ERR_ARG;
    for (int64_t j = 0; j < n; ++j)
        if (!std::isfinite(c[j])) return LP_ERR_NAN;
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(q[i])) return LP_ERR_NAN;
    for (int64_t j = 0; j < n; ++j) {
        if (std::isnan(l[j]) || std::isnan(u[j])) return LP_ERR_NAN;
        if (l[j] > u[j] || l[j] == INFINITY || u[j] == -INFINITY) return LP_ERR_BOUNDS;
    }
    return LP_OK;
}

// rows of a CSR longer than kLongRow (scaled on grids of their own)
std::vector<int> long_rows(const std::vector<int> &rp)
{
    std::vector<int> out;
    for (size_t r = 0; r + 1 < rp.size(); ++r)
        if (rp[r + 1] - rp[r] > kLongRow) out.push_back((int)r);
    return out;
}

template <typename T>
void setup(lp_shared *P, const std::vector<int> &rp, const std::vector<int> &ci, const std::vector<int> &tp,
           const std::vector<int> &ti, const double *kv64, const double *tv64, const double *cs, const double *ls,
           const double *us, const double *qs, const double *Drr, const double *Dcr)
{
    Arena &A = P->arena;
    hipStream_t st = P->stream;
    SDev<T> &S = P->dev<T>();
    Dev<T> &d = S.d;
    const int64_t N = P->n * P->Bp, M = P->m * P->Bp, nnz = P->nnz;
    S.B = P->B;
    S.Bp = P->Bp;
    S.lgB = P->lgB;
    S.n = (int)P->n;
    S.m = (int)P->m;
    d.n = (int)N;
    d.m = (int)M;
    d.m1 = (int)(P->m1 * P->Bp);
    d.Dr = Drr;
    d.Dc = Dcr;
    int *krp = A.make<int>(P->m + 1), *kci = A.make<int>(nnz), *trp = A.make<int>(P->n + 1), *tci = A.make<int>(nnz);
    h2d(st, krp, rp.data(), P->m + 1);
    h2d(st, kci, ci.data(), nnz);
    h2d(st, trp, tp.data(), P->n + 1);
    h2d(st, tci, ti.data(), nnz);
    T *kv = A.make<T>(nnz), *tv = A.make<T>(nnz);
    HIPT(launch_from_double<T>(kv64, kv, nnz, st));
    HIPT(launch_from_double<T>(tv64, tv, nnz, st));
    S.krp = krp; S.kci = kci; S.kv = kv;
    S.trp = trp; S.tci = tci; S.tv = tv;
    if (std::is_same<T, double>::value) {
        d.cs = (const T *)cs; d.ls = (const T *)ls; d.us = (const T *)us; d.qs = (const T *)qs;
    } else {
        T *c2 = A.make<T>(N), *l2 = A.make<T>(N), *u2 = A.make<T>(N), *q2 = A.make<T>(M);
        HIPT(launch_from_double<T>(cs, c2, N, st));
        HIPT(launch_from_double<T>(ls, l2, N, st));
        HIPT(launch_from_double<T>(us, u2, N, st));
        HIPT(launch_from_double<T>(qs, q2, M, st));
        d.cs = c2; d.ls = l2; d.us = u2; d.qs = q2;
    }
    for (int k = 0; k < 2; ++k) {
        d.xb[k] = A.make<T>(N); d.yb[k] = A.make<T>(M); d.Kxb[k] = A.make<T>(M); d.KTyb[k] = A.make<T>(N);
    }
    d.xa = A.make<T>(N); d.ya = A.make<T>(M); d.Kxa = A.make<T>(M); d.KTya = A.make<T>(N);
    d.x0 = A.make<T>(N); d.y0 = A.make<T>(M); d.Kx0 = A.make<T>(M); d.KTy0 = A.make<T>(N);
    d.xo = A.make<T>(N); d.yo = A.make<T>(M); d.KTyo = A.make<T>(N);
    // every iterate vector starts at zero (a state set for one instance leaves the others' entries alone)
    for (T *p : {d.xb[0], d.xb[1], d.KTyb[0], d.KTyb[1], d.xa, d.KTya, d.x0, d.KTy0, d.xo, d.KTyo})
        HIPT(hipMemsetAsync(p, 0, sizeof(T) * (size_t)std::max<int64_t>(N, 1), st));
    for (T *p : {d.yb[0], d.yb[1], d.Kxb[0], d.Kxb[1], d.ya, d.Kxa, d.y0, d.Kx0, d.yo})
        HIPT(hipMemsetAsync(p, 0, sizeof(T) * (size_t)std::max<int64_t>(M, 1), st));
    // the element walks: enough workgroups to cover the longer side, at most
    // 2048 (eight 256-thread workgroups per CU)
    const int64_t wn = (std::max(N, M) + kBlock - 1) / kBlock;
    S.grid = (int)std::max<int64_t>(1, std::min<int64_t>(wn, 2048));
    S.grid_m = (int)std::max<int64_t>(1, std::min<int64_t>((M + kBlock - 1) / kBlock, 2048));
    d.part_primal = A.make<double>((int64_t)S.grid * S.Bp);
    d.part_dual = A.make<double>((int64_t)S.grid_m * S.Bp * 2);
    d.part_check = A.make<double>((int64_t)S.grid * S.Bp * kCheckSums);
    d.part_ray = A.make<double>((int64_t)S.grid * S.Bp * kRaySums);
    S.ctl = A.make<Ctl>(S.Bp);
    d.ctl = S.ctl;
    S.gate = A.make<int>(1);
    HIPT(hipMemsetAsync(S.gate, 0, sizeof(int), st));
    double *nq = A.make<double>(S.Bp), *nc = A.make<double>(S.Bp);
    h2d(st, nq, P->Nq.data(), S.Bp);
    h2d(st, nc, P->Nc.data(), S.Bp);
    S.Nq = nq;
    S.Nc = nc;
    ssync(P);
}

int do_load(lp_shared *P, const lp_csr *K, const double *const *c, const double *const *q, const double *const *l,
            const double *const *u)
{
    const int B = P->B, Bp = P->Bp;
    const int64_t n = P->n, m = P->m;
    hipStream_t st = P->stream;
    std::vector<int> rp, ci, tp, ti;
    std::vector<double> kv, tv;
    rp.push_back(0);
    append_sorted_rows(K, 0, rp, ci, kv);
    transpose_csr((int)m, (int)n, rp, ci, kv, tp, ti, tv);
    const int64_t nnz = (int64_t)ci.size();
    P->nnz = nnz;
    // interleaved data; padded instances: zero data, bounds [0, 0]
    const int64_t N = n * Bp, M = m * Bp;
    std::vector<double> hc(N, 0.0), hl(N, 0.0), hu(N, 0.0), hq(M, 0.0);
    for (int b = 0; b < B; ++b) {
        for (int64_t j = 0; j < n; ++j) {
            hc[j * Bp + b] = c[b][j];
            hl[j * Bp + b] = l[b][j];
            hu[j * Bp + b] = u[b][j];
        }
        for (int64_t i = 0; i < m; ++i) hq[i * Bp + b] = q[b][i];
    }
    // unscaled norms per instance
    P->Nq.assign(Bp, 0.0);
    P->Nc.assign(Bp, 0.0);
    for (int b = 0; b < B; ++b) {
        double sq = 0.0, sc = 0.0;
        for (int64_t i = 0; i < m; ++i) sq += q[b][i] * q[b][i];
        for (int64_t j = 0; j < n; ++j) sc += c[b][j] * c[b][j];
        P->Nq[b] = std::sqrt(sq);
        P->Nc[b] = std::sqrt(sc);
    }
    Arena &A = P->arena;
    if (const char *fb = std::getenv("PDLP_DEBUG_FILL_BYTE")) A.fill = std::atoi(fb) & 255;
    // the scaling of K (one matrix for every instance)
    int *d_rp = A.make<int>(m + 1), *d_ci = A.make<int>(nnz), *d_tp = A.make<int>(n + 1), *d_ti = A.make<int>(nnz);
    double *d_kv = A.make<double>(nnz), *d_tv = A.make<double>(nnz);
    double *Dr = A.make<double>(m), *Dc = A.make<double>(n), *r = A.make<double>(m), *s = A.make<double>(n);
    h2d(st, d_rp, rp.data(), m + 1);
    h2d(st, d_ci, ci.data(), nnz);
    h2d(st, d_kv, kv.data(), nnz);
    h2d(st, d_tp, tp.data(), n + 1);
    h2d(st, d_ti, ti.data(), nnz);
    h2d(st, d_tv, tv.data(), nnz);
    const std::vector<int> klong = long_rows(rp), tlong = long_rows(tp);
    int *d_kl = A.make<int>((int64_t)klong.size()), *d_tl = A.make<int>((int64_t)tlong.size());
    h2d(st, d_kl, klong.data(), (int64_t)klong.size());
    h2d(st, d_tl, tlong.data(), (int64_t)tlong.size());
    HIPT(scale_csr_pair(d_rp, d_ci, d_kv, (int)m, d_tp, d_ti, d_tv, (int)n, Dr, Dc, r, s, P->opt.ruiz_iters,
                        P->opt.pc_alpha, st, d_kl, (int)klong.size(), d_tl, (int)tlong.size()));
    double *red_part = A.make<double>(kMaxGrid), *red_out = A.make<double>(1);
    HIPT(launch_absmax(d_kv, nnz, red_part, red_out, st));
    double kmax = 0.0;
    d2h(st, &kmax, (const double *)red_out, 1);
    P->Dr.resize(m);
    P->Dc.resize(n);
    d2h(st, P->Dr.data(), (const double *)Dr, m);
    d2h(st, P->Dc.data(), (const double *)Dc, n);
    ssync(P);
    P->eta0 = kmax > 0.0 ? 1.0 / kmax : 1.0;
    if (P->opt.fixed_step) P->eta0 = P->opt.fixed_eta;
    // the factors replicated per instance, the scaled interleaved vectors
    std::vector<double> hDr(M), hDc(N);
    for (int64_t i = 0; i < m; ++i)
        for (int b = 0; b < Bp; ++b) hDr[i * Bp + b] = P->Dr[i];
    for (int64_t j = 0; j < n; ++j)
        for (int b = 0; b < Bp; ++b) hDc[j * Bp + b] = P->Dc[j];
    double *Drr = A.make<double>(M), *Dcr = A.make<double>(N);
    double *d_c = A.make<double>(N), *d_l = A.make<double>(N), *d_u = A.make<double>(N), *d_q = A.make<double>(M);
    double *cs = A.make<double>(N), *ls = A.make<double>(N), *us = A.make<double>(N), *qs = A.make<double>(M);
    h2d(st, Drr, hDr.data(), M);
    h2d(st, Dcr, hDc.data(), N);
    h2d(st, d_c, hc.data(), N);
    h2d(st, d_l, hl.data(), N);
    h2d(st, d_u, hu.data(), N);
    h2d(st, d_q, hq.data(), M);
    HIPT(launch_scale_vectors(d_c, d_l, d_u, d_q, Dcr, Drr, cs, ls, us, qs, (int)N, (int)M, st));
    // omega0 = |c~| / |q~| per instance (1 if either is tiny)
    P->omega0.assign(Bp, 1.0);
    for (int b = 0; b < B; ++b) {
        double sq = 0.0, sc = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double t = q[b][i] / P->Dr[i];
            sq += t * t;
        }
        for (int64_t j = 0; j < n; ++j) {
            const double t = c[b][j] / P->Dc[j];
            sc += t * t;
        }
        const double nq = std::sqrt(sq), nc = std::sqrt(sc);
        P->omega0[b] = (nc > 1e-10 && nq > 1e-10) ? nc / nq : 1.0;
    }
    P->stage_n0 = A.make<double>(N);
    P->stage_n1 = A.make<double>(N);
    P->stage_m = A.make<double>(M);
    P->pick_n = A.make<double>(n);
    P->pick_m = A.make<double>(m);
    P->start_x = A.make<double>(N);
    P->start_y = A.make<double>(M);
    if (P->mixed) setup<float>(P, rp, ci, tp, ti, d_kv, d_tv, cs, ls, us, qs, Drr, Dcr);
    else setup<double>(P, rp, ci, tp, ti, d_kv, d_tv, cs, ls, us, qs, Drr, Dcr);
    for (void *pp : {(void *)d_rp, (void *)d_ci, (void *)d_tp, (void *)d_ti, (void *)r, (void *)s, (void *)Dr,
                     (void *)Dc, (void *)d_kl, (void *)d_tl, (void *)d_c, (void *)d_l, (void *)d_u, (void *)d_q,
                     (void *)red_part, (void *)red_out})
        A.release(pp);
    if (P->mixed) {
        // kept for the FP64 re-check of termination tests passed on FP32 products
        P->kv64 = d_kv; P->tv64 = d_tv; P->cs64 = cs; P->ls64 = ls; P->us64 = us; P->qs64 = qs;
        P->cDr = A.make<double>(m);
        P->cDc = A.make<double>(n);
        h2d(st, P->cDr, P->Dr.data(), m);
        h2d(st, P->cDc, P->Dc.data(), n);
        for (int k = 0; k < 10; ++k) P->cvec[k] = A.make<double>(k < 6 ? n : m);
        for (int k = 0; k < 2; ++k) {
            P->ckx[k] = A.make<double>(m);
            P->ckty[k] = A.make<double>(n);
        }
        P->cpart = A.make<double>((int64_t)kMaxGrid * kCheckSums);
    } else {
        A.release(d_kv);
        A.release(d_tv);
    }
    // the controllers: padded instances are finished from the start
    std::memset(P->hctl, 0, sizeof(Ctl) * (size_t)Bp);
    for (int b = B; b < Bp; ++b) P->hctl[b].done = 1;
    Ctl *dctl = P->mixed ? P->s32.ctl : P->s64.ctl;
    HIPT(hipMemcpyAsync(dctl, P->hctl, sizeof(Ctl) * (size_t)Bp, hipMemcpyHostToDevice, st));
    ssync(P);
    return LP_OK;
}

void put_ctls(lp_shared *P, Ctl *d)
{
    HIPT(hipMemcpyAsync(d, P->hctl, sizeof(Ctl) * (size_t)P->Bp, hipMemcpyHostToDevice, P->stream));
    ssync(P);
}

void get_ctls(lp_shared *P, const Ctl *d)
{
    HIPT(hipMemcpyAsync(P->hctl, d, sizeof(Ctl) * (size_t)P->Bp, hipMemcpyDeviceToHost, P->stream));
    ssync(P);
}

void apply_options(const lp_shared *P, Ctl &c, double tol, int64_t max_iters)
{
    c.tol = tol;
    c.infeas_tol = P->opt.infeas_tol;
    c.kkt_p = P->opt.kkt_omega_power;
    c.fixed_eta = P->opt.fixed_eta;
    c.max_iters = max_iters;
    c.check_every = P->opt.check_every;
    c.fixed_step = P->opt.fixed_step;
    c.final_status = LP_ITERATION_LIMIT;
    c.confirm_on = P->mixed ? 1 : 0;
    c.confirm = 0;
    c.veto = 0;
}

// Mixed precision: members whose termination test passed on FP32 products
// stopped with `confirm` set.  Each is re-checked with FP64 products of the
// FP64 scaled matrix on FP64 copies of its vectors: confirmed, it ends
// OPTIMAL with the FP64 quantities; otherwise its check decision runs again
// without the termination test and it resumes in the next window.
template <typename T>
void resolve_shared_confirms(lp_shared *P)
{
    if (!P->mixed) return;
    SDev<T> &S = P->dev<T>();
    const Dev<T> &d = S.d;
    hipStream_t st = P->stream;
    const int n = (int)P->n, m = (int)P->m;
    double *const *v = P->cvec;   // n-vectors x, x avg, x0, c~, l~, u~; m-vectors y, y avg, y0, q~
    std::vector<char> conf((size_t)P->Bp, 0);
    bool any = false;
    for (int b = 0; b < P->B; ++b) {
        const Ctl &c = P->hctl[b];
        if (!c.confirm) continue;
        any = true;
        conf[(size_t)b] = 1;
        const int cur = c.cur;
        HIPT(launch_shared_extract<T>(d.xb[cur], S.lgB, b, v[0], n, st));
        HIPT(launch_shared_extract<T>(d.xa, S.lgB, b, v[1], n, st));
        HIPT(launch_shared_extract<T>(d.x0, S.lgB, b, v[2], n, st));
        HIPT(launch_shared_extract<double>(P->cs64, S.lgB, b, v[3], n, st));
        HIPT(launch_shared_extract<double>(P->ls64, S.lgB, b, v[4], n, st));
        HIPT(launch_shared_extract<double>(P->us64, S.lgB, b, v[5], n, st));
        HIPT(launch_shared_extract<T>(d.yb[cur], S.lgB, b, v[6], m, st));
        HIPT(launch_shared_extract<T>(d.ya, S.lgB, b, v[7], m, st));
        HIPT(launch_shared_extract<T>(d.y0, S.lgB, b, v[8], m, st));
        HIPT(launch_shared_extract<double>(P->qs64, S.lgB, b, v[9], m, st));
        Dev<double> w{};   // member b as a plain FP64 LP (only what the re-check reads)
        w.m = m;
        w.n = n;
        w.m1 = (int)P->m1;
        w.Dr = P->cDr;
        w.Dc = P->cDc;
        w.xb[0] = w.xb[1] = v[0];
        w.xa = v[1];
        w.x0 = v[2];
        w.yb[0] = w.yb[1] = v[6];
        w.ya = v[7];
        w.y0 = v[8];
        w.ctl = S.ctl + b;
        Conf64 cf{};
        cf.rp = S.krp; cf.ci = S.kci; cf.kv = P->kv64;
        cf.tp = S.trp; cf.ti = S.tci; cf.tv = P->tv64;
        cf.cs = v[3]; cf.ls = v[4]; cf.us = v[5]; cf.qs = v[9];
        for (int k = 0; k < 2; ++k) {
            cf.kx[k] = P->ckx[k];
            cf.kty[k] = P->ckty[k];
        }
        cf.part = P->cpart;
        Geo g{};
        g.vb_n = (n + kBlock - 1) / kBlock;
        g.vb_m = (m + kBlock - 1) / kBlock;
        g.grid = std::max(1, std::min(kMaxGrid, g.vb_n + g.vb_m));
        HIPT(launch_confirm<double>(w, g, cf, 0, P->Nq[b], P->Nc[b], st));
    }
    if (!any) return;
    // the vetoed members' check decisions (the confirmed ones only copy out);
    // every other member is kept out of these check kernels (its next step
    // decision sets its mode afresh)
    get_ctls(P, S.ctl);
    for (int b = 0; b < P->Bp; ++b)
        if (!conf[(size_t)b]) P->hctl[b].mode = MODE_NONE;
    put_ctls(P, S.ctl);
    HIPT(launch_shared_check<T>(S, 0, st));
    get_ctls(P, S.ctl);
}

template <typename T>
int do_solve(lp_shared *P, double tol, int64_t max_iters, double time_limit)
{
    SDev<T> &S = P->dev<T>();
    Dev<T> &d = S.d;
    hipStream_t st = P->stream;
    const int B = P->B, Bp = P->Bp;
    const int64_t N = P->n * Bp, M = P->m * Bp;
    auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    const bool resume = std::all_of(P->state_set.begin(), P->state_set.end(), [](char v) { return v != 0; });
    P->result_ready = false;
    if (!resume) {
        // start: x = proj_X(start or 0), y = proj_Y(start or 0), per instance
        bool any_start = false;
        for (int b = 0; b < B; ++b) any_start = any_start || P->has_start[b];
        HIPT(launch_start<T>(d, any_start ? P->start_x : nullptr, any_start ? P->start_y : nullptr, 0, st));
        for (int b = 0; b < Bp; ++b) {
            Ctl c{};
            if (b < B) {
                c.eta = P->eta0;
                c.omega = P->omega_start[b] > 0.0 ? P->omega_start[b] : P->omega0[b];
                c.KKT_prev = INFINITY;
                c.mode = MODE_INIT;
                apply_options(P, c, tol, max_iters);
            } else {
                c.done = 1;
            }
            P->hctl[b] = c;
        }
        put_ctls(P, S.ctl);
        HIPT(launch_shared_product<T>(S, 0, d.xb[0], d.Kxb[0], st));
        HIPT(launch_shared_product<T>(S, 1, d.yb[0], d.KTyb[0], st));
        d2d(st, d.xa, (const T *)d.xb[0], N);
        d2d(st, d.x0, (const T *)d.xb[0], N);
        d2d(st, d.KTya, (const T *)d.KTyb[0], N);
        d2d(st, d.ya, (const T *)d.yb[0], M);
        d2d(st, d.y0, (const T *)d.yb[0], M);
        d2d(st, d.Kxa, (const T *)d.Kxb[0], M);
        d2d(st, d.Kx0, (const T *)d.Kxb[0], M);
        d2d(st, d.KTy0, (const T *)d.KTyb[0], N);
        HIPT(launch_shared_check<T>(S, 0, st));
    } else {
        // every instance's state was set (its vectors went to buffer 0)
        for (int b = 0; b < B; ++b) {
            Ctl &c = P->hctl[b];
            c.mode = MODE_RESUME;
            c.done = 0;
            c.status = LP_NOT_SOLVED;
            c.numerical = 0;
            c.restart_to = 0;
            c.copy_out = 0;
            c.need_primal = 1;
            c.cur = 0;
            apply_options(P, c, tol, max_iters);
        }
        put_ctls(P, S.ctl);
        HIPT(launch_shared_product<T>(S, 0, d.x0, d.Kx0, st));
        HIPT(launch_shared_product<T>(S, 1, d.y0, d.KTy0, st));
        HIPT(launch_shared_apply<T>(S, st));
    }
    std::fill(P->state_set.begin(), P->state_set.end(), 0);
    get_ctls(P, S.ctl);
    bool any_at_limit = false;
    for (int b = 0; b < B; ++b)
        if (!P->hctl[b].done && P->hctl[b].k >= max_iters) any_at_limit = true;
    if (any_at_limit) {
        HIPT(launch_shared_set_final(S.ctl, Bp, LP_ITERATION_LIMIT, st));
        HIPT(launch_shared_check<T>(S, 0, st));
        get_ctls(P, S.ctl);
        resolve_shared_confirms<T>(P);
    }
    P->finish_s.assign(B, -1.0);
    const int W = std::max(1, P->opt.window);
    if (P->opt.use_graph && (!P->graph || P->graph_window != W)) {
        if (P->graph) {
            (void)hipGraphExecDestroy(P->graph);
            P->graph = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPT(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        for (int s = 0; s < W; ++s) HIPT(launch_shared_slot<T>(S, st));
        HIPT(hipStreamEndCapture(st, &g));
        HIPT(hipGraphInstantiate(&P->graph, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        P->graph_window = W;
    }
    auto note_finished = [&] {
        int left = 0;
        const double now = elapsed();
        for (int b = 0; b < B; ++b) {
            if (P->hctl[b].done && P->finish_s[b] < 0) P->finish_s[b] = now;
            if (!P->hctl[b].done) ++left;
        }
        return left;
    };
    int left = note_finished();
    while (left > 0) {
        long long moved = 0;
        for (int b = 0; b < B; ++b) moved -= P->hctl[b].attempts;
        if (P->opt.use_graph) HIPT(hipGraphLaunch(P->graph, st));
        else
            for (int s = 0; s < W; ++s) HIPT(launch_shared_slot<T>(S, st));
        get_ctls(P, S.ctl);
        for (int b = 0; b < B; ++b) moved += P->hctl[b].attempts;
        resolve_shared_confirms<T>(P);
        left = note_finished();
        if (left > 0 && moved == 0) {
            // every slot takes a step decision for every unfinished instance
            P->err = "no step decision in a whole window (controller stalled)";
            return LP_ERR_HIP;
        }
        if (left > 0 && time_limit > 0.0 && elapsed() > time_limit) {
            HIPT(launch_shared_set_final(S.ctl, Bp, LP_TIME_LIMIT, st));
            HIPT(launch_shared_check<T>(S, 0, st));
            get_ctls(P, S.ctl);
            resolve_shared_confirms<T>(P);
            left = note_finished();
            break;
        }
    }
    ssync(P);
    P->seconds = elapsed();
    P->has_result = true;
    return LP_OK;
}

template <typename T>
int do_result(lp_shared *P, int i, double *x, double *y, double *lam, lp_info *info)
{
    SDev<T> &S = P->dev<T>();
    hipStream_t st = P->stream;
    if (x || y || lam) {
        if (!P->result_ready) {
            HIPT(launch_result<T>(S.d, P->stage_n0, P->stage_m, P->stage_n1, st));
            P->result_ready = true;
        }
        const int n = (int)P->n, m = (int)P->m;
        if (x) {
            HIPT(launch_shared_extract<double>(P->stage_n0, P->lgB, i, P->pick_n, n, st));
            d2h(st, x, (const double *)P->pick_n, n);
            ssync(P);
        }
        if (lam) {
            HIPT(launch_shared_extract<double>(P->stage_n1, P->lgB, i, P->pick_n, n, st));
            d2h(st, lam, (const double *)P->pick_n, n);
            ssync(P);
        }
        if (y) {
            HIPT(launch_shared_extract<double>(P->stage_m, P->lgB, i, P->pick_m, m, st));
            d2h(st, y, (const double *)P->pick_m, m);
            ssync(P);
        }
    }
    if (info) {
        Ctl c;
        HIPT(hipMemcpyAsync(&c, S.ctl + i, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        ssync(P);
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
void state_vecs(lp_shared *P, int cur, T *(&v)[10], bool (&is_n)[10])
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
int do_get_state(lp_shared *P, int i, double *buf)
{
    SDev<T> &S = P->dev<T>();
    hipStream_t st = P->stream;
    Ctl c;
    HIPT(hipMemcpyAsync(&c, S.ctl + i, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    ssync(P);
    std::fill(buf, buf + kNScalars, 0.0);
    buf[0] = c.eta; buf[1] = c.omega; buf[2] = c.W; buf[3] = c.KKT0; buf[4] = c.KKT_prev;
    buf[5] = (double)c.k; buf[6] = (double)c.t; buf[7] = (double)c.attempts; buf[8] = (double)c.restarts;
    buf[9] = c.status; buf[10] = c.eta_last;
    T *v[10];
    bool is_n[10];
    state_vecs<T>(P, c.cur, v, is_n);
    double *p = buf + kNScalars;
    for (int k = 0; k < 10; ++k) {
        const int rows = (int)(is_n[k] ? P->n : P->m);
        double *pick = is_n[k] ? P->pick_n : P->pick_m;
        HIPT(launch_shared_extract<T>(v[k], P->lgB, i, pick, rows, st));
        d2h(st, p, (const double *)pick, rows);
        ssync(P);
        p += rows;
    }
    return LP_OK;
}

template <typename T>
int do_set_state(lp_shared *P, int i, const double *buf)
{
    SDev<T> &S = P->dev<T>();
    hipStream_t st = P->stream;
    Ctl c{};
    c.eta = buf[0]; c.omega = buf[1]; c.W = buf[2]; c.KKT0 = buf[3]; c.KKT_prev = buf[4];
    c.k = (long long)buf[5]; c.t = (long long)buf[6]; c.attempts = (long long)buf[7];
    c.restarts = (long long)buf[8]; c.eta_last = buf[10];
    c.cur = 0;   // a resume reads every instance's state from buffer 0
    T *v[10];
    bool is_n[10];
    state_vecs<T>(P, 0, v, is_n);
    const double *p = buf + kNScalars;
    for (int k = 0; k < 10; ++k) {
        const int rows = (int)(is_n[k] ? P->n : P->m);
        double *pick = is_n[k] ? P->pick_n : P->pick_m;
        h2d(st, pick, p, rows);
        HIPT(launch_shared_insert<T>(pick, P->lgB, i, v[k], rows, st));
        ssync(P);
        p += rows;
    }
    P->hctl[i] = c;
    HIPT(hipMemcpyAsync(S.ctl + i, &P->hctl[i], sizeof(Ctl), hipMemcpyHostToDevice, st));
    ssync(P);
    P->state_set[i] = 1;
    return LP_OK;
}

}  // namespace

extern "C" {

int lp_shared_load(lp_shared **out, int32_t count, const lp_csr *K, const double *const *c, const double *const *q,
                   const double *const *l, const double *const *u, int64_t m1, const lp_options *opt)
{
    if (!out) return LP_ERR_ARG;
    *out = nullptr;
    if (count <= 0 || count > kMaxShared || !K || !c || !q || !l || !u) return LP_ERR_ARG;
    if (opt && (opt->ptr_kind != LP_HOST || opt->workspace || opt->presolve)) return LP_ERR_ARG;
    int rc = validate_lp(K, c[0], q[0], l[0], u[0], m1);
    if (rc != LP_OK) return rc;
    for (int b = 1; b < count; ++b) {
        rc = validate_vectors(K->n, K->m, c[b], q[b], l[b], u[b]);
        if (rc != LP_OK) return rc;
    }
    lp_options o;
    if (opt) o = *opt;
    else lp_default_options(&o);
    if ((o.precision != LP_FP64 && o.precision != LP_MIXED) || o.check_every <= 0 || o.ruiz_iters < 0 ||
        (o.fixed_step && !(o.fixed_eta > 0.0)) || o.window <= 0 || !(o.infeas_tol >= 0.0) ||
        std::isinf(o.infeas_tol))
        return LP_ERR_ARG;
    std::unique_ptr<lp_shared> P(new lp_shared());
    P->B = count;
    while (P->Bp < count) {
        P->Bp <<= 1;
        ++P->lgB;
    }
    // interleaved vectors and element indices stay below 2^30
    if ((K->n + 1) * P->Bp >= (int64_t(1) << 30) || (K->m + 1) * P->Bp >= (int64_t(1) << 30))
        return LP_ERR_TOO_LARGE;
    P->n = K->n;
    P->m = K->m;
    P->m1 = m1;
    P->opt = o;
    P->mixed = o.precision == LP_MIXED;
    P->stream = (hipStream_t)o.stream;
    P->state_set.assign(count, 0);
    P->has_start.assign(count, 0);
    P->omega_start.assign(count, 0.0);
    try {
        if (!P->stream) {
            HIPT(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
            P->own_stream = true;
        }
        HIPT(hipHostMalloc((void **)&P->hctl, sizeof(Ctl) * (size_t)P->Bp, hipHostMallocDefault));
        rc = do_load(P.get(), K, c, q, l, u);
        if (rc == LP_OK) {
            HIPT(hipMemsetAsync(P->start_x, 0, sizeof(double) * (size_t)std::max<int64_t>(P->n * P->Bp, 1), P->stream));
            HIPT(hipMemsetAsync(P->start_y, 0, sizeof(double) * (size_t)std::max<int64_t>(P->m * P->Bp, 1), P->stream));
            ssync(P.get());
        }
    } catch (const HipError &h) {
        rc = fail(P.get(), h);
    } catch (const std::bad_alloc &) {
        rc = LP_ERR_NOMEM;
    }
    if (rc != LP_OK) return rc;
    *out = P.release();
    return LP_OK;
}

int lp_shared_set_start(lp_shared *P, int32_t i, const double *x0, const double *y0, double omega)
{
    if (!P || i < 0 || i >= P->B || std::isnan(omega) || std::isinf(omega)) return LP_ERR_ARG;
    try {
        hipStream_t st = P->stream;
        const int n = (int)P->n, m = (int)P->m;
        // the instance's slice of the interleaved start (zeros where NULL)
        if (x0) h2d(st, P->pick_n, x0, n);
        else if (n) HIPT(hipMemsetAsync(P->pick_n, 0, sizeof(double) * (size_t)n, st));
        HIPT(launch_shared_insert<double>(P->pick_n, P->lgB, i, P->start_x, n, st));
        if (y0) h2d(st, P->pick_m, y0, m);
        else if (m) HIPT(hipMemsetAsync(P->pick_m, 0, sizeof(double) * (size_t)m, st));
        HIPT(launch_shared_insert<double>(P->pick_m, P->lgB, i, P->start_y, m, st));
        ssync(P);
    } catch (const HipError &h) {
        return fail(P, h);
    }
    P->has_start[i] = (x0 || y0) ? 1 : 0;
    P->omega_start[i] = omega > 0.0 ? omega : 0.0;
    std::fill(P->state_set.begin(), P->state_set.end(), 0);
    return LP_OK;
}

int lp_shared_solve(lp_shared *P, double tol, int64_t max_iters, double time_limit_s)
{
    if (!P || max_iters < 0 || std::isnan(tol)) return LP_ERR_ARG;
    try {
        return P->mixed ? do_solve<float>(P, tol, max_iters, time_limit_s)
                        : do_solve<double>(P, tol, max_iters, time_limit_s);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_shared_result(const lp_shared *Pc, int32_t i, double *x, double *y, double *lambda, lp_info *info)
{
    lp_shared *P = const_cast<lp_shared *>(Pc);
    if (!P || i < 0 || i >= P->B) return LP_ERR_ARG;
    if (!P->has_result) return LP_ERR_STATE;
    try {
        return P->mixed ? do_result<float>(P, i, x, y, lambda, info) : do_result<double>(P, i, x, y, lambda, info);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_shared_get_state(const lp_shared *Pc, int32_t i, double *buf, int64_t *len)
{
    lp_shared *P = const_cast<lp_shared *>(Pc);
    if (!P || !len || i < 0 || i >= P->B) return LP_ERR_ARG;
    *len = kNScalars + 5 * P->n + 5 * P->m;
    if (!buf) return LP_OK;
    try {
        return P->mixed ? do_get_state<float>(P, i, buf) : do_get_state<double>(P, i, buf);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_shared_set_state(lp_shared *P, int32_t i, const double *buf, int64_t len)
{
    if (!P || !buf || i < 0 || i >= P->B) return LP_ERR_ARG;
    if (len != kNScalars + 5 * P->n + 5 * P->m) return LP_ERR_STATE;
    try {
        return P->mixed ? do_set_state<float>(P, i, buf) : do_set_state<double>(P, i, buf);
    } catch (const HipError &h) {
        return fail(P, h);
    }
}

int lp_shared_device_bytes(const lp_shared *P, int64_t *bytes)
{
    if (!P || !bytes) return LP_ERR_ARG;
    *bytes = P->arena.bytes;
    return LP_OK;
}

void lp_shared_free(lp_shared *P)
{
    if (!P) return;
    (void)hipStreamSynchronize(P->stream);
    delete P;
}

const char *lp_shared_last_error(const lp_shared *P) { return P ? P->err.c_str() : ""; }

}  // extern "C"
