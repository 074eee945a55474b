// Host side of libpdlp_amd: the C ABI of include/lp.h.
//
// lp_load validates the LP of the cuPDLP-C paper's eq. (LP), reorders rows
// and columns into lane-count segments, builds the CSR of K' by a counting
// sort (so the K' product needs no atomics), copies everything to the GPU and
// runs the diagonal scaling there.  lp_solve drives the device-side
// iteration: it launches fixed windows of attempt slots (optionally replayed
// as one captured hipGraph) and polls the device done flag once per window.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "host_util.h"
#include "internal.h"
#include "presolve.h"

using namespace pdlp;

namespace {

constexpr int kNScalars = 16;

// Number of column slices for a gathered vector of `bytes`: the smallest
// power of two that brings a slice under `slice_bytes` (at most 32).
int slices_for(int64_t bytes, int64_t slice_bytes)
{
    int S = 1;
    while (S < 32 && bytes > (int64_t)S * slice_bytes) S *= 2;
    return S;
}

// Host side of a Sliced product: per-slice CSR (slice-major), the position
// of every sliced entry in the source CSR, the row blocks, and the long rows
// with the chunk slots of each.
struct HostSliced {
    int S = 1, rows = 0, cols = 0, nb = kStreamNB, rb = kStreamRB;
    std::vector<int> rp, ci, src, brow, boff;
    std::vector<unsigned short> ro;   // per slice and row: start relative to its row block's first entry
    std::vector<int4> blk;   // per row block: first row, end row, first entry, end entry
    std::vector<int> lrow, loff{0};   // long rows and their slot offsets
    int max_blocks = 0;
};

// Run fn(t) for t in [0, T) on T threads (fn(0) on the caller's); an
// exception thrown by any of them (std::bad_alloc) is rethrown here after
// all have joined.
template <typename F>
void run_threads(int T, F &&fn)
{
    std::vector<std::exception_ptr> err((size_t)T);
    auto guarded = [&](int t) {
        try {
            fn(t);
        } catch (...) {
            err[(size_t)t] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(guarded, t);
    guarded(0);
    for (auto &x : th) x.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// Rows of the source CSR must have their columns sorted, so that each
// slice's part of a row is one contiguous run.  The split and the row blocks
// run on host threads (by row chunks, then by slices); the result does not
// depend on the thread count.
void build_sliced(HostSliced &H, int rows, int cols, const std::vector<int> &rp, const std::vector<int> &ci, int S,
                  int nb = kStreamNB, int rb = kStreamRB)
{
    if (nb > kStreamNB || nb < 1) nb = kStreamNB;   // a chunk is at most one staged block
    if (rb > kStreamRB || rb < 1) rb = kStreamRB;
    H.S = S;
    H.nb = nb;
    H.rb = rb;
    H.rows = rows;
    H.cols = cols;
    const int64_t nnz = rp[rows];
    H.rp.assign((size_t)S * (rows + 1), 0);
    H.ci.resize((size_t)std::max<int64_t>(nnz, 1));
    H.src.resize((size_t)std::max<int64_t>(nnz, 1));
    H.brow.clear();
    H.blk.clear();
    H.boff.assign(S + 1, 0);
    std::vector<int> bnd((size_t)S + 1);   // slice s holds columns [bnd[s], bnd[s+1])
    for (int s = 0; s <= S; ++s) bnd[(size_t)s] = (int)((int64_t)cols * s / S);

    // entries per (row chunk, slice), then each chunk's offset in every slice
    // (slice-major, chunks in row order), then the entries themselves
    const int T = std::max(1, std::min(host_threads(), rows / 16384 + 1));
    auto chunk = [&](int t) {
        return std::make_pair((int)((int64_t)rows * t / T), (int)((int64_t)rows * (t + 1) / T));
    };
    std::vector<int64_t> cnt((size_t)T * S, 0);
    run_threads(T, [&](int t) {
        const auto [r0, r1] = chunk(t);
        int64_t *c = &cnt[(size_t)t * S];
        for (int i = r0; i < r1; ++i) {
            int sl = 0;
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                while (ci[p] >= bnd[(size_t)sl + 1]) ++sl;
                ++c[sl];
            }
        }
    });
    std::vector<int64_t> off((size_t)T * S);
    int64_t acc = 0;
    for (int sl = 0; sl < S; ++sl)
        for (int t = 0; t < T; ++t) {
            off[(size_t)t * S + sl] = acc;
            acc += cnt[(size_t)t * S + sl];
        }
    run_threads(T, [&](int t) {
        const auto [r0, r1] = chunk(t);
        std::vector<int64_t> cur(off.begin() + (size_t)t * S, off.begin() + (size_t)(t + 1) * S);
        for (int i = r0; i < r1; ++i) {
            for (int sl = 0; sl < S; ++sl) H.rp[(size_t)sl * (rows + 1) + i] = (int)cur[(size_t)sl];
            int sl = 0;
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                while (ci[p] >= bnd[(size_t)sl + 1]) ++sl;
                const int64_t at = cur[(size_t)sl]++;
                H.ci[(size_t)at] = ci[p];
                H.src[(size_t)at] = p;
            }
        }
    });
    acc = 0;
    for (int sl = 0; sl < S; ++sl) {
        for (int t = 0; t < T; ++t) acc += cnt[(size_t)t * S + sl];
        H.rp[(size_t)sl * (rows + 1) + rows] = (int)acc;
    }

    // long rows: slots slice-major, one per chunk of at most nb entries;
    // lslot[k*S + s] is the first slot of long row k in slice s
    H.lrow.clear();
    H.loff.assign(1, 0);
    for (int i = 0; i < rows; ++i)
        if (rp[i + 1] - rp[i] > kLongRow) H.lrow.push_back(i);
    std::vector<int> lslot(H.lrow.size() * (size_t)S);
    for (size_t k = 0; k < H.lrow.size(); ++k) {
        int next = H.loff.back();
        for (int sl = 0; sl < S; ++sl) {
            const int *r = &H.rp[(size_t)sl * (rows + 1)];
            lslot[k * S + sl] = next;
            next += (r[H.lrow[k] + 1] - r[H.lrow[k]] + nb - 1) / nb;
        }
        H.loff.push_back(next);
    }

    // row blocks, slice by slice
    std::vector<std::vector<int4>> bs((size_t)S);
    const int T2 = std::max(1, std::min(host_threads(), S));
    run_threads(T2, [&](int t) {
        std::vector<int> brow;
        std::vector<char> wave;
        for (int sl = t; sl < S; sl += T2) {
            const int *r = &H.rp[(size_t)sl * (rows + 1)];
            std::vector<int4> &out = bs[(size_t)sl];
            auto plain = [&](int r_begin, int r_end) {
                brow.assign(1, r_begin);
                wave.clear();
                row_blocks(r, r_begin, r_end, brow, wave, nb, rb);
                for (size_t k = 0; k + 1 < brow.size(); ++k) {
                    const int r0 = brow[k], r1 = brow[k + 1];
                    out.push_back(make_int4(r0, wave[k] ? ~r1 : r1, r[r0], r[r1]));
                }
            };
            int start = 0;
            for (size_t k = 0; k < H.lrow.size(); ++k) {
                const int lr = H.lrow[k];
                plain(start, lr);
                int slot = lslot[k * S + sl];
                for (int b = r[lr]; b < r[lr + 1]; b += nb)
                    out.push_back(make_int4(~slot++, 0, b, std::min(b + nb, r[lr + 1])));
                start = lr + 1;
            }
            plain(start, rows);
        }
    });
    // row starts relative to their block (a block holds at most kStreamNB
    // entries unless it is a single row, so the offsets fit 16 bits)
    H.ro.assign((size_t)S * (size_t)rows, 0);
    run_threads(T2, [&](int t) {
        for (int sl = t; sl < S; sl += T2) {
            const int *r = &H.rp[(size_t)sl * (rows + 1)];
            unsigned short *o = &H.ro[(size_t)sl * (size_t)rows];
            for (const int4 &q : bs[(size_t)sl]) {
                if (q.x < 0) continue;   // a chunk of a long row
                const int r1 = q.y < 0 ? ~q.y : q.y;
                for (int i = q.x; i < r1; ++i) o[i] = (unsigned short)(r[i] - q.z);
            }
        }
    });
    H.max_blocks = 0;
    for (int sl = 0; sl < S; ++sl) {
        const int c = (int)bs[(size_t)sl].size();
        H.blk.insert(H.blk.end(), bs[(size_t)sl].begin(), bs[(size_t)sl].end());
        H.boff[(size_t)sl + 1] = H.boff[(size_t)sl] + c;
        H.max_blocks = std::max(H.max_blocks, c);
    }
}

// size of one device allocation as the handle makes it
size_t dev_round(size_t bytes)
{
    if (bytes == 0) bytes = 8;
    return (bytes + 255) & ~(size_t)255;
}

struct TuneTrial {
    int S, nb, rb;
    float ms;
};

// workgroups of a partial pass: enough for every row block of the busiest
// slice, a multiple of 8 (XCDs) and of S, at most 4096
int partial_grid(int S, int max_blocks)
{
    const int unit = std::max(S, kXcds);
    int64_t g = (int64_t)S * std::max(max_blocks, 1);
    g = (g + unit - 1) / unit * unit;
    const int cap = std::max(4096 / unit, 1) * unit;
    return (int)std::min<int64_t>(g, cap);
}

}  // namespace

struct lp_problem {
    int64_t m = 0, n = 0, nnz = 0, m1 = 0;   // of the problem on the GPU (the reduced one after presolve)
    std::unique_ptr<pdlp::Presolved> pre;   // set when presolve reduced the problem
    lp_options opt{};
    hipStream_t stream = nullptr;
    Geo geo{};
    std::string err;
    double Nq = 0, Nc = 0, omega0 = 1, eta0 = 1;
    bool has_result = false, state_ready = false;
    std::vector<double> xs, ys;
    bool has_xs = false, has_ys = false;
    double omega_start = 0.0;       // > 0: primal weight of the next cold/warm start
    Ctl *hctl = nullptr;            // pinned host mirror of the device controller
    std::vector<void *> allocs;     // device allocations owned by the handle
    std::vector<int64_t> alloc_bytes;
    int64_t dev_bytes = 0;
    char *ws = nullptr;             // caller's workspace: bump-allocated, never returned before lp_free
    size_t ws_size = 0, ws_used = 0;
    bool mixed = false;
    Dev<double> d64{};
    Dev<float> d32{};
    Conf64 conf{};                  // mixed precision: the FP64 re-check of the termination test
    double *stage_n0 = nullptr, *stage_n1 = nullptr, *stage_m = nullptr, *red_part = nullptr, *red_out = nullptr;
    void *tmp_n = nullptr, *tmp_m = nullptr;   // T scratch for lp_spmv
    hipGraphExec_t graph = nullptr;
    int graph_window = 0;
    bool graph_timed = false, graph_events_failed = false;
    bool own_stream = false;
    int slices_K = 1, slices_KT = 1;
    int device = -1;                // device current at lp_load (the handle's GPU)
    void *nscratch = nullptr;       // that device's fixed scratch array (lp_spmv_noalloc); null if unavailable
    int shape_K[3] = {1, kStreamNB, kStreamRB}, shape_KT[3] = {1, kStreamNB, kStreamRB};  // S, nnz, rows per block
    int split_K = 0, split_KT = 0;   // Sliced::split of the two products
    std::vector<TuneTrial> tune_log_K, tune_log_KT;   // layouts tried by the autotuner
    std::vector<hipEvent_t> ev;
    int64_t t_count[2] = {0, 0};
    double t_ms[2] = {0, 0};
    double seconds = 0;

    template <typename T> Dev<T> &dev();

    void *dalloc(size_t bytes)
    {
        bytes = dev_round(bytes);
        if (ws) {
            if (bytes > ws_size - ws_used) throw HipError{hipErrorOutOfMemory, "workspace too small for lp_load"};
            void *p = ws + ws_used;
            ws_used += bytes;
            dev_bytes = (int64_t)ws_used;
            return p;
        }
        void *p = nullptr;
        HIPT(hipMalloc(&p, bytes));
        allocs.push_back(p);
        alloc_bytes.push_back((int64_t)bytes);
        dev_bytes += (int64_t)bytes;
        return p;
    }
    void dfree(void *p)
    {
        if (ws) return;   // workspace memory goes back to the caller at lp_free
        for (size_t i = 0; i < allocs.size(); ++i)
            if (allocs[i] == p) {
                (void)hipFree(p);
                allocs[i] = nullptr;
                dev_bytes -= alloc_bytes[i];
            }
    }
    ~lp_problem()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        for (auto e : ev) (void)hipEventDestroy(e);
        for (void *p : allocs)
            if (p) (void)hipFree(p);
        if (hctl) (void)hipHostFree(hctl);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

template <> Dev<double> &lp_problem::dev<double>() { return d64; }
template <> Dev<float> &lp_problem::dev<float>() { return d32; }

namespace {

int fail_hip(lp_problem *P, const HipError &h)
{
    char buf[512];
    snprintf(buf, sizeof(buf), "%s failed: %s", h.what, hipGetErrorString(h.e));
    if (P) P->err = buf;
    return LP_ERR_HIP;
}

template <typename T>
void upload(lp_problem *P, T *dst, const T *src, int64_t count)
{
    if (count > 0) HIPT(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)count, hipMemcpyHostToDevice, P->stream));
}

template <typename T>
void download(lp_problem *P, T *dst, const T *src, int64_t count)
{
    if (count > 0) HIPT(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost, P->stream));
}

void sync(lp_problem *P) { HIPT(hipStreamSynchronize(P->stream)); }

// ---------------------------------------------------------------------------
// load: transpose, slice, upload, scale
// ---------------------------------------------------------------------------

// Device side of a sliced product: structure uploaded from H, values gathered
// from the scaled FP64 CSR values by the recorded source positions.
template <typename T>
Sliced<T> upload_sliced(lp_problem *P, const HostSliced &H, const double *scaled_csr_vals, int split)
{
    const int64_t nnz = H.rp[(size_t)H.S * (H.rows + 1) - 1];
    Sliced<T> q{};
    q.S = H.S;
    q.split = split;
    q.rows = H.rows;
    q.grid = partial_grid(H.S, H.max_blocks);
    int *rp = (int *)P->dalloc(sizeof(int) * H.rp.size());
    unsigned short *ro = (unsigned short *)P->dalloc(sizeof(unsigned short) * std::max<size_t>(H.ro.size(), 1));
    int *ci = (int *)P->dalloc(sizeof(int) * (size_t)std::max<int64_t>(nnz, 1));
    int4 *blk = (int4 *)P->dalloc(sizeof(int4) * std::max<size_t>(H.blk.size(), 1));
    int *boff = (int *)P->dalloc(sizeof(int) * H.boff.size());
    T *v = (T *)P->dalloc(sizeof(T) * (size_t)std::max<int64_t>(nnz, 1));
    T *part = (T *)P->dalloc(sizeof(T) * (size_t)H.S * (size_t)std::max(H.rows, 1));
    const int nlong = (int)H.lrow.size();
    int *lrow = (int *)P->dalloc(sizeof(int) * (size_t)std::max(nlong, 1));
    int *loff = (int *)P->dalloc(sizeof(int) * H.loff.size());
    T *lpart = (T *)P->dalloc(sizeof(T) * (size_t)std::max(H.loff.back(), 1));
    int *src = (int *)P->dalloc(sizeof(int) * (size_t)std::max<int64_t>(nnz, 1));
    upload(P, lrow, H.lrow.data(), nlong);
    upload(P, loff, H.loff.data(), (int64_t)H.loff.size());
    upload(P, rp, H.rp.data(), (int64_t)H.rp.size());
    upload(P, ro, H.ro.data(), (int64_t)H.ro.size());
    upload(P, ci, H.ci.data(), nnz);
    upload(P, blk, H.blk.data(), (int64_t)H.blk.size());
    upload(P, boff, H.boff.data(), (int64_t)H.boff.size());
    upload(P, src, H.src.data(), nnz);
    HIPT(launch_gather_values<T>(scaled_csr_vals, src, v, nnz, P->stream));
    sync(P);
    P->dfree(src);
    q.rp = rp; q.ro = ro; q.ci = ci; q.blk = blk; q.boff = boff; q.v = v; q.part = part;
    q.nlong = nlong; q.lrow = lrow; q.loff = loff; q.lpart = lpart;
    q.nlpart = H.loff.back();
    return q;
}

template <typename T>
void free_sliced(lp_problem *P, Sliced<T> &q)
{
    for (const void *p : {(const void *)q.rp, (const void *)q.ro, (const void *)q.ci, (const void *)q.blk, (const void *)q.boff,
                          (const void *)q.v, (const void *)q.part, (const void *)q.lrow, (const void *)q.loff,
                          (const void *)q.lpart})
        P->dfree(const_cast<void *>(p));
    q = Sliced<T>{};
}

// Mean time of one product (partial pass + slice sums) on a vector of ones.
template <typename T>
float time_product(lp_problem *P, const Sliced<T> &q, T *in, T *out, int64_t in_len)
{
    std::vector<T> ones((size_t)std::max<int64_t>(in_len, 1), T(1));
    upload(P, in, ones.data(), in_len);
    EventPair ev;
    for (int r = 0; r < 2; ++r) HIPT(launch_spmv<T>(q, in, out, P->stream));
    HIPT(hipEventRecord(ev.a, P->stream));
    const int reps = 5;
    for (int r = 0; r < reps; ++r) HIPT(launch_spmv<T>(q, in, out, P->stream));
    HIPT(hipEventRecord(ev.b, P->stream));
    HIPT(hipEventSynchronize(ev.b));
    return ev.ms() / reps;
}

// Row blocks from which a product's short-row sums are split by entries by
// default: below that the partial pass is a few workgroups whose time is
// latency, which the split's two extra barriers lengthen (the 5,000-entry LP:
// 51k against 44k iterations per second in launched slots), while above it
// the split evens out the threads' work (the 2e7-entry power-law LP: K' pass
// 128 against 124 us).
constexpr size_t kSplitMinBlocks = 1024;

// A trial layout replaces the incumbent only when it is this much faster, so
// that near-ties (timing noise) keep the earlier, default-side layout and
// two processes rarely pick different layouts.
constexpr float kTuneMargin = 0.97f;

// Autotuner for one product: times the default layout, then walks the slice
// count down by halving while that keeps helping (else up by doubling, to at
// most 32), then tries halved nonzeros per row block and 256 rows per block at
// the best slice count, on the actual matrix, and keeps the fastest.  The walk
// matters on very sparse matrices with many rows: each slice adds a row
// pointer and a partial per row, which can outweigh the L2 locality it buys.
// Last, when split_sums is -1, it times the other form of the row sums on the
// chosen layout (same device arrays) and keeps the faster.
template <typename T>
Sliced<T> tuned_sliced(lp_problem *P, const HostSliced &H0, const std::vector<int> &rp, const std::vector<int> &ci,
                       const double *vals, T *in, T *out, int64_t in_len, std::vector<TuneTrial> &log, int *shape,
                       int split)
{
    Sliced<T> best = upload_sliced<T>(P, H0, vals, split);
    float best_ms = time_product<T>(P, best, in, out, in_len);
    log.push_back({H0.S, H0.nb, H0.rb, best_ms});
    shape[0] = H0.S; shape[1] = H0.nb; shape[2] = H0.rb;
    // time one layout; keep it if it is the fastest so far
    auto trial = [&](int S, int nb, int rb) {
        HostSliced H;
        build_sliced(H, H0.rows, H0.cols, rp, ci, S, nb, rb);
        Sliced<T> q = upload_sliced<T>(P, H, vals, split);
        const float ms = time_product<T>(P, q, in, out, in_len);
        log.push_back({S, nb, rb, ms});
        if (ms < kTuneMargin * best_ms) {
            free_sliced<T>(P, best);
            best = q;
            best_ms = ms;
            shape[0] = S; shape[1] = nb; shape[2] = rb;
            return true;
        }
        free_sliced<T>(P, q);
        return false;
    };
    bool down = false;
    for (int S = H0.S / 2; S >= 1 && trial(S, H0.nb, H0.rb); S /= 2) down = true;
    if (!down)
        for (int S = H0.S * 2; S <= 32 && trial(S, H0.nb, H0.rb); S *= 2) {}
    const int S = shape[0];
    if (H0.nb / 2 >= 1) trial(S, H0.nb / 2, H0.rb);
    if (H0.rb != 256) trial(S, shape[1], 256);
    if (P->opt.split_sums == -1) {
        Sliced<T> q = best;
        q.split = !best.split;
        const float ms = time_product<T>(P, q, in, out, in_len);
        if (P->opt.verbose)
            std::fprintf(stderr, "[lp] layout %s row sums %s: %.3f ms against %.3f\n", &log == &P->tune_log_K ? "K" : "K'",
                         q.split ? "split by entries" : "by rows", ms, best_ms);
        if (ms < kTuneMargin * best_ms) {
            best.split = q.split;
            best_ms = ms;
        }
    }
    if (P->opt.verbose)
        for (const auto &t : log)
            std::fprintf(stderr, "[lp] layout %s S=%d nnz/block=%d rows/block=%d: %.3f ms\n",
                         &log == &P->tune_log_K ? "K" : "K'", t.S, t.nb, t.rb, t.ms);
    return best;
}

template <typename T>
void setup_typed(lp_problem *P, const HostSliced &HK, const HostSliced &HT, const double *kv64, const double *tv64,
                 const double *cs64, const double *ls64, const double *us64, const double *qs64, const double *Dr,
                 const double *Dc, const std::vector<int> &rp, const std::vector<int> &ci, const std::vector<int> &tp,
                 const std::vector<int> &ti)
{
    const int64_t m = P->m, n = P->n;
    Dev<T> &d = P->dev<T>();
    d.m = (int)m;
    d.n = (int)n;
    d.m1 = (int)P->m1;
    d.Dr = Dr; d.Dc = Dc;
    auto tvec = [&](int64_t len) { return (T *)P->dalloc(sizeof(T) * (size_t)std::max<int64_t>(len, 1)); };
    P->tmp_n = tvec(n);
    P->tmp_m = tvec(m);
    // row sums split by entries where a product has enough row blocks to
    // fill the GPU (split_sums -1), or as asked (0 or 1)
    auto split_of = [&](const HostSliced &H) {
        return P->opt.split_sums == -1 ? (int)(H.blk.size() >= (size_t)kSplitMinBlocks) : P->opt.split_sums;
    };
    const int split_K = split_of(HK), split_KT = split_of(HT);
    if (P->opt.autotune && !P->ws) {
        d.K = tuned_sliced<T>(P, HK, rp, ci, kv64, (T *)P->tmp_n, (T *)P->tmp_m, n, P->tune_log_K, P->shape_K, split_K);
        d.KT = tuned_sliced<T>(P, HT, tp, ti, tv64, (T *)P->tmp_m, (T *)P->tmp_n, m, P->tune_log_KT, P->shape_KT,
                               split_KT);
    } else {
        d.K = upload_sliced<T>(P, HK, kv64, split_K);
        d.KT = upload_sliced<T>(P, HT, tv64, split_KT);
        P->shape_K[0] = HK.S; P->shape_K[1] = HK.nb; P->shape_K[2] = HK.rb;
        P->shape_KT[0] = HT.S; P->shape_KT[1] = HT.nb; P->shape_KT[2] = HT.rb;
    }
    P->slices_K = d.K.S;
    P->slices_KT = d.KT.S;
    P->split_K = d.K.split;
    P->split_KT = d.KT.split;
    if (std::is_same<T, double>::value) {
        d.cs = (const T *)cs64; d.ls = (const T *)ls64; d.us = (const T *)us64; d.qs = (const T *)qs64;
    } else {
        T *cs = tvec(n), *ls = tvec(n), *us = tvec(n), *qs = tvec(m);
        HIPT(launch_from_double<T>(cs64, cs, n, P->stream));
        HIPT(launch_from_double<T>(ls64, ls, n, P->stream));
        HIPT(launch_from_double<T>(us64, us, n, P->stream));
        HIPT(launch_from_double<T>(qs64, qs, m, P->stream));
        d.cs = cs; d.ls = ls; d.us = us; d.qs = qs;
    }
    for (int b = 0; b < 2; ++b) {
        d.xb[b] = tvec(n); d.yb[b] = tvec(m); d.Kxb[b] = tvec(m); d.KTyb[b] = tvec(n);
    }
    d.xa = tvec(n); d.ya = tvec(m); d.Kxa = tvec(m); d.KTya = tvec(n);
    d.x0 = tvec(n); d.y0 = tvec(m); d.Kx0 = tvec(m); d.KTy0 = tvec(n);
    d.xo = tvec(n); d.yo = tvec(m); d.KTyo = tvec(n);
    d.part_primal = (double *)P->dalloc(sizeof(double) * kMaxGrid);
    d.part_dual = (double *)P->dalloc(sizeof(double) * kMaxGrid * 2);
    d.part_check = (double *)P->dalloc(sizeof(double) * kMaxGrid * kCheckSums);
    d.part_ray = (double *)P->dalloc(sizeof(double) * kMaxGrid * kRaySums);
    d.ctl = (Ctl *)P->dalloc(sizeof(Ctl));
}

// Host copies of lp_load's arrays when the caller passed device pointers.
struct HostLP {
    std::vector<int32_t> rp, ci;
    std::vector<double> v, c, q, l, u;
    lp_csr K{};
};

template <typename T>
void fetch(std::vector<T> &dst, const T *src, int64_t count, hipStream_t st)
{
    dst.resize((size_t)std::max<int64_t>(count, 0));
    if (count > 0 && src) HIPT(hipMemcpyAsync(dst.data(), src, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost, st));
}

// Copies the device arrays (pattern only when c is NULL) and points H.K at
// them; sizes are checked first so no copy reads past the caller's arrays.
int fetch_lp(const lp_csr *K, const double *c, const double *q, const double *l, const double *u, hipStream_t st,
             HostLP &H)
{
    int rc = validate_dims(K);
    if (rc != LP_OK) return rc;
    fetch(H.rp, K->row_ptr, K->m + 1, st);
    fetch(H.ci, K->col, K->nnz, st);
    if (c) {
        if ((K->nnz > 0 && !K->val) || (K->n > 0 && (!l || !u)) || (K->m > 0 && !q)) return LP_ERR_ARG;
        fetch(H.v, K->val, K->nnz, st);
        fetch(H.c, c, K->n, st);
        fetch(H.l, l, K->n, st);
        fetch(H.u, u, K->n, st);
        fetch(H.q, q, K->m, st);
    }
    HIPT(hipStreamSynchronize(st));
    H.K = *K;
    H.K.row_ptr = H.rp.data();
    H.K.col = H.ci.data();
    H.K.val = c ? H.v.data() : nullptr;
    return LP_OK;
}

int check_options(const lp_options &o)
{
    if ((o.precision != LP_FP64 && o.precision != LP_MIXED) || o.check_every <= 0 || o.ruiz_iters < 0 ||
        (o.fixed_step && !(o.fixed_eta > 0.0)) || o.window <= 0 || o.slice_kib <= 0 ||
        (o.ptr_kind != LP_HOST && o.ptr_kind != LP_DEVICE) || !(o.infeas_tol >= 0.0) || std::isinf(o.infeas_tol) ||
        o.kernel_timing < 0 || o.kernel_timing > 2 ||
        (o.workspace && (reinterpret_cast<uintptr_t>(o.workspace) % 256 != 0)) ||
        (o.presolve != 0 && o.presolve != 1) || (o.presolve && (o.ptr_kind == LP_DEVICE || o.workspace)) ||
        o.persistent < -1 || o.persistent > 1 || o.split_sums < -1 || o.split_sums > 1)
        return LP_ERR_ARG;
    return LP_OK;
}

// The host layout lp_load builds for K (sorted rows, transpose, slices).
void host_layout(const lp_csr *K, bool mixed, int slice_kib, std::vector<int> &rp, std::vector<int> &ci,
                 std::vector<double> &kv, std::vector<int> &tp, std::vector<int> &ti, std::vector<double> &tv,
                 HostSliced &HK, HostSliced &HT)
{
    const int64_t m = K->m, n = K->n;
    append_sorted_rows(K, 0, rp, ci, kv);
    transpose_csr((int)m, (int)n, rp, ci, kv, tp, ti, tv);
    // column slices sized so a slice of the gathered vector stays in one XCD's L2
    const int64_t tsz = mixed ? 4 : 8;
    const int64_t slice_bytes = (int64_t)slice_kib * 1024;
    build_sliced(HK, (int)m, (int)n, rp, ci, slices_for(n * tsz, slice_bytes));
    build_sliced(HT, (int)n, (int)m, tp, ti, slices_for(m * tsz, slice_bytes));
}

// Every device allocation do_load and setup_typed make, in bytes as dalloc
// rounds them, for the default layout: the size of a caller's workspace.
// Kept next to the code it mirrors; a GPU test checks the two agree.
size_t load_plan_bytes(int64_t m, int64_t n, int64_t nnz, const HostSliced &HK, const HostSliced &HT, bool mixed)
{
    const size_t T = mixed ? sizeof(float) : sizeof(double);
    auto one = [](int64_t v) { return (size_t)std::max<int64_t>(v, 1); };
    size_t b = 0;
    auto add = [&](size_t bytes) { b += dev_round(bytes); };
    // do_load: CSR pair and vectors for the scaling, norms, staging
    add(4 * one(m + 1)); add(4 * one(nnz)); add(4 * one(n + 1)); add(4 * one(nnz));
    add(8 * one(nnz)); add(8 * one(nnz));
    for (int64_t len : {n, n, n, m, m, n, m, n, n, n, n, m}) add(8 * one(len));   // c l u q Dr Dc r s cs ls us qs
    add(8 * kMaxGrid); add(8 * 8);
    add(8 * one(n)); add(8 * one(n)); add(8 * one(m));
    add(4 * one((int64_t)HK.lrow.size())); add(4 * one((int64_t)HT.lrow.size()));   // long rows for the scaling
    // setup_typed: lp_spmv scratch, the two sliced products, vectors, partials, controller
    add(T * one(n)); add(T * one(m));
    for (const HostSliced *H : {&HK, &HT}) {
        add(sizeof(int) * H->rp.size());
        add(sizeof(unsigned short) * std::max<size_t>(H->ro.size(), 1));
        add(4 * one(nnz));
        add(sizeof(int4) * std::max<size_t>(H->blk.size(), 1));
        add(sizeof(int) * H->boff.size());
        add(T * one(nnz));
        add(T * (size_t)H->S * (size_t)std::max(H->rows, 1));
        add(4 * one((int64_t)H->lrow.size())); add(4 * H->loff.size()); add(T * one(H->loff.back()));
        add(4 * one(nnz));
    }
    if (mixed) for (int64_t len : {n, n, n, m}) add(T * one(len));
    for (int k = 0; k < 2; ++k) for (int64_t len : {n, m, m, n}) add(T * one(len));
    for (int64_t len : {n, m, m, n, n, m, m, n, n, m, n}) add(T * one(len));   // averages, anchor (+ products), output
    add(8 * kMaxGrid); add(8 * kMaxGrid * 2); add(8 * kMaxGrid * kCheckSums); add(8 * kMaxGrid * kRaySums);
    add(sizeof(Ctl));
    // mixed precision: the FP64 re-check keeps the CSR pair above and adds its products and partials
    if (mixed) {
        for (int64_t len : {m, m, n, n}) add(8 * one(len));
        add(8 * kMaxGrid * kCheckSums);
    }
    return b;
}

int do_load(lp_problem *P, const lp_csr *K, const double *c, const double *q, const double *l, const double *u)
{
    const int64_t m = P->m, n = P->n, nnz = P->nnz;
    // K with the columns of each row sorted, K' by a counting sort, both sliced
    std::vector<int> rp, ci, tp, ti;
    std::vector<double> kv, tv;
    HostSliced HK, HT;
    host_layout(K, P->mixed, P->opt.slice_kib, rp, ci, kv, tp, ti, tv, HK, HT);
    P->slices_K = HK.S;
    P->slices_KT = HT.S;
    if (P->ws && P->ws_size < load_plan_bytes(m, n, nnz, HK, HT, P->mixed)) {
        char buf[160];
        snprintf(buf, sizeof(buf), "workspace of %zu bytes, lp_load needs %zu", P->ws_size,
                 load_plan_bytes(m, n, nnz, HK, HT, P->mixed));
        P->err = buf;
        return LP_ERR_NOMEM;
    }

    // device copies of the CSR pair (for the scaling) and the vectors
    auto ialloc = [&](int64_t len) { return (int *)P->dalloc(sizeof(int) * (size_t)std::max<int64_t>(len, 1)); };
    auto dalloc = [&](int64_t len) { return (double *)P->dalloc(sizeof(double) * (size_t)std::max<int64_t>(len, 1)); };
    int *d_rp = ialloc(m + 1), *d_ci = ialloc(nnz), *d_tp = ialloc(n + 1), *d_ti = ialloc(nnz);
    double *d_kv = dalloc(nnz), *d_tv = dalloc(nnz);
    double *d_c = dalloc(n), *d_l = dalloc(n), *d_u = dalloc(n), *d_q = dalloc(m);
    double *Dr = dalloc(m), *Dc = dalloc(n), *r = dalloc(m), *s = dalloc(n);
    double *cs = dalloc(n), *ls = dalloc(n), *us = dalloc(n), *qs = dalloc(m);
    P->red_part = dalloc(kMaxGrid);
    P->red_out = dalloc(8);
    P->stage_n0 = dalloc(n); P->stage_n1 = dalloc(n); P->stage_m = dalloc(m);
    upload(P, d_rp, rp.data(), m + 1);
    upload(P, d_ci, ci.data(), nnz);
    upload(P, d_kv, kv.data(), nnz);
    upload(P, d_tp, tp.data(), n + 1);
    upload(P, d_ti, ti.data(), nnz);
    upload(P, d_tv, tv.data(), nnz);
    upload(P, d_c, c, n);
    upload(P, d_l, l, n);
    upload(P, d_u, u, n);
    upload(P, d_q, q, m);

    // scaling: Ruiz inf-norm rounds, then one Pock-Chambolle round; row and
    // column factors both come from the same current matrix
    const int M = (int)m, N = (int)n;
    hipStream_t st = P->stream;
    // the rows longer than kLongRow (the same ones the products cut into chunks)
    int *d_klong = ialloc((int64_t)HK.lrow.size()), *d_tlong = ialloc((int64_t)HT.lrow.size());
    upload(P, d_klong, HK.lrow.data(), (int64_t)HK.lrow.size());
    upload(P, d_tlong, HT.lrow.data(), (int64_t)HT.lrow.size());
    HIPT(scale_csr_pair(d_rp, d_ci, d_kv, M, d_tp, d_ti, d_tv, N, Dr, Dc, r, s, P->opt.ruiz_iters, P->opt.pc_alpha, st,
                        d_klong, (int)HK.lrow.size(), d_tlong, (int)HT.lrow.size()));
    HIPT(launch_scale_vectors(d_c, d_l, d_u, d_q, Dc, Dr, cs, ls, us, qs, N, M, st));
    double h[5] = {0, 0, 0, 0, 0};
    HIPT(launch_sumsq(d_q, m, P->red_part, P->red_out + 0, st));
    HIPT(launch_sumsq(d_c, n, P->red_part, P->red_out + 1, st));
    HIPT(launch_sumsq(qs, m, P->red_part, P->red_out + 2, st));
    HIPT(launch_sumsq(cs, n, P->red_part, P->red_out + 3, st));
    HIPT(launch_absmax(d_kv, nnz, P->red_part, P->red_out + 4, st));
    download(P, h, P->red_out, 5);
    sync(P);
    P->Nq = std::sqrt(h[0]);
    P->Nc = std::sqrt(h[1]);
    const double nq = std::sqrt(h[2]), nc = std::sqrt(h[3]);
    P->omega0 = (nc > 1e-10 && nq > 1e-10) ? nc / nq : 1.0;
    P->eta0 = h[4] > 0.0 ? 1.0 / h[4] : 1.0;
    if (P->opt.fixed_step) P->eta0 = P->opt.fixed_eta;

    if (P->mixed) setup_typed<float>(P, HK, HT, d_kv, d_tv, cs, ls, us, qs, Dr, Dc, rp, ci, tp, ti);
    else setup_typed<double>(P, HK, HT, d_kv, d_tv, cs, ls, us, qs, Dr, Dc, rp, ci, tp, ti);
    if (P->mixed) {
        // the FP64 scaled CSR pair stays for the re-check of the termination test
        Conf64 &cf = P->conf;
        cf.rp = d_rp; cf.ci = d_ci; cf.kv = d_kv; cf.tp = d_tp; cf.ti = d_ti; cf.tv = d_tv;
        cf.cs = cs; cf.ls = ls; cf.us = us; cf.qs = qs;
        cf.kx[0] = dalloc(m); cf.kx[1] = dalloc(m);
        cf.kty[0] = dalloc(n); cf.kty[1] = dalloc(n);
        cf.part = dalloc((int64_t)kMaxGrid * kCheckSums);
    }
    sync(P);
    // otherwise the CSR pair was only needed for the scaling
    if (!P->mixed)
        for (void *pp : {(void *)d_rp, (void *)d_ci, (void *)d_kv, (void *)d_tp, (void *)d_ti, (void *)d_tv})
            P->dfree(pp);
    for (void *pp : {(void *)r, (void *)s, (void *)d_c, (void *)d_l, (void *)d_u, (void *)d_q, (void *)d_klong,
                     (void *)d_tlong})
        P->dfree(pp);

    // one grid size for the elementwise solver kernels (its workgroups are the partial-sum slots)
    Geo &g = P->geo;
    g.vb_n = (int)((n + kBlock - 1) / kBlock);
    g.vb_m = (int)((m + kBlock - 1) / kBlock);
    g.grid = std::max(1, std::min(kMaxGrid, g.vb_n + g.vb_m));
    return LP_OK;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------

template <typename T>
void launch_slot(lp_problem *P, int slot, bool timed)
{
    Dev<T> &d = P->dev<T>();
    hipStream_t st = P->stream;
    if (timed) HIPT(hipEventRecord(P->ev[4 * slot + 0], st));
    HIPT(launch_partial_K<T>(d, st));
    HIPT(launch_dual<T>(d, P->geo, st));
    if (timed) HIPT(hipEventRecord(P->ev[4 * slot + 1], st));
    HIPT(launch_step_decide<T>(d, P->geo, st));
    if (timed) HIPT(hipEventRecord(P->ev[4 * slot + 2], st));
    HIPT(launch_partial_KT<T>(d, st));
    HIPT(launch_update<T>(d, P->geo, st));
    if (timed) HIPT(hipEventRecord(P->ev[4 * slot + 3], st));
    // the check sums of a check step come from the update kernel itself
    HIPT(launch_check_decide<T>(d, P->geo, P->Nq, P->Nc, st));
    HIPT(launch_check_apply<T>(d, P->geo, st));
}

template <typename T>
void run_check(lp_problem *P)
{
    Dev<T> &d = P->dev<T>();
    HIPT(launch_check_reduce<T>(d, P->geo, P->stream));
    HIPT(launch_check_decide<T>(d, P->geo, P->Nq, P->Nc, P->stream));
    HIPT(launch_check_apply<T>(d, P->geo, P->stream));
}

// One line per window (verbose): counters, step size, primal weight, and the
// quantities of the latest check (current iterate, then average).
void trace_window(const Ctl &c)
{
    fprintf(stderr,
            "[lp] k=%lld attempts=%lld restarts=%lld eta=%.6g omega=%.6g | last check: rel_p %.3e/%.3e "
            "rel_d %.3e/%.3e rel_gap %.3e/%.3e KKT_omega %.4e/%.4e KKT0 %.4e%s\n",
            c.k, c.attempts, c.restarts, c.eta, c.omega, c.rel_p[0], c.rel_p[1], c.rel_d[0], c.rel_d[1], c.rel_g[0],
            c.rel_g[1], c.kkt[0], c.kkt[1], c.KKT0, c.done ? " (done)" : "");
}

void put_ctl(lp_problem *P, const Ctl &c, Ctl *dctl)
{
    *P->hctl = c;
    HIPT(hipMemcpyAsync(dctl, P->hctl, sizeof(Ctl), hipMemcpyHostToDevice, P->stream));
    sync(P);
}

void get_ctl(lp_problem *P, Ctl *dctl)
{
    HIPT(hipMemcpyAsync(P->hctl, dctl, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream));
    sync(P);
}

// Mixed precision: the last check passed the termination test on FP32
// products and stopped the loop.  Redo its sums with FP64 products of the
// FP64 scaled matrix: confirmed, the solve ends and the point is copied out;
// otherwise the check decision runs again without its termination test
// (restart logic, next primal trial) and the loop goes on.
template <typename T>
void resolve_confirm(lp_problem *P)
{
    if (!P->hctl->confirm) return;
    Dev<T> &d = P->dev<T>();
    HIPT(launch_confirm<T>(d, P->geo, P->conf, P->hctl->cur, P->Nq, P->Nc, P->stream));
    // not confirmed: the check sums again (the one-workgroup loop keeps its own
    // in registers), then the decision without its termination test; both
    // return at once when confirmed
    HIPT(launch_check_reduce<T>(d, P->geo, P->stream));
    HIPT(launch_check_decide<T>(d, P->geo, P->Nq, P->Nc, P->stream));
    HIPT(launch_check_apply<T>(d, P->geo, P->stream));
    get_ctl(P, d.ctl);
}

template <typename T>
void copy_dev(lp_problem *P, T *dst, const T *src, int64_t len)
{
    if (len > 0) HIPT(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)len, hipMemcpyDeviceToDevice, P->stream));
}

// The one-workgroup loop applies when both products are a single column
// slice without long rows (their slice is then a plain CSR) and the option
// asks for it: persistent = 1 always then; the default (-1) only when K, K'
// and the gathered vectors fit in LDS, the case where it beats the
// launches (without the LDS copies each thread walks its elements with a
// round trip to L2 apiece, slower than the launches from a few thousand
// columns on).
template <typename T>
bool small_loop_eligible(lp_problem *P)
{
    const Dev<T> &d = P->dev<T>();
    if (P->opt.persistent == 0 || d.K.S != 1 || d.KT.S != 1 || d.K.nlong != 0 || d.KT.nlong != 0) return false;
    return P->opt.persistent == 1 ||
           small_stage_bytes<T>((int)P->m, (int)P->n, (int)P->nnz, (int)P->nnz) <= kSmallStageMax;
}

template <typename T>
int do_solve(lp_problem *P, double tol, int64_t max_iters, double time_limit)
{
    Dev<T> &d = P->dev<T>();
    const int64_t m = P->m, n = P->n;
    hipStream_t st = P->stream;
    auto t0 = std::chrono::steady_clock::now();
    P->t_count[0] = P->t_count[1] = 0;
    P->t_ms[0] = P->t_ms[1] = 0;
    if (!P->state_ready) {
        // start point, products, averages/anchor = start, KKT0, first primal trial
        const double *xs = nullptr, *ys = nullptr;
        if (P->has_xs) {
            upload(P, P->stage_n0, P->xs.data(), n);
            sync(P);
            xs = P->stage_n0;
        }
        if (P->has_ys) {
            upload(P, P->stage_m, P->ys.data(), m);
            sync(P);
            ys = P->stage_m;
        }
        HIPT(launch_start<T>(d, xs, ys, 0, st));
        Ctl c{};
        c.eta = P->eta0;
        c.omega = P->omega_start > 0.0 ? P->omega_start : P->omega0;
        c.KKT_prev = INFINITY;
        c.mode = MODE_INIT;
        c.tol = tol;
        c.infeas_tol = P->opt.infeas_tol;
        c.kkt_p = P->opt.kkt_omega_power;
        c.fixed_eta = P->opt.fixed_eta;
        c.max_iters = max_iters;
        c.check_every = P->opt.check_every;
        c.fixed_step = P->opt.fixed_step;
        c.final_status = LP_ITERATION_LIMIT;
        c.confirm_on = P->mixed ? 1 : 0;
        put_ctl(P, c, d.ctl);
        HIPT(launch_spmv<T>(d.K, d.xb[0], d.Kxb[0], st));
        HIPT(launch_spmv<T>(d.KT, d.yb[0], d.KTyb[0], st));
        copy_dev(P, d.xa, d.xb[0], n);
        copy_dev(P, d.x0, d.xb[0], n);
        copy_dev(P, d.KTya, d.KTyb[0], n);
        copy_dev(P, d.ya, d.yb[0], m);
        copy_dev(P, d.y0, d.yb[0], m);
        copy_dev(P, d.Kxa, d.Kxb[0], m);
        copy_dev(P, d.Kx0, d.Kxb[0], m);
        copy_dev(P, d.KTy0, d.KTyb[0], n);
        run_check<T>(P);
    } else {
        Ctl c = *P->hctl;   // set by lp_set_state
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
        put_ctl(P, c, d.ctl);
        // the anchor's products (the state holds the anchor, not its products)
        HIPT(launch_spmv<T>(d.K, d.x0, d.Kx0, st));
        HIPT(launch_spmv<T>(d.KT, d.y0, d.KTy0, st));
        HIPT(launch_check_apply<T>(d, P->geo, st));
    }
    P->state_ready = false;
    get_ctl(P, d.ctl);
    if (!P->hctl->done && P->hctl->k >= max_iters) {
        Ctl c = *P->hctl;
        c.mode = MODE_FINAL;
        c.final_status = LP_ITERATION_LIMIT;
        put_ctl(P, c, d.ctl);
        run_check<T>(P);
        get_ctl(P, d.ctl);
        resolve_confirm<T>(P);
    }
    const int W = std::max(1, P->opt.window);
    if (small_loop_eligible<T>(P)) {
        // the whole loop in one workgroup: 64 W attempt slots per launch
        for (; !P->hctl->done;) {
            const long long k_before = P->hctl->k, a_before = P->hctl->attempts;
            HIPT(launch_small_loop<T>(d, (int)P->nnz, (int)P->nnz, 64 * W, P->Nq, P->Nc, st));
            get_ctl(P, d.ctl);
            resolve_confirm<T>(P);
            if (P->opt.verbose) trace_window(*P->hctl);
            if (P->hctl->done) break;
            if (P->hctl->k == k_before && P->hctl->attempts == a_before) {
                P->err = "no step decision in a whole window (controller stalled)";
                return LP_ERR_HIP;
            }
            if (time_limit > 0.0 &&
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > time_limit) {
                Ctl c = *P->hctl;
                c.mode = MODE_FINAL;
                c.final_status = LP_TIME_LIMIT;
                put_ctl(P, c, d.ctl);
                run_check<T>(P);
                get_ctl(P, d.ctl);
                resolve_confirm<T>(P);
                break;
            }
        }
        sync(P);
        P->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        P->has_result = true;
        return LP_OK;
    }
    // kernel_timing: 0 none; 1 events around the products of every window;
    // 2 only in the first window (plain launches), the rest replaying the
    // untimed graph
    const int tmode = P->opt.kernel_timing;
    const bool timed = tmode != 0;
    const bool timed_graph = tmode == 1;
    if (timed && (int)P->ev.size() < 4 * W) {
        for (auto e : P->ev) (void)hipEventDestroy(e);
        P->ev.assign(4 * W, nullptr);
        for (auto &e : P->ev) HIPT(hipEventCreate(&e));
    }
    // the window is captured once per handle (with the timing events as
    // event-record nodes when kernel_timing = 1); if the runtime refuses to
    // capture event records, or they carry no timestamps, those runs fall
    // back to plain launches
    bool use_graph = P->opt.use_graph && !(timed_graph && P->graph_events_failed);
    if (use_graph && (!P->graph || P->graph_window != W || P->graph_timed != timed_graph)) {
        if (P->graph) {
            (void)hipGraphExecDestroy(P->graph);
            P->graph = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPT(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        bool ok = true;
        try {
            for (int s = 0; s < W; ++s) launch_slot<T>(P, s, timed_graph);
        } catch (const HipError &) {
            ok = false;
        }
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (ok && ec == hipSuccess && hipGraphInstantiate(&P->graph, g, nullptr, nullptr, 0) == hipSuccess) {
            P->graph_window = W;
            P->graph_timed = timed_graph;
        } else {
            (void)hipGetLastError();
            P->graph = nullptr;
            if (!timed_graph) HIPT(ec != hipSuccess ? ec : hipErrorUnknown);
            P->graph_events_failed = true;
            use_graph = false;
        }
        if (g) (void)hipGraphDestroy(g);
    }
    for (int widx = 0; !P->hctl->done; ++widx) {
        const long long k_before = P->hctl->k, a_before = P->hctl->attempts;
        const bool sampled = tmode == 2 && widx == 0;
        const bool timed_now = tmode == 1 || sampled;
        if (use_graph && !sampled) {
            HIPT(hipGraphLaunch(P->graph, st));
        } else {
            for (int s = 0; s < W; ++s) launch_slot<T>(P, s, timed_now);
        }
        get_ctl(P, d.ctl);
        resolve_confirm<T>(P);
        if (P->opt.verbose) trace_window(*P->hctl);
        if (timed_now && !P->hctl->done) {
            // every slot of a window that ended unfinished did real work
            double ta = 0.0, tb = 0.0;
            bool read = true;
            for (int s = 0; s < W && read; ++s) {
                float a = 0, b = 0;
                const hipError_t ea = hipEventElapsedTime(&a, P->ev[4 * s + 0], P->ev[4 * s + 1]);
                const hipError_t eb = hipEventElapsedTime(&b, P->ev[4 * s + 2], P->ev[4 * s + 3]);
                if (ea != hipSuccess || eb != hipSuccess) {
                    // events recorded by graph nodes carry no timestamps on
                    // this runtime: time the next windows with plain launches
                    (void)hipGetLastError();
                    if (!use_graph || sampled) HIPT(ea != hipSuccess ? ea : eb);
                    read = false;
                    break;
                }
                ta += a;
                tb += b;
            }
            if (read) {
                P->t_ms[0] += ta;
                P->t_ms[1] += tb;
                P->t_count[0] += W;
                P->t_count[1] += W;
            } else {
                P->graph_events_failed = true;
                (void)hipGraphExecDestroy(P->graph);
                P->graph = nullptr;
                use_graph = false;
            }
        }
        if (P->hctl->done) break;
        if (P->hctl->k == k_before && P->hctl->attempts == a_before) {
            // every slot takes a step decision, so a window always moves the counters
            P->err = "no step decision in a whole window (controller stalled)";
            return LP_ERR_HIP;
        }
        if (time_limit > 0.0) {
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el > time_limit) {
                Ctl c = *P->hctl;
                c.mode = MODE_FINAL;
                c.final_status = LP_TIME_LIMIT;
                put_ctl(P, c, d.ctl);
                run_check<T>(P);
                get_ctl(P, d.ctl);
                resolve_confirm<T>(P);
                break;
            }
        }
    }
    sync(P);
    P->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    P->has_result = true;
    return LP_OK;
}

template <typename T>
int do_result(const lp_problem *Pc, double *x, double *y, double *lam, lp_info *info)
{
    lp_problem *P = const_cast<lp_problem *>(Pc);
    Dev<T> &d = P->dev<T>();
    const int64_t m = P->m, n = P->n;
    if ((x || y || lam) && P->opt.ptr_kind == LP_DEVICE) {
        HIPT(launch_result<T>(d, P->stage_n0, P->stage_m, P->stage_n1, P->stream));
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        if (x && n) HIPT(hipMemcpyAsync(x, P->stage_n0, sizeof(double) * (size_t)n, k, P->stream));
        if (lam && n) HIPT(hipMemcpyAsync(lam, P->stage_n1, sizeof(double) * (size_t)n, k, P->stream));
        if (y && m) HIPT(hipMemcpyAsync(y, P->stage_m, sizeof(double) * (size_t)m, k, P->stream));
        sync(P);
    } else if (x || y || lam) {
        HIPT(launch_result<T>(d, P->stage_n0, P->stage_m, P->stage_n1, P->stream));
        if (x) download(P, x, P->stage_n0, n);
        if (y) download(P, y, P->stage_m, m);
        if (lam) download(P, lam, P->stage_n1, n);
        sync(P);
    }
    if (info) {
        get_ctl(P, d.ctl);
        const Ctl &c = *P->hctl;
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
        info->seconds = P->seconds;
    }
    return LP_OK;
}

// state vectors: x y Kx KTy xa ya Kxa KTya x0 y0
template <typename T>
void state_vectors(lp_problem *P, T *(&v)[10], bool (&is_n)[10])
{
    Dev<T> &d = P->dev<T>();
    const int c = P->hctl->cur;
    T *list[10] = {d.xb[c], d.yb[c], d.Kxb[c], d.KTyb[c], d.xa, d.ya, d.Kxa, d.KTya, d.x0, d.y0};
    const bool nn[10] = {true, false, false, true, true, false, false, true, true, false};
    for (int i = 0; i < 10; ++i) {
        v[i] = list[i];
        is_n[i] = nn[i];
    }
}

template <typename T>
int do_get_state(const lp_problem *Pc, double *buf)
{
    lp_problem *P = const_cast<lp_problem *>(Pc);
    Dev<T> &d = P->dev<T>();
    get_ctl(P, d.ctl);
    const Ctl &c = *P->hctl;
    std::fill(buf, buf + kNScalars, 0.0);
    buf[0] = c.eta; buf[1] = c.omega; buf[2] = c.W; buf[3] = c.KKT0; buf[4] = c.KKT_prev;
    buf[5] = (double)c.k; buf[6] = (double)c.t; buf[7] = (double)c.attempts; buf[8] = (double)c.restarts;
    buf[9] = c.status; buf[10] = c.eta_last;
    T *v[10];
    bool is_n[10];
    state_vectors<T>(P, v, is_n);
    double *p = buf + kNScalars;
    for (int i = 0; i < 10; ++i) {
        const int64_t len = is_n[i] ? P->n : P->m;
        double *stage = is_n[i] ? P->stage_n0 : P->stage_m;
        HIPT(launch_to_double<T>(v[i], stage, len, P->stream));
        download(P, p, stage, len);
        sync(P);
        p += len;
    }
    return LP_OK;
}

template <typename T>
int do_set_state(lp_problem *P, const double *buf)
{
    Dev<T> &d = P->dev<T>();
    Ctl c{};
    c.eta = buf[0]; c.omega = buf[1]; c.W = buf[2]; c.KKT0 = buf[3]; c.KKT_prev = buf[4];
    c.k = (long long)buf[5]; c.t = (long long)buf[6]; c.attempts = (long long)buf[7];
    c.restarts = (long long)buf[8]; c.eta_last = buf[10];
    c.cur = 0;
    *P->hctl = c;
    T *v[10];
    bool is_n[10];
    state_vectors<T>(P, v, is_n);
    const double *p = buf + kNScalars;
    for (int i = 0; i < 10; ++i) {
        const int64_t len = is_n[i] ? P->n : P->m;
        double *stage = is_n[i] ? P->stage_n0 : P->stage_m;
        upload(P, stage, p, len);
        HIPT(launch_from_double<T>(stage, v[i], len, P->stream));
        sync(P);
        p += len;
    }
    HIPT(hipMemcpyAsync(d.ctl, P->hctl, sizeof(Ctl), hipMemcpyHostToDevice, P->stream));
    sync(P);
    P->state_ready = true;
    return LP_OK;
}

template <typename T>
int do_spmv(lp_problem *P, int transpose, const double *in, double *out)
{
    Dev<T> &d = P->dev<T>();
    const int64_t lin = transpose ? P->m : P->n, lout = transpose ? P->n : P->m;
    double *sin = transpose ? P->stage_m : P->stage_n0;
    double *sout = transpose ? P->stage_n0 : P->stage_m;
    T *tin = (T *)(transpose ? P->tmp_m : P->tmp_n);
    T *tout = (T *)(transpose ? P->tmp_n : P->tmp_m);
    upload(P, sin, in, lin);
    HIPT(launch_from_double<T>(sin, tin, lin, P->stream));
    if (transpose)
        HIPT(launch_spmv<T>(d.KT, tin, tout, P->stream));
    else
        HIPT(launch_spmv<T>(d.K, tin, tout, P->stream));
    HIPT(launch_to_double<T>(tout, sout, lout, P->stream));
    download(P, out, sout, lout);
    sync(P);
    return LP_OK;
}

// Bytes of fixed scratch one product of lp_spmv_noalloc uses, laid out as
// [S partial vectors][long-row chunk sums][mixed only: FP32 input, FP32 output],
// each part 256-byte aligned.
template <typename T>
size_t noalloc_plan(const Sliced<T> &q, int64_t lin, int64_t lout, size_t off[4])
{
    size_t at = 0;
    off[0] = at;
    at += dev_round(sizeof(T) * (size_t)q.S * (size_t)std::max(q.rows, 1));
    off[1] = at;
    at += dev_round(sizeof(T) * (size_t)std::max(q.nlpart, 1));
    off[2] = at;
    if (sizeof(T) != sizeof(double)) {
        at += dev_round(sizeof(T) * (size_t)std::max<int64_t>(lin, 1));
        off[3] = at;
        at += dev_round(sizeof(T) * (size_t)std::max<int64_t>(lout, 1));
    } else {
        off[3] = at;
    }
    return at;
}

// The product of lp_spmv on device buffers, with every intermediate in the
// fixed scratch array: no allocation, no synchronisation.
template <typename T>
int do_spmv_noalloc(lp_problem *P, int transpose, const double *in, double *out)
{
    Dev<T> &d = P->dev<T>();
    const int64_t lin = transpose ? P->m : P->n, lout = transpose ? P->n : P->m;
    Sliced<T> q = transpose ? d.KT : d.K;
    size_t off[4];
    const size_t need = noalloc_plan(q, lin, lout, off);
    if (need > kNoallocScratchBytes) {
        char buf[200];
        snprintf(buf, sizeof(buf), "lp_spmv_noalloc: this product needs %zu bytes of scratch, the fixed array holds %zu",
                 need, kNoallocScratchBytes);
        P->err = buf;
        return LP_ERR_NOMEM;
    }
    unsigned char *base = (unsigned char *)P->nscratch;
    q.part = (T *)(base + off[0]);
    q.lpart = (T *)(base + off[1]);
    // every partial slot the slice sums read is written by the partial pass
    // (each slice's row blocks cover all rows; long rows use lpart, whose
    // chunks are all written), so nothing in the scratch needs clearing
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPT(launch_spmv<T>(q, (const T *)in, (T *)out, P->stream));
    } else {
        T *tin = (T *)(base + off[2]), *tout = (T *)(base + off[3]);
        HIPT(launch_from_double<T>(in, tin, lin, P->stream));
        HIPT(launch_spmv<T>(q, tin, tout, P->stream));
        HIPT(launch_to_double<T>(tout, out, lout, P->stream));
    }
    return LP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void lp_default_options(lp_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = LP_FP64;
    o->stream = nullptr;
    o->ruiz_iters = 10;
    o->pc_alpha = 1.0;
    o->check_every = 64;
    o->kkt_omega_power = 2.0;
    o->fixed_step = 0;
    o->fixed_eta = 0.0;
    o->use_graph = 1;
    o->window = 64;
    o->kernel_timing = 0;
    o->slice_kib = 2048;
    o->autotune = 0;
    o->verbose = 0;
    o->infeas_tol = 1e-8;
    o->persistent = -1;
    o->split_sums = -1;
}

int lp_workspace_size(const lp_csr *K, const lp_options *opt, size_t *bytes)
{
    if (!K || !bytes) return LP_ERR_ARG;
    lp_options o;
    if (opt) o = *opt;
    else lp_default_options(&o);
    int rc = check_options(o);
    if (rc != LP_OK) return rc;
    if (o.presolve) return LP_ERR_ARG;   // the reduced size is only known with the data
    try {
        HostLP H;
        if (o.ptr_kind == LP_DEVICE) {
            rc = fetch_lp(K, nullptr, nullptr, nullptr, nullptr, (hipStream_t)o.stream, H);
            if (rc != LP_OK) return rc;
            K = &H.K;
        }
        rc = validate_pattern(K);
        if (rc != LP_OK) return rc;
        // the layout depends on the pattern only: zeros stand in for the values
        std::vector<double> zeros((size_t)std::max<int64_t>(K->nnz, 1), 0.0);
        lp_csr P = *K;
        P.val = zeros.data();
        std::vector<int> rp, ci, tp, ti;
        std::vector<double> kv, tv;
        HostSliced HK, HT;
        host_layout(&P, o.precision == LP_MIXED, o.slice_kib, rp, ci, kv, tp, ti, tv, HK, HT);
        *bytes = load_plan_bytes(K->m, K->n, K->nnz, HK, HT, o.precision == LP_MIXED);
    } catch (const HipError &) {
        return LP_ERR_HIP;
    } catch (const std::bad_alloc &) {
        return LP_ERR_NOMEM;
    }
    return LP_OK;
}

int lp_load(lp_problem **out, const lp_csr *K, const double *c, const double *q, const double *l, const double *u,
            int64_t m1, const lp_options *opt)
{
    if (!out) return LP_ERR_ARG;
    *out = nullptr;
    lp_options o;
    if (opt) o = *opt;
    else lp_default_options(&o);
    int rc = check_options(o);
    if (rc != LP_OK) return rc;
    HostLP H;
    if (o.ptr_kind == LP_DEVICE) {
        if (!K || (K->n > 0 && !c)) return LP_ERR_ARG;
        try {
            rc = fetch_lp(K, c, q, l, u, (hipStream_t)o.stream, H);
        } catch (const HipError &) {
            return LP_ERR_HIP;
        } catch (const std::bad_alloc &) {
            return LP_ERR_NOMEM;
        }
        if (rc != LP_OK) return rc;
        K = &H.K;
        c = H.c.data(); q = H.q.data(); l = H.l.data(); u = H.u.data();
    }
    rc = validate_lp(K, c, q, l, u, m1);
    if (rc != LP_OK) return rc;
    std::unique_ptr<lp_problem> P;
    try {
        P.reset(new lp_problem());
        if (o.presolve) {
            std::unique_ptr<Presolved> R(new Presolved());
            if (presolve(K, c, q, l, u, m1, *R)) {
                K = &R->K;
                c = R->c.data(); q = R->q.data(); l = R->l.data(); u = R->u.data();
                m1 = R->m1;
                P->pre = std::move(R);
            }
        }
    } catch (...) {
        return LP_ERR_NOMEM;
    }
    P->m = K->m; P->n = K->n; P->nnz = K->nnz; P->m1 = m1;
    P->opt = o;
    P->mixed = o.precision == LP_MIXED;
    P->stream = (hipStream_t)o.stream;
    P->ws = (char *)o.workspace;
    P->ws_size = o.workspace ? o.workspace_bytes : 0;
    try {
        if (!P->stream) {
            // a stream of our own (default priority) so the window can be graph-captured
            HIPT(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking));
            P->own_stream = true;
        }
        HIPT(hipHostMalloc((void **)&P->hctl, sizeof(Ctl), hipHostMallocDefault));
        std::memset(P->hctl, 0, sizeof(Ctl));
        HIPT(hipGetDevice(&P->device));
        // set-up of lp_spmv_noalloc's scratch on this device (once per device);
        // a failed lookup only disables that call
        if (noalloc_scratch(&P->nscratch) != hipSuccess) {
            P->nscratch = nullptr;
            (void)hipGetLastError();
        }
        rc = do_load(P.get(), K, c, q, l, u);
    } catch (const HipError &h) {
        rc = h.e == hipErrorOutOfMemory ? LP_ERR_NOMEM : LP_ERR_HIP;
        if (o.verbose) fprintf(stderr, "lp_load: %s failed: %s\n", h.what, hipGetErrorString(h.e));
    } catch (const std::bad_alloc &) {
        rc = LP_ERR_NOMEM;
    }
    if (rc != LP_OK) {
        if (o.verbose && !P->err.empty()) fprintf(stderr, "lp_load: %s\n", P->err.c_str());
        return rc;
    }
    *out = P.release();
    return LP_OK;
}

int lp_set_start(lp_problem *P, const double *x0, const double *y0)
{
    if (!P) return LP_ERR_ARG;
    P->has_xs = x0 != nullptr;
    P->has_ys = y0 != nullptr;
    if (P->opt.ptr_kind == LP_DEVICE) {
        try {
            if (x0) fetch(P->xs, x0, P->n, P->stream);
            if (y0) fetch(P->ys, y0, P->m, P->stream);
            HIPT(hipStreamSynchronize(P->stream));
        } catch (const HipError &h) {
            return fail_hip(P, h);
        }
    } else if (P->pre) {
        // original-space start point: keep the entries of the reduced problem
        const Presolved &R = *P->pre;
        if (x0) {
            P->xs.assign((size_t)P->n, 0.0);
            for (int64_t j = 0; j < R.n0; ++j)
                if (R.col_new[(size_t)j] >= 0) P->xs[(size_t)R.col_new[(size_t)j]] = x0[j];
        }
        if (y0) {
            P->ys.assign((size_t)P->m, 0.0);
            for (int64_t i = 0; i < R.m0; ++i)
                if (R.row_new[(size_t)i] >= 0) P->ys[(size_t)R.row_new[(size_t)i]] = y0[i];
        }
    } else {
        if (x0) P->xs.assign(x0, x0 + P->n);
        if (y0) P->ys.assign(y0, y0 + P->m);
    }
    P->state_ready = false;
    return LP_OK;
}

int lp_set_start_weight(lp_problem *P, double omega)
{
    if (!P || std::isnan(omega) || std::isinf(omega)) return LP_ERR_ARG;
    P->omega_start = omega > 0.0 ? omega : 0.0;
    P->state_ready = false;
    return LP_OK;
}

int lp_solve(lp_problem *P, double tol, int64_t max_iters, double time_limit_s)
{
    if (!P || max_iters < 0 || std::isnan(tol)) return LP_ERR_ARG;
    try {
        return P->mixed ? do_solve<float>(P, tol, max_iters, time_limit_s)
                        : do_solve<double>(P, tol, max_iters, time_limit_s);
    } catch (const HipError &h) {
        return fail_hip(P, h);
    } catch (const std::bad_alloc &) {
        return LP_ERR_NOMEM;
    }
}

int lp_result(const lp_problem *P, double *x, double *y, double *lambda, lp_info *info)
{
    if (!P) return LP_ERR_ARG;
    if (!P->has_result) return LP_ERR_STATE;
    try {
        if (!P->pre)
            return P->mixed ? do_result<float>(P, x, y, lambda, info) : do_result<double>(P, x, y, lambda, info);
        // presolved: the reduced point, mapped back and evaluated on the original problem
        const Presolved &R = *P->pre;
        std::vector<double> xr((size_t)std::max<int64_t>(P->n, 1)), yr((size_t)std::max<int64_t>(P->m, 1));
        lp_info ri{};
        const int rc = P->mixed ? do_result<float>(P, xr.data(), yr.data(), nullptr, &ri)
                                : do_result<double>(P, xr.data(), yr.data(), nullptr, &ri);
        if (rc != LP_OK) return rc;
        if (ri.status == LP_PRIMAL_INFEASIBLE || ri.status == LP_DUAL_INFEASIBLE) {
            // the rays of the reduced problem, zero on the removed rows and columns
            for (int64_t j = 0; j < R.n0; ++j) {
                const int k = R.col_new[(size_t)j];
                if (x) x[j] = k >= 0 ? xr[(size_t)k] : 0.0;
                if (lambda) lambda[j] = 0.0;
            }
            if (y)
                for (int64_t i = 0; i < R.m0; ++i) {
                    const int k = R.row_new[(size_t)i];
                    y[i] = k >= 0 ? yr[(size_t)k] : 0.0;
                }
        } else {
            postsolve(R, xr.data(), yr.data(), x, y, lambda, ri.pobj, ri.dobj, ri.rel_primal, ri.rel_dual,
                      ri.rel_gap);
        }
        if (info) *info = ri;
        return LP_OK;
    } catch (const HipError &h) {
        return fail_hip(const_cast<lp_problem *>(P), h);
    } catch (const std::bad_alloc &) {
        return LP_ERR_NOMEM;
    }
}

int lp_presolved_size(const lp_problem *P, int64_t *m, int64_t *n)
{
    if (!P) return LP_ERR_ARG;
    if (m) *m = P->m;
    if (n) *n = P->n;
    return LP_OK;
}

int lp_get_state(const lp_problem *P, double *buf, int64_t *len)
{
    if (!P || !len) return LP_ERR_ARG;
    *len = kNScalars + 5 * P->n + 5 * P->m;
    if (!buf) return LP_OK;
    try {
        return P->mixed ? do_get_state<float>(P, buf) : do_get_state<double>(P, buf);
    } catch (const HipError &h) {
        return fail_hip(const_cast<lp_problem *>(P), h);
    }
}

int lp_set_state(lp_problem *P, const double *buf, int64_t len)
{
    if (!P || !buf) return LP_ERR_ARG;
    if (len != kNScalars + 5 * P->n + 5 * P->m) return LP_ERR_STATE;
    try {
        return P->mixed ? do_set_state<float>(P, buf) : do_set_state<double>(P, buf);
    } catch (const HipError &h) {
        return fail_hip(P, h);
    }
}

int lp_get_scaling(const lp_problem *Pc, double *Dr, double *Dc)
{
    if (!Pc) return LP_ERR_ARG;
    lp_problem *P = const_cast<lp_problem *>(Pc);
    try {
        const double *dDr = P->mixed ? P->d32.Dr : P->d64.Dr;
        const double *dDc = P->mixed ? P->d32.Dc : P->d64.Dc;
        if (Dr) download(P, Dr, dDr, P->m);
        if (Dc) download(P, Dc, dDc, P->n);
        sync(P);
    } catch (const HipError &h) {
        return fail_hip(P, h);
    }
    return LP_OK;
}

int lp_spmv(lp_problem *P, int transpose, const double *in, double *out)
{
    if (!P || !in || !out) return LP_ERR_ARG;
    try {
        return P->mixed ? do_spmv<float>(P, transpose, in, out) : do_spmv<double>(P, transpose, in, out);
    } catch (const HipError &h) {
        return fail_hip(P, h);
    }
}

int lp_spmv_noalloc(lp_problem *P, int transpose, const double *in, double *out)
{
    if (!P || !in || !out) return LP_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != P->device) {
        P->err = "lp_spmv_noalloc: the handle's device is not the current device";
        return LP_ERR_ARG;
    }
    if (!P->nscratch) {
        P->err = "lp_spmv_noalloc: the fixed scratch array is not available on this device";
        return LP_ERR_HIP;
    }
    try {
        return P->mixed ? do_spmv_noalloc<float>(P, transpose, in, out)
                        : do_spmv_noalloc<double>(P, transpose, in, out);
    } catch (const HipError &h) {
        return fail_hip(P, h);
    }
}

int lp_gather_probe(const int32_t *idx, const void *x, int precision, int64_t count, int slices, int64_t slice_len,
                    void *out, int reps, void *stream, double *ms_per_pass)
{
    if (!idx || !x || !out || !ms_per_pass || count <= 0 || slices <= 0 || slice_len <= 0 || reps <= 0 ||
        count % slices != 0 || slices > 4096 || (precision != LP_FP64 && precision != LP_MIXED))
        return LP_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int64_t per = count / slices;
    const int unit = std::max(slices, kXcds);
    const int grid = std::max(4096 / unit, 1) * unit;
    try {
        EventPair ev;
        auto pass = [&] {
            if (precision == LP_FP64)
                HIPT(launch_gather_probe<double>(idx, (const double *)x, per, slices, slice_len, (double *)out, grid,
                                                 st));
            else
                HIPT(launch_gather_probe<float>(idx, (const float *)x, per, slices, slice_len, (float *)out, grid, st));
        };
        pass();
        HIPT(hipEventRecord(ev.a, st));
        for (int r = 0; r < reps; ++r) pass();
        HIPT(hipEventRecord(ev.b, st));
        HIPT(hipEventSynchronize(ev.b));
        *ms_per_pass = (double)ev.ms() / reps;
    } catch (const HipError &) {
        return LP_ERR_HIP;
    }
    return LP_OK;
}

int lp_kernel_time(const lp_problem *P, int which, int64_t *count, double *total_ms)
{
    if (!P || !count || !total_ms || which < 0 || which > 1) return LP_ERR_ARG;
    *count = P->t_count[which];
    *total_ms = P->t_ms[which];
    return LP_OK;
}

int lp_device_bytes(const lp_problem *P, int64_t *bytes)
{
    if (!P || !bytes) return LP_ERR_ARG;
    *bytes = P->dev_bytes;
    return LP_OK;
}

int lp_layout(const lp_problem *P, int *slices_K, int *slices_KT)
{
    if (!P) return LP_ERR_ARG;
    if (slices_K) *slices_K = P->slices_K;
    if (slices_KT) *slices_KT = P->slices_KT;
    return LP_OK;
}

int lp_layout_blocks(const lp_problem *P, int which, int *slices, int *nnz_per_block, int *rows_per_block)
{
    if (!P || (which != 0 && which != 1)) return LP_ERR_ARG;
    const int *s = which ? P->shape_KT : P->shape_K;
    if (slices) *slices = s[0];
    if (nnz_per_block) *nnz_per_block = s[1];
    if (rows_per_block) *rows_per_block = s[2];
    return LP_OK;
}

int lp_layout_split(const lp_problem *P, int which, int *split)
{
    if (!P || (which != 0 && which != 1) || !split) return LP_ERR_ARG;
    *split = which ? P->split_KT : P->split_K;
    return LP_OK;
}

void lp_free(lp_problem *P)
{
    if (!P) return;
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    else (void)hipDeviceSynchronize();
    delete P;
}

const char *lp_strerror(int code)
{
    switch (code) {
    case LP_OK: return "ok";
    case LP_ERR_ARG: return "invalid argument";
    case LP_ERR_DIM: return "inconsistent dimensions or CSR structure";
    case LP_ERR_NAN: return "NaN or infinity in the data";
    case LP_ERR_BOUNDS: return "inconsistent variable bounds";
    case LP_ERR_TOO_LARGE: return "problem too large for 32-bit indices";
    case LP_ERR_STATE: return "call out of order or state of the wrong size";
    case LP_ERR_HIP: return "HIP runtime error";
    case LP_ERR_NOMEM: return "out of memory";
    default: return "unknown error";
    }
}

const char *lp_last_error(const lp_problem *P)
{
    if (!P) return "";
    return P->err.c_str();
}

}  // extern "C"
