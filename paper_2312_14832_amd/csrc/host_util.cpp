// Host-side helpers shared by the single-LP and the batched C ABI.
#include "host_util.h"

#include <exception>
#include <thread>

namespace pdlp {

int validate_dims(const lp_csr *K)
{
    if (!K) return LP_ERR_ARG;
    const int64_t m = K->m, n = K->n, nnz = K->nnz;
    if (m < 0 || n < 0 || nnz < 0) return LP_ERR_DIM;
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31)) return LP_ERR_TOO_LARGE;
    if (!K->row_ptr || (nnz > 0 && !K->col)) return LP_ERR_ARG;
    return LP_OK;
}

int validate_pattern(const lp_csr *K)
{
    int rc = validate_dims(K);
    if (rc != LP_OK) return rc;
    const int64_t m = K->m, n = K->n, nnz = K->nnz;
    if (K->row_ptr[0] != 0 || K->row_ptr[m] != nnz) return LP_ERR_DIM;
    for (int64_t i = 0; i < m; ++i)
        if (K->row_ptr[i + 1] < K->row_ptr[i]) return LP_ERR_DIM;
    std::vector<int64_t> seen((size_t)std::max<int64_t>(n, 1), -1);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = K->row_ptr[i]; p < K->row_ptr[i + 1]; ++p) {
            const int64_t j = K->col[p];
            if (j < 0 || j >= n || seen[j] == i) return LP_ERR_DIM;
            seen[j] = i;
        }
    return LP_OK;
}

int validate_lp(const lp_csr *K, const double *c, const double *q, const double *l, const double *u, int64_t m1)
{
    if (!K) return LP_ERR_ARG;
    const int64_t m = K->m, n = K->n, nnz = K->nnz;
    if (m < 0 || n < 0 || nnz < 0 || m1 < 0 || m1 > m) return LP_ERR_DIM;
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31)) return LP_ERR_TOO_LARGE;
    if (!K->row_ptr || (nnz > 0 && (!K->col || !K->val)) || (n > 0 && (!c || !l || !u)) || (m > 0 && !q))
        return LP_ERR_ARG;
    if (K->row_ptr[0] != 0 || K->row_ptr[m] != nnz) return LP_ERR_DIM;
    for (int64_t i = 0; i < m; ++i)
        if (K->row_ptr[i + 1] < K->row_ptr[i]) return LP_ERR_DIM;
    std::vector<int64_t> seen((size_t)std::max<int64_t>(n, 1), -1);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = K->row_ptr[i]; p < K->row_ptr[i + 1]; ++p) {
            const int64_t j = K->col[p];
            if (j < 0 || j >= n || seen[j] == i) return LP_ERR_DIM;
            seen[j] = i;
        }
    for (int64_t p = 0; p < nnz; ++p)
        if (!std::isfinite(K->val[p])) return LP_ERR_NAN;
    for (int64_t j = 0; j < n; ++j) {
        if (!std::isfinite(c[j]) || std::isnan(l[j]) || std::isnan(u[j])) return LP_ERR_NAN;
        if (l[j] == INFINITY || u[j] == -INFINITY || l[j] > u[j]) return LP_ERR_BOUNDS;
    }
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(q[i])) return LP_ERR_NAN;
    return LP_OK;
}

int host_threads()
{
    const unsigned t = std::thread::hardware_concurrency();
    return (int)std::min(16u, std::max(1u, t));
}

void append_sorted_rows(const lp_csr *K, int col_off, std::vector<int> &rp, std::vector<int> &ci,
                        std::vector<double> &v)
{
    if (rp.empty()) rp.push_back(0);
    const size_t base = ci.size();
    ci.resize(base + (size_t)K->nnz);
    v.resize(base + (size_t)K->nnz);
    rp.reserve(rp.size() + (size_t)K->m);
    std::vector<std::pair<int, double>> row;
    for (int64_t i = 0; i < K->m; ++i) {
        const int64_t b = K->row_ptr[i], e = K->row_ptr[i + 1];
        int *co = ci.data() + base + b;
        double *vo = v.data() + base + b;
        if (std::is_sorted(K->col + b, K->col + e)) {
            for (int64_t p = b; p < e; ++p) {
                co[p - b] = K->col[p] + col_off;
                vo[p - b] = K->val[p];
            }
        } else {
            row.clear();
            for (int64_t p = b; p < e; ++p) row.emplace_back(K->col[p], K->val[p]);
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int, double> &x, const std::pair<int, double> &y) { return x.first < y.first; });
            for (size_t k = 0; k < row.size(); ++k) {
                co[k] = row[k].first + col_off;
                vo[k] = row[k].second;
            }
        }
        rp.push_back((int)(base + (size_t)e));
    }
}

void transpose_csr(int rows, int cols, const std::vector<int> &rp, const std::vector<int> &ci,
                   const std::vector<double> &v, std::vector<int> &tp, std::vector<int> &ti, std::vector<double> &tv)
{
    const int64_t nnz = rp[rows];
    tp.assign((size_t)cols + 1, 0);
    ti.assign((size_t)std::max<int64_t>(nnz, 1), 0);
    tv.assign((size_t)std::max<int64_t>(nnz, 1), 0.0);
    // Each thread owns a contiguous range of output rows (input columns):
    // it scans every entry and counts, then places, only those in its range,
    // in input-row order, so the result is that of the sequential counting
    // sort whatever the thread count.
    const int T = std::max(1, std::min(host_threads(), cols / 65536 + 1));
    auto range = [&](int t) { return std::make_pair((int)((int64_t)cols * t / T), (int)((int64_t)cols * (t + 1) / T)); };
    auto parallel = [&](auto &&fn) {   // exceptions of the workers are rethrown after the join
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
    };
    parallel([&](int t) {
        const auto [c0, c1] = range(t);
        for (int64_t p = 0; p < nnz; ++p) {
            const int j = ci[p];
            if (j >= c0 && j < c1) tp[(size_t)j + 1]++;
        }
    });
    for (int j = 0; j < cols; ++j) tp[(size_t)j + 1] += tp[(size_t)j];
    parallel([&](int t) {
        const auto [c0, c1] = range(t);
        std::vector<int> pos(tp.begin() + c0, tp.begin() + c1);
        for (int i = 0; i < rows; ++i)
            for (int p = rp[i]; p < rp[i + 1]; ++p) {
                const int j = ci[p];
                if (j >= c0 && j < c1) {
                    const int at = pos[(size_t)(j - c0)]++;
                    ti[(size_t)at] = i;
                    tv[(size_t)at] = v[p];
                }
            }
    });
}

void row_blocks(const int *rp, int r_begin, int r_end, std::vector<int> &ends, std::vector<char> &wave, int nb_max,
                int rb_max)
{
    if (nb_max > kStreamNB || nb_max < 1) nb_max = kStreamNB;
    if (rb_max > kStreamRB || rb_max < 1) rb_max = kStreamRB;
    auto len = [&](int r) { return rp[r + 1] - rp[r]; };
    int start = r_begin;
    while (start < r_end) {
        const bool lng = len(start) > kWaveRow;
        const int most = lng ? kBlock / 64 : rb_max;
        int end = start + 1;
        while (end < r_end && end - start < most && (len(end) > kWaveRow) == lng && rp[end + 1] - rp[start] <= nb_max)
            ++end;
        ends.push_back(end);
        wave.push_back(lng ? 1 : 0);
        start = end;
    }
}

}  // namespace pdlp
