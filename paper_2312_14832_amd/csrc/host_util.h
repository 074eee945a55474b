// Host-side helpers shared by the single-LP and the batched C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "internal.h"

namespace pdlp {

struct HipError {
    hipError_t e;
    const char *what;
};

#define HIPT(expr)                                                       \
    do {                                                                 \
        hipError_t _e = (expr);                                          \
        if (_e != hipSuccess) throw pdlp::HipError{_e, #expr};           \
    } while (0)

// Device allocations owned by one handle, released together.
struct Arena {
    std::vector<void *> ptrs;
    std::vector<int64_t> sizes;
    int64_t bytes = 0;
    int fill = -1;   // >= 0: every new allocation is filled with this byte (a test hook for reads of unset memory)
    void *alloc(size_t n)
    {
        void *p = nullptr;
        if (n == 0) n = 8;
        n = (n + 255) & ~(size_t)255;
        HIPT(hipMalloc(&p, n));
        if (fill >= 0) {
            HIPT(hipMemset(p, fill, n));
            HIPT(hipDeviceSynchronize());
        }
        ptrs.push_back(p);
        sizes.push_back((int64_t)n);
        bytes += (int64_t)n;
        return p;
    }
    template <typename T> T *make(int64_t count) { return (T *)alloc(sizeof(T) * (size_t)std::max<int64_t>(count, 1)); }
    void release(void *p)
    {
        for (size_t i = 0; i < ptrs.size(); ++i)
            if (ptrs[i] == p) {
                (void)hipFree(p);
                ptrs[i] = nullptr;
                bytes -= sizes[i];
            }
    }
    ~Arena()
    {
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    }
};

// Two timing events, destroyed with the object (also when a call between
// them throws).
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair()
    {
        HIPT(hipEventCreate(&a));
        const hipError_t e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            throw HipError{e, "hipEventCreate"};
        }
    }
    ~EventPair()
    {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    float ms() const
    {
        float t = 0;
        HIPT(hipEventElapsedTime(&t, a, b));
        return t;
    }
};

template <typename T>
inline void h2d(hipStream_t st, T *dst, const T *src, int64_t count)
{
    if (count > 0) HIPT(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)count, hipMemcpyHostToDevice, st));
}

template <typename T>
inline void d2h(hipStream_t st, T *dst, const T *src, int64_t count)
{
    if (count > 0) HIPT(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost, st));
}

template <typename T>
inline void d2d(hipStream_t st, T *dst, const T *src, int64_t count)
{
    if (count > 0) HIPT(hipMemcpyAsync(dst, src, sizeof(T) * (size_t)count, hipMemcpyDeviceToDevice, st));
}

// The input rules of lp_load (LP_ERR_* codes of lp.h).
int validate_lp(const lp_csr *K, const double *c, const double *q, const double *l, const double *u, int64_t m1);
// Sizes and pointers of a CSR only; then its structure (no values).
int validate_dims(const lp_csr *K);
int validate_pattern(const lp_csr *K);

// Worker threads for host-side layout work (at most 16).
int host_threads();

// Append the rows of K (columns sorted inside each row, columns shifted by
// col_off) to a CSR under construction.
void append_sorted_rows(const lp_csr *K, int col_off, std::vector<int> &rp, std::vector<int> &ci,
                        std::vector<double> &v);

// CSR of the transpose by a counting sort over the rows (each output row
// comes out sorted by the input row index).
void transpose_csr(int rows, int cols, const std::vector<int> &rp, const std::vector<int> &ci,
                   const std::vector<double> &v, std::vector<int> &tp, std::vector<int> &ti, std::vector<double> &tv);

// CSR-Stream row blocks of rows [r_begin, r_end): at most kStreamRB rows and
// nb_max (<= kStreamNB) nonzeros each (a longer single row is a block of its
// own).  Appends block end rows to `ends` (the first block starts at r_begin).
// Row blocks of rows [r_begin, r_end): runs of rows of at most kWaveRow
// entries (at most rb_max rows and nb_max entries), and groups of up to
// kBlock/64 longer rows (at most nb_max entries; a row longer than that is a
// block of its own).  ends[k] is the end row of block k; wave[k] = 1 marks a
// group of long rows.
void row_blocks(const int *rp, int r_begin, int r_end, std::vector<int> &ends, std::vector<char> &wave,
                int nb_max = kStreamNB, int rb_max = kStreamRB);

}  // namespace pdlp
