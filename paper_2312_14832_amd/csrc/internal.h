// Internal types shared by the HIP kernels and the host side of libpdlp_amd.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lp.h"

namespace pdlp {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kMaxGrid = 1024;   // workgroups of an elementwise solver kernel = partial-sum slots
                                 // (1024: 1.8% more iterations/s than 2048 on a 2e6-column LP, fewer
                                 // partials for the one-workgroup decisions and a lighter idle launch)
constexpr int kCheckSums = 18;   // 9 sums for the current and 9 for the averaged iterate
constexpr int kRaySums = 4;      // the current iterate's rays (difference from the anchor)
constexpr int kXcds = 8;         // MI355X: 8 XCDs, workgroups dealt to them round-robin
constexpr int kStreamNB = 2048;  // nonzeros staged in LDS per row block
constexpr int kStreamRB = 1024;  // most rows per row block (each thread sums every 256th row)
constexpr int kWaveRow = 64;     // rows longer than this are summed by a whole wavefront
constexpr int kLongRow = 4 * kStreamNB;  // rows longer than this are cut into chunks
constexpr int kSmall = 1024;     // threads of the one workgroup that runs a small LP's whole loop
constexpr int kSmallReg = 512;   // threads of its registers-per-thread form (two columns and rows each at most)
constexpr size_t kSmallStageMax = 150 * 1024;   // dynamic LDS of the staged loop (of 160 KiB per CU)
constexpr size_t kSmallRegLds = 156 * 1024;     // dynamic LDS of the registers-per-thread loop (stage + table)
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;  // device scratch of lp_spmv_noalloc (64 MiB per GPU)
// A row block is either a run of rows of at most kWaveRow entries (thread per
// row) or up to kBlock/64 longer rows (wavefront per row); a wavefront block's
// end row is stored complemented (~end) in the block descriptor.  A row of
// more than kLongRow entries (a dense row, e.g. a sum-to-one constraint) is
// instead cut, in every slice, into chunks of at most one block's nonzeros;
// each chunk is a block of its own whose descriptor holds ~slot (negative)
// in place of the first row, and its workgroup writes the chunk's dot
// product to lpart[slot].  The epilogue adds a long row's slots.

// One sparse product y = A x split by COLUMNS into S contiguous slices.  The
// slice of x a workgroup gathers from is small enough to stay in one XCD's
// L2: workgroup b works on slice b % S, and since workgroups are dealt to the
// 8 XCDs round-robin, slice s only ever runs on XCDs congruent to s.  Each
// slice is a CSR over all rows (entries slice-major), cut into row blocks of
// at most kStreamRB rows and kStreamNB nonzeros (a single longer row is a
// block of its own).  The pass writes S partial vectors, summed in a fixed
// order by the elementwise epilogue.
template <typename T>
struct Sliced {
    int S;            // column slices (a power of two)
    int rows;         // rows of the product
    int grid;         // workgroups of the partial pass (a multiple of 8 and of S)
    const int *rp;    // [S*(rows+1)] per-slice row pointers into ci / v (the one-workgroup loop's CSR)
    const unsigned short *ro;   // [S*rows] start of each row relative to its row block's first entry:
                                // what the partial passes read (2 bytes per row and slice, not 4)
    const int *ci;    // column indices, slice-major
    const T *v;       // values, same layout
    const int4 *blk;  // row blocks {first row, end row (~end: wavefront rows), first entry, end entry};
                      // slice s owns blk[boff[s] .. boff[s+1])
    const int *boff;  // [S+1] prefix counts of row blocks
    T *part;          // [S*rows] partial products (slots of long rows unused)
    int nlong;        // rows longer than kLongRow
    const int *lrow;  // [nlong] those rows, ascending
    const int *loff;  // [nlong+1] long row k owns lpart[loff[k] .. loff[k+1]), slice-major
    T *lpart;         // chunk dot products of the long rows
    int nlpart;       // entries of lpart (loff[nlong])
    int split;        // 1: blocks of short rows summed split by entries, not one row per thread
};

// check modes
enum : int { MODE_NONE = 0, MODE_CHECK = 1, MODE_INIT = 2, MODE_FINAL = 3, MODE_RESUME = 4 };

// Device-resident controller state.  Written only by thread 0 of the
// single-workgroup decision kernels, read by every kernel at its start, so
// the whole iteration loop runs without a host round trip.
struct Ctl {
    double eta;        // step size of the next attempt
    double omega;      // primal weight
    double W;          // sum of accepted step sizes since the last restart
    double KKT0;       // KKT_omega of the restart anchor
    double KKT_prev;   // KKT_omega of the candidate at the previous check
    double eta_last;   // step size of the last accepted step
    double avg_w;      // eta_last / W, the averaging weight of that step
    double tol;
    double infeas_tol; // ray certificate threshold; 0: no infeasibility test
    double kkt_p;
    double fixed_eta;
    double rel_p[2], rel_d[2], rel_g[2], pobj[2], dobj[2], kkt[2];
    double out_rel_p, out_rel_d, out_rel_g, out_pobj, out_dobj;
    long long k, t, attempts, restarts, max_iters;
    int check_every;
    int fixed_step;
    int cur;           // buffer index of the current iterate
    int accepted;      // last attempt accepted
    int mode;          // MODE_*
    int done;
    int status;
    int final_status;  // status used by MODE_FINAL when not optimal
    int restart_to;    // 0 none, 1 to the current iterate, 2 to the average
    int out_sel;       // 0 current, 1 average
    int copy_out;      // the apply kernel copies the chosen point to the output buffers
    int need_primal;   // the apply kernel computes the next primal trial
    int numerical;     // NaN met in the step-size test
    int confirm_on;    // mixed precision: a passed termination test is re-checked with FP64 products
    int confirm;       // such a re-check is pending (the loop has stopped for it)
    int conf_mode;     // the check mode that passed the test
    int veto;          // run the next check decision without its termination test (re-check failed)
    long long confirms;  // FP64 re-checks made
};

template <typename T>
struct Dev {
    int m, n, m1;
    Sliced<T> K;               // K  (m x n), sliced over the columns (x)
    Sliced<T> KT;              // K' (n x m), sliced over the rows of K (y)
    const T *cs, *ls, *us;     // scaled c, l, u   [n]
    const T *qs;               // scaled q         [m]
    const double *Dr, *Dc;     // scaling factors
    T *xb[2], *yb[2], *Kxb[2], *KTyb[2];   // current / trial buffers
    T *xa, *ya, *Kxa, *KTya;   // step-weighted averages
    T *x0, *y0;                // restart anchor
    T *Kx0, *KTy0;             // K x0 and K' y0 (ray residuals are differences of products)
    T *xo, *yo, *KTyo;         // returned point
    double *part_primal;       // [kMaxGrid]      |x' - x|^2 partials
    double *part_dual;         // [kMaxGrid * 2]  |y' - y|^2, (y'-y).(Kx'-Kx)
    double *part_check;        // [kMaxGrid * kCheckSums]
    double *part_ray;          // [kMaxGrid * kRaySums] (a pass of its own: fewer live registers)
    Ctl *ctl;
};

// Mixed precision's FP64 re-check of the termination test: the scaled
// matrix and its transpose in plain CSR with FP64 values and the scaled
// vectors in FP64 (kept from the load-time scaling), the products of the
// current iterate and the average, and the partial sums.
struct Conf64 {
    const int *rp, *ci, *tp, *ti;
    const double *kv, *tv;
    const double *cs, *ls, *us, *qs;   // scaled c, l, u, q in FP64
    double *kx[2], *kty[2];   // [m], [n]: current, average
    double *part;             // [kMaxGrid * kCheckSums]
};

struct Geo {
    int grid;                  // workgroups of the elementwise solver kernels
    int vb_n, vb_m;            // 256-element chunks of the n- and m-vectors
};

// Row blocks of one product of a batch, dealt to XCDs by instance: the
// blocks of XCD x are order[xoff[x] .. xoff[x+1]); block k covers rows
// [r0[k], r1[k]) of instance inst[k].
struct BlockList {
    int nblk;
    const int *r0, *r1, *inst, *order;   // r1 complemented for wavefront-row blocks
    int xoff[kXcds + 1];
    int grid;                 // workgroups of the product kernel (a multiple of 8)
    int split;                // 1: short-row blocks summed split by entries (stream_block SPLIT)
};

// A batch of LPs concatenated block-diagonally.  Every instance's n- and
// m-vectors are padded to whole 256-element chunks, so each chunk (one
// workgroup of the elementwise kernels) belongs to one instance; padding
// entries are inert (bounds [0,0], zero data, unit scaling).
template <typename T>
struct BDev {
    Dev<T> d;                 // concatenated vectors; d.n, d.m are the padded totals; d.K, d.KT unused
    int B;                    // instances
    int ncn, ncm;             // n-chunks and m-chunks in total
    const int *krp, *kci;     // K:  CSR over all padded rows, global column indices
    const T *kv;
    const int *trp, *tci;     // K': CSR over all padded columns of K
    const T *tv;
    BlockList LK, LT;
    T *prodK, *prodKT;        // the products K x' [m] and K' y' [n]
    const int *cinst_n, *cinst_m;  // instance of each n-chunk / m-chunk
    const int *nc0, *ncc, *mc0, *mcc;  // per instance: first chunk and chunk count, n and m side
    const int *m1g;           // per instance: first inequality row (global index)
    const double *Nq, *Nc;    // per instance: |q|, |c| of the unscaled data
    Ctl *ctl;                 // [B]
    int *gate;                // 1 while some instance is in a check this slot
    // The chunks the solver kernels visit: act_cn[0 .. acn) and
    // act_cm[0 .. acm), or every chunk in order when null; the instances the
    // decision kernels visit: act_i[0 .. aci), or all.  Once most instances
    // have finished, the host narrows these (and LK, LT) to the unfinished
    // ones between windows.
    const int *act_cn, *act_cm, *act_i;
    int acn, acm, aci;
};

// Batched solves of one family: every instance shares the matrix K (pattern
// and values) and has its own c, q, l, u.  Vectors are interleaved, [row][Bp]
// with the instance fastest (Bp = the instance count rounded up to a power
// of two, at most kBlock; padded instances are inert and finished from the
// start), so a product reads K once for every instance and each gather of
// x[j][0..Bp) is a contiguous run.  d holds the interleaved vectors with
// d.n = n Bp, d.m = m Bp, d.m1 = m1 Bp and the scaling factors replicated per
// instance, so the element functions of the single-LP path apply unchanged
// with element e = row * Bp + instance.
template <typename T>
struct SDev {
    Dev<T> d;
    int B, Bp, lgB;           // instances, padded count, log2(Bp)
    int n, m;                 // columns and rows of K (per instance)
    const int *krp, *kci;     // K~  (m x n) CSR, shared
    const T *kv;
    const int *trp, *tci;     // K~' (n x m) CSR, shared
    const T *tv;
    int grid;                 // workgroups of the update / check / apply walks (the same walk in each)
    int grid_m;               // workgroups of the dual kernel
    const double *Nq, *Nc;    // [Bp] |q|, |c| of each instance's unscaled data
    Ctl *ctl;                 // [Bp]
    int *gate;                // 1 while some instance is in a check this slot
};

template <typename T> hipError_t launch_shared_slot(const SDev<T> &S, hipStream_t s);
// the check kernels alone (ungated: start, resume and final checks)
template <typename T> hipError_t launch_shared_check(const SDev<T> &S, int gated, hipStream_t s);
template <typename T> hipError_t launch_shared_apply(const SDev<T> &S, hipStream_t s);
// out = K~ in (which = 0) or K~' in (which = 1) for every instance, interleaved
template <typename T> hipError_t launch_shared_product(const SDev<T> &S, int which, const T *in, T *out,
                                                       hipStream_t s);
// instance b of an interleaved vector of `rows` rows to / from a plain FP64 vector
template <typename T> hipError_t launch_shared_extract(const T *src, int lgB, int b, double *dst, int rows,
                                                       hipStream_t s);
template <typename T> hipError_t launch_shared_insert(const double *src, int lgB, int b, T *dst, int rows,
                                                      hipStream_t s);
hipError_t launch_shared_set_final(Ctl *ctl, int Bp, int status, hipStream_t s);

template <typename T> hipError_t launch_batch_product(const BDev<T> &b, int which, hipStream_t s);
template <typename T> hipError_t launch_batch_product_plain(const BDev<T> &b, int which, const T *in, T *out,
                                                            hipStream_t s);
template <typename T> hipError_t launch_batch_dual(const BDev<T> &b, hipStream_t s);
template <typename T> hipError_t launch_batch_step_decide(const BDev<T> &b, hipStream_t s);
template <typename T> hipError_t launch_batch_update(const BDev<T> &b, hipStream_t s);
// gated = 1 inside the solve loop: the check kernels return at once unless
// this slot's step decisions raised the gate
template <typename T> hipError_t launch_batch_check(const BDev<T> &b, int gated, hipStream_t s);
template <typename T> hipError_t launch_batch_apply(const BDev<T> &b, hipStream_t s);
template <typename T> hipError_t launch_batch_start(const BDev<T> &b, hipStream_t s);
hipError_t launch_batch_set_final(Ctl *ctl, int B, int status, hipStream_t s);
hipError_t launch_seg_sumsq(const double *a, const int64_t *off, int B, double *out, hipStream_t s);
hipError_t launch_seg_absmax(const double *a, const int64_t *off, int B, double *out, hipStream_t s);

// launchers (kernels.hip); each returns the hipError_t of the launch
// per-device address of the fixed scratch array of lp_spmv_noalloc (noalloc.hip)
hipError_t noalloc_scratch(void **ptr);
template <typename T>
hipError_t launch_confirm(const Dev<T> &d, const Geo &g, const Conf64 &cf, int cur, double Nq, double Nc,
                          hipStream_t s);
// the same re-check with the FP64 products gathering from gx, gxa (current
// and averaged x) and gy, gya, which cf's column indices address: an LP's own
// vectors, or a whole batch's when cf holds one instance's rows of the
// batch's matrices (the products are written to cf's buffers by local row)
template <typename T>
hipError_t launch_confirm_gather(const Dev<T> &d, const Geo &g, const Conf64 &cf, int cur, const T *gx,
                                 const T *gxa, const T *gy, const T *gya, double Nq, double Nc, hipStream_t s);
// Bytes of LDS the staged one-workgroup loop needs: K and K' (values,
// columns, row pointers) and the two gathered vectors (the primal trial and
// the dual trial), values first so they stay 8-byte aligned.
template <typename T>
__host__ __device__ inline size_t small_stage_bytes(int m, int n, int nnz_k, int nnz_t)
{
    return sizeof(T) * ((size_t)nnz_k + nnz_t + n + m) + sizeof(int) * ((size_t)m + 1 + nnz_k + n + 1 + nnz_t);
}

// attempt slots of a small LP in one workgroup (one column slice per product,
// no long rows); K and K' (nnz_k, nnz_t entries) and the gathered vectors are
// staged in LDS when they fit in kSmallStageMax bytes
template <typename T> hipError_t launch_small_loop(const Dev<T> &d, int nnz_k, int nnz_t, int max_slots, double Nq,
                                                   double Nc, hipStream_t s);
// the register form of that loop for count LPs at once, workgroup b on LP b
// (devs[b]: its view; nq, nc: its norms): R = 1 when every LP has at most
// kSmallReg rows and columns, 2 for at most twice that; stage_bytes the
// largest small_stage_bytes of them; max_slots the slots per launch (its
// step factors are tabulated in the LDS after the stage)
template <typename T>
hipError_t launch_small_loop_batch(const Dev<T> *devs, const double *nq, const double *nc, int count, int R,
                                   size_t stage_bytes, int max_slots, hipStream_t s);
template <typename T>
hipError_t launch_gather_probe(const int *idx, const T *x, int64_t per_slice, int S, int64_t slice_len, T *out,
                               int grid, hipStream_t s);
template <typename T> hipError_t launch_partial_K(const Dev<T> &d, hipStream_t s);
template <typename T> hipError_t launch_partial_KT(const Dev<T> &d, hipStream_t s);
template <typename T> hipError_t launch_dual(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_step_decide(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_update(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_check_reduce(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_check_decide(const Dev<T> &d, const Geo &g, double Nq, double Nc, hipStream_t s);
template <typename T> hipError_t launch_check_apply(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_spmv(const Sliced<T> &P, const T *in, T *out, hipStream_t s);
template <typename T> hipError_t launch_gather_values(const double *src_vals, const int *src_pos, T *dst, int64_t len,
                                                      hipStream_t s);
template <typename T> hipError_t launch_start(const Dev<T> &d, const double *xs, const double *ys, int cur, hipStream_t s);
template <typename T> hipError_t launch_result(const Dev<T> &d, double *x, double *y, double *lam, hipStream_t s);
template <typename T> hipError_t launch_to_double(const T *in, double *out, int64_t len, hipStream_t s);
template <typename T> hipError_t launch_from_double(const double *in, T *out, int64_t len, hipStream_t s);

// one-time scaling helpers (FP64)
hipError_t launch_row_absmax(const int *rp, const double *v, int nrows, double *out, hipStream_t s);
hipError_t launch_row_abspow_sum(const int *rp, const double *v, int nrows, double p, double *out, hipStream_t s);
hipError_t launch_finish_factor(double *f, int len, hipStream_t s);
hipError_t launch_rescale_rows(const int *rp, const int *ci, double *v, int nrows, const double *rowf,
                               const double *colf, hipStream_t s);
hipError_t launch_mul_inplace(double *a, const double *f, int len, hipStream_t s);
hipError_t launch_fill(double *a, double v, int len, hipStream_t s);
hipError_t launch_scale_vectors(const double *c, const double *l, const double *u, const double *q,
                                const double *Dc, const double *Dr, double *cs, double *ls, double *us,
                                double *qs, int n, int m, hipStream_t s);
// klong[nklong] / tlong[ntlong]: device lists of the rows of K / K' longer
// than kLongRow, scaled on grids of their own (NULL, 0: every row one wave)
hipError_t scale_csr_pair(const int *rp, const int *ci, double *kv, int m, const int *tp, const int *ti, double *tv,
                          int n, double *Dr, double *Dc, double *r, double *s, int ruiz_iters, double alpha,
                          hipStream_t st, const int *klong = nullptr, int nklong = 0, const int *tlong = nullptr,
                          int ntlong = 0);
// deterministic sum of squares / max |.| over a vector: partials then one workgroup
hipError_t launch_sumsq(const double *a, int64_t len, double *part, double *out, hipStream_t s);
hipError_t launch_absmax(const double *a, int64_t len, double *part, double *out, hipStream_t s);

}  // namespace pdlp
