// Internal types shared by the HIP kernels and the host side of libpdlp_amd.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lp.h"

namespace pdlp {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kMaxSeg = 32;      // row segments per CSR
constexpr int kMaxGrid = 2048;   // workgroups of a solver kernel = partial-sum slots
constexpr int kCheckSums = 18;   // 9 sums for the current and 9 for the averaged iterate

// Rows of one CSR (after reordering) fall into segments of consecutive rows
// that share a lane count: 1..64 lanes of a wave per row, or 256 = a whole
// workgroup per row.  Virtual block v of the grid-stride loop maps to
// segment s with vb_begin[s] <= v < vb_begin[s+1].
struct Segments {
    int nseg;
    int row_begin[kMaxSeg];
    int row_end[kMaxSeg];
    int lanes[kMaxSeg];
    int vb_begin[kMaxSeg + 1];
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
    int pad;
};

template <typename T>
struct Dev {
    int m, n, m1;
    const int *rp, *ci;        // K   (rows permuted by bin, columns renumbered)
    const T *kv;
    const int *tp, *ti;        // K'  (CSR of the transpose, same renumbering)
    const T *tv;
    const T *cs, *ls, *us;     // scaled c, l, u   [n]
    const T *qs;               // scaled q         [m]
    const double *Dr, *Dc;     // scaling factors
    T *xb[2], *yb[2], *Kxb[2], *KTyb[2];   // current / trial buffers
    T *xa, *ya, *Kxa, *KTya;   // step-weighted averages
    T *x0, *y0;                // restart anchor
    T *xo, *yo, *KTyo;         // returned point
    double *part_primal;       // [kMaxGrid]      |x' - x|^2 partials
    double *part_dual;         // [kMaxGrid * 2]  |y' - y|^2, (y'-y).(Kx'-Kx)
    double *part_check;        // [kMaxGrid * kCheckSums]
    Ctl *ctl;
};

struct Geo {
    int grid;                  // workgroups of every solver kernel
    int vb_K, vb_KT, vb_n, vb_m;
    Segments segK, segKT;
};

// launchers (kernels.hip); each returns the hipError_t of the launch
template <typename T> hipError_t launch_dual(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_step_decide(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_update(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_check_reduce(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_check_decide(const Dev<T> &d, const Geo &g, double Nq, double Nc, hipStream_t s);
template <typename T> hipError_t launch_check_apply(const Dev<T> &d, const Geo &g, hipStream_t s);
template <typename T> hipError_t launch_spmv(const int *rp, const int *ci, const T *v, const T *in, T *out,
                                             const Segments &seg, int total_vb, int grid, hipStream_t s);
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
// deterministic sum of squares / max |.| over a vector: partials then one workgroup
hipError_t launch_sumsq(const double *a, int64_t len, double *part, double *out, hipStream_t s);
hipError_t launch_absmax(const double *a, int64_t len, double *part, double *out, hipStream_t s);

}  // namespace pdlp
