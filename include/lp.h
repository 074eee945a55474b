/*
 * lp.h -- C ABI of the MI355X restarted-PDHG LP solver (libpdlp_amd.so).
 *
 * Problem (cuPDLP-C paper, Sec. 2, eq. (LP)):
 *     min c'x   s.t.  A x = b,  G x >= h,  l <= x <= u
 * passed stacked as K = [A; G] (m x n CSR, the m1 equality rows first) and
 * q = [b; h].  The dual is  max q'y + l'lam+ - u'lam-  s.t. c - K'y = lam,
 * y_{m1..m-1} >= 0, lam in Lambda; lam is never stored and is returned as
 * proj_Lambda(c - K'y) (the remark after the termination criteria).
 *
 * Method (Sec. 2, "Restarted PDHG" and "Restart criteria"): PDHG on the
 * saddle-point problem (eq. (saddle-point)) with the primal update
 * x+ = proj_X(x - (eta/omega)(c - K'y)) and the dual update
 * y+ = proj_Y(y + eta*omega*(q - K(2x+ - x))), averaging, and restarts chosen
 * by the KKT_omega error with the constants 0.2, 0.8 and 0.36.  The solve
 * stops when the three relative criteria of "Optimality termination criteria"
 * hold at tolerance tol for the current or the averaged iterate.
 *
 * Conventions shared by every call
 *   - Every call returns int: LP_OK (0) or a negative LP_ERR_* code.  The
 *     solve outcome is lp_info.status.
 *   - Indices are int32 and 0-based; values are IEEE binary64.  Absent bounds
 *     are -INFINITY in l and +INFINITY in u.
 *   - The arrays of lp_load, lp_set_start and lp_result are host pointers, or
 *     device pointers when lp_options.ptr_kind = LP_DEVICE (every other call
 *     takes host pointers).  Inputs are copied during the call; the library
 *     keeps no caller pointer.  Outputs go to caller-allocated buffers.
 *   - Device memory: by default the library allocates it at lp_load and
 *     releases it at lp_free.  With lp_options.workspace set, every byte comes
 *     from that caller-owned device buffer instead (lp_workspace_size tells
 *     how many bytes) and the library calls no device allocator.  All GPU work
 *     is ordered on lp_options.stream (a hipStream_t; NULL = a non-blocking
 *     stream the library creates) and every call returns after that work is
 *     done.
 *   - A handle is not thread-safe; separate handles are independent.
 */
#ifndef PDLP_AMD_LP_H
#define PDLP_AMD_LP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define LP_OK 0
#define LP_ERR_ARG (-1)        /* NULL where a pointer is required, bad option value */
#define LP_ERR_DIM (-2)        /* m1 > m, row_ptr not monotone / not ending at nnz, column out of range, duplicate (row, col) */
#define LP_ERR_NAN (-3)        /* NaN or +-inf in K, c or q; NaN in l or u */
#define LP_ERR_BOUNDS (-4)     /* l_j > u_j, l_j = +inf or u_j = -inf */
#define LP_ERR_TOO_LARGE (-5)  /* m, n or nnz >= 2^31 */
#define LP_ERR_STATE (-6)      /* lp_result before any lp_solve; state buffer of the wrong size */
#define LP_ERR_HIP (-7)        /* a HIP runtime call failed; lp_last_error() has the message */
#define LP_ERR_NOMEM (-8)      /* host or device allocation failed */

/* lp_options.ptr_kind */
#define LP_HOST 0              /* array arguments are host pointers */
#define LP_DEVICE 1            /* array arguments of lp_load, lp_set_start, lp_result are device pointers */

/* lp_options.precision */
#define LP_FP64 0              /* FP64 values, iterates and reductions */
#define LP_MIXED 1             /* FP32 matrix values and iterates; FP64 reductions, step size and primal weight */

/* lp_info.status */
#define LP_NOT_SOLVED 0
#define LP_OPTIMAL 1           /* relative KKT error <= tol */
#define LP_ITERATION_LIMIT 2
#define LP_TIME_LIMIT 3
#define LP_NUMERICAL 4         /* NaN in a step-size or KKT quantity */
#define LP_PRIMAL_INFEASIBLE 5 /* a dual ray certifies that no x meets the constraints (see lp_result) */
#define LP_DUAL_INFEASIBLE 6   /* a primal ray certifies that the dual has no feasible point: the LP is
                                  unbounded if it is feasible (see lp_result) */

typedef struct lp_problem lp_problem;   /* opaque; owned by the library */

/* K in CSR: row_ptr[m+1] (row_ptr[0] = 0, row_ptr[m] = nnz, non-decreasing),
 * col[nnz] in [0, n) with no duplicate inside a row (any order), val[nnz]. */
typedef struct {
    int64_t m, n, nnz;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;
} lp_csr;

typedef struct {
    int precision;          /* LP_FP64 or LP_MIXED */
    void *stream;           /* hipStream_t for all GPU work; NULL = a stream the library creates */
    int ruiz_iters;         /* Ruiz inf-norm equilibration rounds (10) */
    double pc_alpha;        /* Pock-Chambolle exponent (1); < 0 skips that round */
    int check_every;        /* accepted steps between termination/restart checks (64) */
    double kkt_omega_power; /* exponent of omega in KKT_omega (2, as printed) */
    int fixed_step;         /* 0: adaptive step size; 1: constant step fixed_eta, every step accepted */
    double fixed_eta;
    int use_graph;          /* 1: replay the iteration window as a captured hipGraph */
    int window;             /* attempt slots launched between host polls of the done flag (64) */
    int kernel_timing;      /* 1: bracket the two SpMV kernel pairs of every slot with hipEvents (see
                               lp_kernel_time; the window then runs as plain launches on runtimes whose
                               graph-recorded events carry no timestamps); 2: only in the first window of
                               each lp_solve, launched plainly, the other windows replaying the untimed
                               captured graph; 0: none */
    int slice_kib;          /* target KiB of a gathered vector per column slice of K and K' (2048 = half an XCD's L2) */
    int autotune;           /* 1: at lp_load, time the slice count from slice_kib, then halve it (else
                               double it, to at most 32) while that keeps helping, then smaller row blocks,
                               on the actual matrix, and keep the fastest, per product (0); a candidate
                               replaces the current choice only when at least 3% faster.  Ignored when a
                               workspace is given.  At lp_batch_load: the row-block shape
                               (lp_batch_layout_blocks) */
    int verbose;            /* 1: messages on stderr, and one trace line per window of the solve (k, attempts,
                               restarts, eta, omega, and rel_p, rel_d, rel_gap, KKT_omega of the last check) */
    int ptr_kind;           /* LP_HOST (default) or LP_DEVICE */
    void *workspace;        /* NULL, or device memory of workspace_bytes bytes, 256-byte aligned, owned by
                               the caller, untouched by it until lp_free */
    size_t workspace_bytes;
    double infeas_tol;      /* relative residual at which a ray certifies infeasibility (1e-8; 0 disables
                               the test).  At each check the differences of the current iterate from the
                               restart anchor are tested as Farkas rays on the unscaled problem: a dual ray
                               w (y_G part >= 0) with q'w + l'lam+ - u'lam- > 0, lam = proj_Lambda(-K'w),
                               and |(-K'w - lam, min(w_G,0))| <= infeas_tol times that objective proves
                               primal infeasibility; a primal ray d with c'd < 0 and
                               |(A d, max(-G d,0), bound-cone violation of d)| <= infeas_tol |c'd| proves
                               dual infeasibility.  The paper does not specify detection. */
    int presolve;           /* 1: reduce the LP on the host before loading it (0): fixed columns, empty
                               columns, empty rows, singleton rows (an equality fixes its variable, an
                               inequality tightens a bound), to a fixed point; a reduction that would prove
                               infeasibility or unboundedness is left to the solve.  lp_set_start and
                               lp_result keep the original index space (lp_result maps the point back, with
                               the duals of removed rows, and reports the termination quantities of the
                               original problem); the state, scaling, product and layout calls refer to the
                               reduced problem (lp_presolved_size).  A stand-in for the presolvers the
                               paper's experiments run first (Table 1).  Not with LP_DEVICE or a workspace
                               (LP_ERR_ARG). */
    int persistent;         /* small LPs: run the whole iteration loop in one workgroup (one kernel launch per
                               64 x window attempt slots, barriers in place of kernel boundaries) instead of
                               seven launches per slot.  Eligible: both products one column slice and no row
                               longer than 8192 entries.  -1 (default): when eligible and K, K' and the two
                               vectors the products gather fit in 150 KiB of LDS (about 5,600 nonzeros with
                               1,500 rows and columns in FP64), where it is faster than the launches; 1:
                               whenever eligible; 0: never.  Same method, same results up to the summation
                               order of the reductions.  lp_kernel_time reports zeros for such solves.
                               lp_batch_load: -1 or 1 run a batch as one workgroup per instance, each on its
                               own loop (one launch per 64 x window slots for the whole batch), when every
                               instance has 1 to 1024 rows and columns and its K, K' and vectors fit the
                               LDS (lp_batch_loop_form); 0: the batched kernel launches. */
    int split_sums;         /* how the products' partial passes add up blocks of short rows (at most 64
                               entries per row and column slice).  0: one row per thread, in index order;
                               1: split by entries, each thread adding the products of 8 consecutive
                               entries row by row and a row that crosses those chunks finished from the
                               chunks' open parts in a fixed order (a few long rows among short ones then
                               no longer hold up their wavefront); -1 (default): split in a product of at
                               least 1024 row blocks (about 2 million nonzeros; in smaller ones the
                               split's extra barriers cost more than they save), and with autotune the
                               other form is timed on each product's chosen layout and kept when at
                               least 3% faster (lp_layout_split).  Both forms are deterministic;
                               they differ only in the rounding order of the row sums.  lp_batch_load:
                               1 split, -1 or 0 by rows (the batched workloads' rows are short and even,
                               and splitting them measured no faster); shared-matrix batches: ignored. */
} lp_options;

typedef struct {
    int status;                             /* LP_OPTIMAL ... */
    double pobj, dobj;                      /* c'x and q'y + l'lam+ - u'lam- of the returned point */
    double rel_primal, rel_dual, rel_gap;   /* the three relative termination quantities */
    int64_t iterations;                     /* accepted PDHG steps */
    int64_t attempts;                       /* step attempts, rejected ones included */
    int64_t restarts;
    double omega, eta;                      /* final primal weight and next step size */
    double seconds;                         /* wall time of the last lp_solve (load excluded) */
} lp_info;

/* Fill *opt with the defaults listed above. */
void lp_default_options(lp_options *opt);

/* Bytes of device workspace lp_load needs for K under *opt (the layout,
 * vectors, scratch and the load-time copies used by the scaling).  Host-side
 * only: sorts and slices the pattern of K as lp_load does, no GPU work (with
 * ptr_kind = LP_DEVICE it copies K to the host first).  opt may be NULL
 * (defaults).  Errors: LP_ERR_ARG, _DIM, _TOO_LARGE. */
int lp_workspace_size(const lp_csr *K, const lp_options *opt, size_t *bytes);

/* Validate, build the CSR of K' (counting sort, so the K' product needs no
 * atomics), cut both products into column slices sized to stay resident in
 * one XCD's L2, copy to the GPU and apply the diagonal scaling there.  The scaling is
 * the diagonal preconditioning the paper's experiments apply before PDHG
 * (Sec. 3.1).  On success *P owns all device memory (or its part of the
 * caller's workspace); on error *P = NULL.  A workspace smaller than
 * lp_workspace_size reports LP_ERR_NOMEM; one not 256-byte aligned LP_ERR_ARG.
 * Errors: LP_ERR_ARG, _DIM, _NAN, _BOUNDS, _TOO_LARGE, _HIP, _NOMEM. */
int lp_load(lp_problem **P, const lp_csr *K, const double *c, const double *q,
            const double *l, const double *u, int64_t m1, const lp_options *opt);

/* Start point for the next lp_solve: x0[n], y0[m] in the original (unscaled)
 * space, either may be NULL (= x projected 0, y = 0).  Both are projected onto
 * X and Y.  Cancels any state set by lp_set_state. */
int lp_set_start(lp_problem *P, const double *x0, const double *y0);

/* Primal weight omega the next start uses instead of |c~|/|q~| (omega <= 0
 * restores that default).  For warm starts of a parametric family, where a
 * converged member's weight suits its neighbours.  Errors: LP_ERR_ARG for
 * NaN or infinity. */
int lp_set_start_weight(lp_problem *P, double omega);

/* Run restarted PDHG until the relative KKT error <= tol, max_iters accepted
 * steps in total, or time_limit_s seconds (<= 0: none).  Starts from the
 * start point, or resumes from a state given by lp_set_state.  A check runs
 * every check_every accepted steps and at max_iters.  Returns LP_OK even when
 * the limit is hit; see lp_info.status.  Errors: LP_ERR_ARG, LP_ERR_HIP. */
int lp_solve(lp_problem *P, double tol, int64_t max_iters, double time_limit_s);

/* Copy the returned point to buffers x[n], y[m], lambda[n] (each may be
 * NULL; device buffers when ptr_kind = LP_DEVICE), unscaled and in the
 * original order; lambda = proj_Lambda(c - K'y).  info may be NULL.
 * After LP_PRIMAL_INFEASIBLE or LP_DUAL_INFEASIBLE the point is the pair of
 * rays (x = d, y = w, lambda = proj_Lambda(-K'w); see infeas_tol), with
 * info->pobj = c'd and info->dobj = q'w + l'lam+ - u'lam-; the rel_* fields
 * are those of the current iterate.
 * Errors: LP_ERR_STATE before the first lp_solve. */
int lp_result(const lp_problem *P, double *x, double *y, double *lambda, lp_info *info);

/* Rows *m and columns *n of the problem on the GPU: the original ones, or
 * the reduced ones when lp_options.presolve removed some.  Either pointer may
 * be NULL.  Errors: LP_ERR_ARG. */
int lp_presolved_size(const lp_problem *P, int64_t *m, int64_t *n);

/* Solver state for checkpoint/resume and per-step comparison, as doubles in
 * the scaled space and the original order: 16 scalars
 * [eta, omega, W, KKT0, KKT_prev, k, t, attempts, restarts, status, eta_last, 0 ...]
 * then x[n] y[m] Kx[m] K'y[n] xbar[n] ybar[m] Kxbar[m] K'ybar[n] x_anchor[n]
 * y_anchor[m].  *len receives 16 + 5n + 5m.  buf may be NULL to query len. */
int lp_get_state(const lp_problem *P, double *buf, int64_t *len);
/* Restore such a state (len must match); the next lp_solve resumes from it. */
int lp_set_state(lp_problem *P, const double *buf, int64_t len);

/* Scaling factors: K~ = D_r^-1 K D_c^-1.  Dr[m], Dc[n]; either may be NULL. */
int lp_get_scaling(const lp_problem *P, double *Dr, double *Dc);

/* One product with the scaled matrix on the GPU: out = K~ in (transpose = 0,
 * in[n], out[m]) or out = K~' in (transpose = 1, in[m], out[n]); host
 * buffers, original order.  Runs the same SpMV kernels as the solve. */
int lp_spmv(lp_problem *P, int transpose, const double *in, double *out);

/* lp_spmv for callers that cannot allocate device memory or synchronise:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same product, same kernels and the same result bit for bit as
 * lp_spmv, but in[] and out[] are DEVICE pointers (double; in[n], out[m], or
 * in[m], out[n] with transpose = 1, original order), and the intermediates
 * (the per-slice partial vectors, the long-row chunk sums and, in LP_MIXED,
 * FP32 copies of in and out) live in a fixed 64 MiB device array that the
 * library holds on every GPU it runs on until the process ends.  It calls no
 * allocator and does not wait: the work is only enqueued on the handle's
 * stream (lp_options.stream), so the caller synchronises that stream before
 * reading out.  Nothing in the array needs to start at zero.  Every call on
 * one GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other threads, other handles) race and must be serialised by the
 * caller.  The handle's GPU must be the current device.
 * Errors: LP_ERR_ARG (NULL pointer, wrong current device), LP_ERR_NOMEM (the
 * product needs more than the 64 MiB array: S*rows*value size plus the
 * long-row sums plus, in LP_MIXED, 4(n+m) bytes, each rounded up to 256;
 * lp_last_error() states the size), LP_ERR_HIP (a launch failed or the array
 * is not available). */
int lp_spmv_noalloc(lp_problem *P, int transpose, const double *in, double *out);

/* Launch statistics of the two products of the last lp_solve when
 * kernel_timing was set: which = 0 (K x' partial pass + fused dual step) or
 * 1 (K' y' partial pass + fused averages and next primal step); *count
 * launch pairs with *total_ms summed hipEvent time (the first window's only
 * with kernel_timing = 2).  Zeros when timing was off. */
int lp_kernel_time(const lp_problem *P, int which, int64_t *count, double *total_ms);

/* Measurement helper (not a step of the method): the rate of the random
 * gathers that bound the sparse products, without their matrix.  idx
 * (device, int32, count entries, slice-major: count / slices per slice, each
 * in [0, slice_len)) indexes x (device; double for LP_FP64, float for
 * LP_MIXED; slices * slice_len entries, slice s at s * slice_len).
 * Workgroups are dealt to slices as in the products (slice s on the XCDs
 * congruent to s); each thread makes eight gathers per 2048-index chunk.
 * out (device, same type as x) receives 4096 * 256 sums at most.  Runs one
 * untimed pass, then reps passes on stream, and stores the mean pass time.
 * Errors: LP_ERR_ARG (NULL, non-positive sizes, count not divisible by
 * slices, more than 4096 slices), LP_ERR_HIP. */
int lp_gather_probe(const int32_t *idx, const void *x, int precision, int64_t count, int slices, int64_t slice_len,
                    void *out, int reps, void *stream, double *ms_per_pass);

/* Device bytes held by the handle. */
int lp_device_bytes(const lp_problem *P, int64_t *bytes);

/* Column slices chosen for K (over x) and K' (over y); either may be NULL. */
int lp_layout(const lp_problem *P, int *slices_K, int *slices_KT);

/* The full layout of one product (which = 0: K, 1: K'): column slices, the
 * most nonzeros and the most rows of one row block (a single longer row
 * forms a block of its own).  Any output may be NULL; LP_ERR_ARG for a bad
 * `which`. */
int lp_layout_blocks(const lp_problem *P, int which, int *slices, int *nnz_per_block, int *rows_per_block);
/* How the partial passes of K (which = 0) or K' (which = 1) add up their
 * blocks of short rows: *split = 1 split by entries, 0 one row per thread
 * (lp_options.split_sums).  LP_ERR_ARG on a NULL pointer or another which. */
int lp_layout_split(const lp_problem *P, int which, int *split);

void lp_free(lp_problem *P);

/* ------------------------------------------------------------------------
 * Batched solves: many independent LPs of the form above advanced together
 * by one set of kernels per iteration (one captured hipGraph window), or,
 * when every instance is small, by one workgroup per instance running that
 * instance's whole loop (lp_options.persistent, lp_batch_loop_form); each
 * instance has its own step size, primal weight, restarts and termination.
 * The method per instance is exactly the one lp_solve runs, including mixed
 * precision's FP64 re-check of a termination test passed on FP32 products.
 * ------------------------------------------------------------------------ */
typedef struct lp_batch lp_batch;   /* opaque; owned by the library */

/* count instances: K[i], c[i], q[i], l[i], u[i], m1[i] as in lp_load (host
 * pointers, copied).  Options apply to every instance.  Same error codes as
 * lp_load (the first failing instance decides).  A batch takes host pointers
 * and allocates its own device memory: ptr_kind = LP_DEVICE, a workspace or
 * presolve is LP_ERR_ARG.  Rows longer than one row block (2048 entries) are
 * summed by a whole workgroup, without the chunking of lp_load. */
int lp_batch_load(lp_batch **B, int32_t count, const lp_csr *K, const double *const *c, const double *const *q,
                  const double *const *l, const double *const *u, const int64_t *m1, const lp_options *opt);
/* Solve every instance (cold start, or resume when lp_batch_set_state was
 * called for every instance since the last solve) until each is optimal at
 * tol, reaches max_iters accepted steps, or the time limit ends the call. */
int lp_batch_solve(lp_batch *B, double tol, int64_t max_iters, double time_limit_s);
/* Result of instance i as lp_result; info->seconds is the time into the last
 * lp_batch_solve at which the host saw instance i finish. */
int lp_batch_result(const lp_batch *B, int32_t i, double *x, double *y, double *lambda, lp_info *info);
/* State of instance i in the layout of lp_get_state. */
int lp_batch_get_state(const lp_batch *B, int32_t i, double *buf, int64_t *len);
int lp_batch_set_state(lp_batch *B, int32_t i, const double *buf, int64_t len);
int lp_batch_device_bytes(const lp_batch *B, int64_t *bytes);
/* Row-block shape of the batch's products (which = 0: K, 1: K'): the most
 * nonzeros and rows of one block.  With lp_options.autotune set, lp_batch_load
 * times four shapes per product (2048 or 1024 nonzeros, 1024 or 256 rows) on
 * the block-diagonal matrix and keeps the fastest; otherwise 2048 and 1024.
 * Errors: LP_ERR_ARG for a bad `which`. */
int lp_batch_layout_blocks(const lp_batch *B, int which, int *nnz_per_block, int *rows_per_block);
/* How the batch iterates: *form = 0 for the batched kernel launches (one set
 * per attempt slot, captured as a hipGraph window), 1 for one workgroup per
 * instance running that instance's whole loop (lp_options.persistent, small
 * instances only). */
int lp_batch_loop_form(const lp_batch *B, int *form);
void lp_batch_free(lp_batch *B);
const char *lp_batch_last_error(const lp_batch *B);
const char *lp_strerror(int code);
/* Message of the last LP_ERR_HIP on this handle ("" when none). */
const char *lp_last_error(const lp_problem *P);

/* ------------------------------------------------------------------------
 * Batched solves of one family: count <= 256 LPs that share the matrix K
 * (pattern and values) and the number of equality rows m1, each with its own
 * c, q, l, u (a parametric family, e.g. the training set of the warm-start
 * network).  The method per instance is exactly the one lp_solve runs; the
 * scaling depends on K alone, so every instance gets the same factors.  The
 * iterates of all instances are interleaved on the device, so each sparse
 * product of an iteration (K x and K'y, Sec. 2 "Restarted PDHG") reads K
 * once for all instances (an SpMM) instead of once per instance.  Host
 * pointers only; the handle allocates its own device memory (ptr_kind =
 * LP_DEVICE, a workspace or presolve is LP_ERR_ARG).
 * ------------------------------------------------------------------------ */
typedef struct lp_shared lp_shared;   /* opaque; owned by the library */

/* K as in lp_load (validated once); c[i], q[i], l[i], u[i] of instance i,
 * validated as in lp_load (l[i] or u[i] may point to the same array for every
 * instance).  Errors: LP_ERR_ARG (count outside 1..256, NULL, unsupported
 * options), the lp_load codes of K and of the first failing instance,
 * LP_ERR_TOO_LARGE when (n + 1) or (m + 1) times count rounded up to a power
 * of two reaches 2^30. */
int lp_shared_load(lp_shared **S, int32_t count, const lp_csr *K, const double *const *c, const double *const *q,
                   const double *const *l, const double *const *u, int64_t m1, const lp_options *opt);
/* Start of instance i for the next lp_shared_solve, as lp_set_start (x0[n],
 * y0[m] unscaled, either NULL = projected 0), with primal weight omega
 * (<= 0: |c~|/|q~|), as lp_set_start_weight.  Cancels states set by
 * lp_shared_set_state.  Errors: LP_ERR_ARG for a bad i or a NaN/inf omega. */
int lp_shared_set_start(lp_shared *S, int32_t i, const double *x0, const double *y0, double omega);
/* Solve every instance from its start (or resume, when lp_shared_set_state
 * was called for every instance since the last solve) until each is optimal
 * at tol, reaches max_iters accepted steps, or the time limit ends the call.
 * In LP_MIXED an instance whose termination test passes on FP32 products is
 * confirmed with FP64 products before it ends OPTIMAL, as in lp_solve. */
int lp_shared_solve(lp_shared *S, double tol, int64_t max_iters, double time_limit_s);
/* Result of instance i as lp_result; info->seconds is the time into the last
 * lp_shared_solve at which the host saw instance i finish.  LP_ERR_STATE
 * before the first solve. */
int lp_shared_result(const lp_shared *S, int32_t i, double *x, double *y, double *lambda, lp_info *info);
/* State of instance i in the layout of lp_get_state; set_state restores it. */
int lp_shared_get_state(const lp_shared *S, int32_t i, double *buf, int64_t *len);
int lp_shared_set_state(lp_shared *S, int32_t i, const double *buf, int64_t len);
int lp_shared_device_bytes(const lp_shared *S, int64_t *bytes);
void lp_shared_free(lp_shared *S);
const char *lp_shared_last_error(const lp_shared *S);

/* ------------------------------------------------------------------------
 * Learned warm start for a parametric LP family (fixed K; b, h, c vary).
 * A network maps a standardized sketch of an instance's perturbation to a
 * primal-dual start point for lp_set_start: `layers` ReLU layers of width
 * `hidden`, a linear layer to `rank` coefficients, and a linear layer of
 * width out_dim (= n + m; its bias starts at the base solution).  Shapes are
 * row-major with the batch first.  Data arguments of the calls below are
 * DEVICE pointers (float32) supplied by the caller; parameters move through
 * host buffers.  The cold-start solve stays the fallback: a warm solve that
 * fails is redone cold by the caller.
 * ------------------------------------------------------------------------ */
#define LPW_BF16 0   /* bf16 weights and activations on MFMA, FP32 accumulation */
#define LPW_FP32 1   /* FP32 throughout (checking mode) */

typedef struct lpw_net lpw_net;
typedef struct {
    int in_dim;      /* sketch features (256) */
    int hidden;      /* width of the ReLU layers (1024) */
    int layers;      /* ReLU layers (3) */
    int rank;        /* coefficients of the low-rank output (64) */
    int out_dim;     /* n + m of the family */
    int max_batch;   /* rows per call (256) */
    int precision;   /* LPW_BF16 or LPW_FP32 */
    void *stream;    /* hipStream_t, NULL = null stream */
} lpw_config;

void lpw_default_config(lpw_config *cfg);
int lpw_create(lpw_net **net, const lpw_config *cfg);
/* Parameters as one flat float vector, layer by layer: W_l [in x out] then
 * b_l [out]. */
int64_t lpw_param_count(const lpw_net *net);
int lpw_set_params(lpw_net *net, const float *host_params);   /* also resets Adam */
int lpw_get_params(const lpw_net *net, float *host_params);
/* Input standardization: features become (x - mu) / sigma (sigma > 0). */
int lpw_set_norm(lpw_net *net, const float *host_mu, const float *host_sigma);
/* Z[B x out_dim] = net(X[B x in_dim]) on the device, B <= max_batch. */
int lpw_forward(lpw_net *net, const float *X, int B, float *Z);
/* Mean squared error against Zstar[B x out_dim] and its gradient (kept on
 * the device; lpw_get_grads copies it out).  *loss may be NULL. */
int lpw_loss_grad(lpw_net *net, const float *X, const float *Zstar, int B, double *loss);
int lpw_get_grads(const lpw_net *net, float *host_grads);
/* One Adam update with the stored gradient. */
int lpw_adam_step(lpw_net *net, float lr, float beta1, float beta2, float eps);
/* lpw_loss_grad then lpw_adam_step(lr, 0.9, 0.999, 1e-8). */
int lpw_train_step(lpw_net *net, const float *X, const float *Zstar, int B, float lr, double *loss);
/* The GEMM kernel alone: C[M x N] = op(A) op(B), op = transpose when
 * trans_* != 0 (A stored [M x K] or [K x M] with leading dimension lda, B
 * stored [K x N] or [N x K]); A, B are bfloat16 bits (uint16) in LPW_BF16
 * mode and float in LPW_FP32 mode; C is float.  Device pointers. */
int lpw_gemm(int precision, int trans_a, int trans_b, int M, int N, int K, const void *A, int lda, const void *B,
             int ldb, float *C, int ldc, void *stream);
/* out[B x rows] = D[B x cols] S' for a sparse S (CSR rows x cols, float),
 * the sketch of each instance's perturbation vector.  Device pointers. */
int lpw_sketch(const int *row_ptr, const int *col, const float *val, int rows, const float *D, int cols, int B,
               float *out, void *stream);
void lpw_free(lpw_net *net);
const char *lpw_last_error(const lpw_net *net);

#ifdef __cplusplus
}
#endif

#endif
