/*
 * FP64 CPU oracle for restarted PDHG on LP -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load this library.  The product path (the HIP library) never links,
 * loads or calls it, and the two share no source.
 *
 * What it computes (cuPDLP-C paper, Sec. 2 "Overview of the Method"):
 *   primal  min c'x  s.t. Ax=b, Gx>=h, l<=x<=u      (eq. (LP), left)
 *   dual    max q'y + l'lam+ - u'lam-  s.t. c-K'y=lam, y_G>=0, lam in Lambda
 *   with K=[A;G], q=[b;h]; Lambda_j = {0} free, R- upper-only, R+ lower-only,
 *   R both bounds finite (the Lambda case list).
 *   Termination: the three relative criteria (primal feasibility, dual
 *   feasibility, duality gap) with lam = proj_Lambda(c - K'y).
 *   Iteration: the PDHG primal step x+ = proj_X(x - (eta/omega)(c - K'y)) and
 *   dual step y+ = proj_Y(y + eta*omega*(q - K(2x+ - x))) of the saddle-point
 *   problem (eq. (saddle-point)), with averaging and the KKT-based restart
 *   (KKT_omega, the candidate rule and restart conditions 1-3).
 *
 * Where the paper is silent the oracle takes these readings (all of them are
 * also what the GPU library implements):
 *   - scaling: R rounds of Ruiz (sqrt of row / column inf-norms, both from the
 *     same matrix), then one Pock-Chambolle round with exponent alpha;
 *   - step size: PDLP's adaptive rule; the counter in its exponents is the
 *     number of accepted steps before this one plus one;
 *   - primal weight: ||c~||/||q~|| (1 if either is <= 1e-10), updated only at
 *     restarts by omega <- exp(0.5 log(dy/dx) + 0.5 log omega);
 *   - averages weighted by the accepted step sizes, reset at restarts;
 *   - termination and restart are checked every `check_every` accepted steps;
 *     termination on the unscaled problem, restart KKT on the scaled one,
 *     with omega raised to `kkt_p` (2 as printed);
 *   - projections propagate NaN;
 *   - infeasibility (the paper is silent): at each check the differences of
 *     the current iterate from the restart anchor are tested as Farkas rays
 *     on the unscaled problem (see ray_status).
 *
 * Plain loops, sequential left-to-right sums, no blocking or reordering.
 * Build with -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_DIM (-2)
#define ORC_ERR_NAN (-3)
#define ORC_ERR_BOUNDS (-4)
#define ORC_ERR_TOO_LARGE (-5)
#define ORC_ERR_STATE (-6)
#define ORC_ERR_NOMEM (-8)

#define ORC_NOT_SOLVED 0
#define ORC_OPTIMAL 1
#define ORC_ITERATION_LIMIT 2
#define ORC_TIME_LIMIT 3
#define ORC_NUMERICAL 4
#define ORC_PRIMAL_INFEASIBLE 5
#define ORC_DUAL_INFEASIBLE 6

#define ORC_NSCALARS 16

/* ORC_MUT (default 0) plants one known mistake, for the tests that check
 * the pins catch it.  Never defined in the oracle the other tests use. */
#ifndef ORC_MUT
#define ORC_MUT 0
#endif

typedef struct {
    int ruiz_iters;     /* Ruiz rounds (10) */
    double pc_alpha;    /* Pock-Chambolle exponent (1); < 0 disables the round */
    int check_every;    /* accepted steps between checks (64) */
    double kkt_p;       /* exponent of omega in KKT_omega (2) */
    int fixed_step;     /* 1: constant eta = fixed_eta, every step accepted */
    double fixed_eta;
    double infeas_tol;  /* ray certificates accepted at this relative residual (1e-8); 0: no detection */
} orc_opts;

typedef struct {
    int64_t m, n, m1, nnz;
    int32_t *rp, *ci;
    double *v;          /* original K values */
    double *kv;         /* scaled K values (same pattern) */
    double *c, *q, *l, *u;
    double *Dr, *Dc;
    double *cs, *qs, *ls, *us;
    double Nq, Nc;
    orc_opts o;
    /* iterate state, scaled space */
    double *x, *y, *Kx, *KTy;
    double *xa, *ya, *Kxa, *KTya;   /* averages */
    double *x0, *y0;                /* restart anchor */
    double *xt, *yt, *Kxt, *KTyt;   /* trial */
    double eta_hat, omega, W, KKT0, KKT_prev, eta_last;
    int64_t k, t, attempts, restarts;
    int status;
    int state_ready;                /* set by orc_set_state: next solve resumes */
    /* warm start (unscaled), optional */
    double *xs, *ys;
    int has_xs, has_ys;
    double omega_start;             /* > 0: primal weight of the next start */
    /* output (scaled) */
    double *xo, *yo, *KTyo;
    double out_rel_p, out_rel_d, out_rel_g, out_pobj, out_dobj;
    int has_output;
    double seconds;
} orc_t;

/* ------------------------------------------------------------------------ */
/* small pieces                                                              */
/* ------------------------------------------------------------------------ */

static double clampx(double v, double lo, double hi)
{
    /* proj onto [lo, hi]; NaN passes through */
    return v < lo ? lo : (v > hi ? hi : v);
}

/* proj onto Lambda_j given which bounds are finite (the Lambda case list) */
static double proj_lambda(double g, int lfin, int ufin)
{
    if (!lfin && !ufin) return 0.0;            /* {0} */
    if (!lfin && ufin) return g < 0.0 ? g : 0.0;   /* R- */
    if (lfin && !ufin) return ORC_MUT == 3 ? g : (g > 0.0 ? g : 0.0);   /* R+ */
    return g;                                  /* R */
}

static void spmv_K(const orc_t *P, const double *x, double *out)
{
    for (int64_t i = 0; i < P->m; ++i) {
        double s = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) s += P->kv[p] * x[P->ci[p]];
        out[i] = s;
    }
}

static void spmv_KT(const orc_t *P, const double *y, double *out)
{
    for (int64_t j = 0; j < P->n; ++j) out[j] = 0.0;
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) out[P->ci[p]] += P->kv[p] * y[i];
}

/* products with the unscaled K (same pattern, original values) */
static void spmv_K_unscaled(const orc_t *P, const double *x, double *out)
{
    for (int64_t i = 0; i < P->m; ++i) {
        double s = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) s += P->v[p] * x[P->ci[p]];
        out[i] = s;
    }
}

static void spmv_KT_unscaled(const orc_t *P, const double *y, double *out)
{
    for (int64_t j = 0; j < P->n; ++j) out[j] = 0.0;
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) out[P->ci[p]] += P->v[p] * y[i];
}

static double norm2(const double *a, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += a[i] * a[i];
    return sqrt(s);
}

double orc_step_next(double eta, double eta_bar, int64_t k_accepted)
{
    /* PDLP adaptive rule; kk counts steps from 1 */
    double kk = (double)(k_accepted + 1) + 1.0;
    double a = (1.0 - pow(kk, ORC_MUT == 5 ? -0.03 : -0.3)) * eta_bar;
    double b = (1.0 + pow(kk, -0.6)) * eta;
    return a < b ? a : b;
}

/* 0 = no restart, 1 = sufficient decay, 2 = necessary decay + no progress,
 * 3 = long inner loop (restart conditions 1-3) */
int orc_restart_decision(double kkt_c, double kkt0, double kkt_prev, int64_t t, int64_t k)
{
    if (kkt_c <= 0.2 * kkt0) return 1;
    if (kkt_c <= 0.8 * kkt0 && kkt_c > kkt_prev) return 2;
    if ((double)t >= 0.36 * (double)k) return 3;
    return 0;
}

double orc_omega_update(double omega, double dx, double dy)
{
    if (dx > 1e-10 && dy > 1e-10) return exp(0.5 * log(dy / dx) + 0.5 * log(omega));
    return omega;
}

/* ------------------------------------------------------------------------ */
/* load / validate / scale                                                   */
/* ------------------------------------------------------------------------ */

static void *xalloc(int64_t count, size_t size)
{
    if (count <= 0) count = 1;
    return calloc((size_t)count, size);
}

void orc_free(orc_t *P)
{
    if (!P) return;
    double **d[] = {&P->v, &P->kv, &P->c, &P->q, &P->l, &P->u, &P->Dr, &P->Dc, &P->cs, &P->qs,
                    &P->ls, &P->us, &P->x, &P->y, &P->Kx, &P->KTy, &P->xa, &P->ya, &P->Kxa,
                    &P->KTya, &P->x0, &P->y0, &P->xt, &P->yt, &P->Kxt, &P->KTyt, &P->xs, &P->ys,
                    &P->xo, &P->yo, &P->KTyo};
    for (size_t i = 0; i < sizeof(d) / sizeof(d[0]); ++i) free(*d[i]);
    free(P->rp);
    free(P->ci);
    free(P);
}

void orc_default_opts(orc_opts *o)
{
    o->ruiz_iters = 10;
    o->pc_alpha = 1.0;
    o->check_every = 64;
    o->kkt_p = 2.0;
    o->fixed_step = 0;
    o->fixed_eta = 0.0;
    o->infeas_tol = 1e-8;
}

static void scale_problem(orc_t *P)
{
    int64_t m = P->m, n = P->n;
    double *r = xalloc(m, sizeof(double)), *s = xalloc(n, sizeof(double));
    for (int64_t i = 0; i < m; ++i) P->Dr[i] = 1.0;
    for (int64_t j = 0; j < n; ++j) P->Dc[j] = 1.0;
    int rounds = P->o.ruiz_iters + (P->o.pc_alpha >= 0.0 ? 1 : 0);
    for (int it = 0; it < rounds; ++it) {
        int pc = it == P->o.ruiz_iters;
        for (int64_t i = 0; i < m; ++i) r[i] = 0.0;
        for (int64_t j = 0; j < n; ++j) s[j] = 0.0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) {
                double a = fabs(P->kv[p]);
                int64_t j = P->ci[p];
                if (!pc) {
                    if (a > r[i]) r[i] = a;
                    if (ORC_MUT == 6 ? r[i] > s[j] : a > s[j]) s[j] = ORC_MUT == 6 ? r[i] : a;
                } else {
                    r[i] += pow(a, 2.0 - P->o.pc_alpha);
                    s[j] += pow(a, P->o.pc_alpha);
                }
            }
        for (int64_t i = 0; i < m; ++i) r[i] = r[i] > 0.0 ? sqrt(r[i]) : 1.0;
        for (int64_t j = 0; j < n; ++j) s[j] = s[j] > 0.0 ? sqrt(s[j]) : 1.0;
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) P->kv[p] = P->kv[p] / (r[i] * s[P->ci[p]]);
        for (int64_t i = 0; i < m; ++i) P->Dr[i] *= r[i];
        for (int64_t j = 0; j < n; ++j) P->Dc[j] *= s[j];
    }
    free(r);
    free(s);
    for (int64_t j = 0; j < n; ++j) {
        P->cs[j] = P->c[j] / P->Dc[j];
        P->ls[j] = P->l[j] * P->Dc[j];   /* -inf stays -inf */
        P->us[j] = P->u[j] * P->Dc[j];
    }
    for (int64_t i = 0; i < m; ++i) P->qs[i] = P->q[i] / P->Dr[i];
}

int orc_load(orc_t **out, int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
             const double *v, const double *c, const double *q, const double *l, const double *u,
             int64_t m1, const orc_opts *opt)
{
    if (!out) return ORC_ERR_ARG;
    *out = NULL;
    if (m < 0 || n < 0 || nnz < 0 || m1 < 0 || m1 > m) return ORC_ERR_DIM;
    if (nnz >= ((int64_t)1 << 31) || m >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31)) return ORC_ERR_TOO_LARGE;
    if (!rp || (nnz > 0 && (!ci || !v)) || (n > 0 && (!c || !l || !u)) || (m > 0 && !q)) return ORC_ERR_ARG;
    if (rp[0] != 0 || rp[m] != nnz) return ORC_ERR_DIM;
    for (int64_t i = 0; i < m; ++i)
        if (rp[i + 1] < rp[i]) return ORC_ERR_DIM;
    int64_t *seen = xalloc(n, sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) seen[j] = -1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            int64_t j = ci[p];
            if (j < 0 || j >= n || seen[j] == i) { free(seen); return ORC_ERR_DIM; }
            seen[j] = i;
        }
    free(seen);
    for (int64_t p = 0; p < nnz; ++p)
        if (!isfinite(v[p])) return ORC_ERR_NAN;
    for (int64_t j = 0; j < n; ++j) {
        if (!isfinite(c[j]) || isnan(l[j]) || isnan(u[j])) return ORC_ERR_NAN;
        if (l[j] == INFINITY || u[j] == -INFINITY || l[j] > u[j]) return ORC_ERR_BOUNDS;
    }
    for (int64_t i = 0; i < m; ++i)
        if (!isfinite(q[i])) return ORC_ERR_NAN;

    orc_t *P = calloc(1, sizeof(orc_t));
    if (!P) return ORC_ERR_NOMEM;
    P->m = m; P->n = n; P->m1 = m1; P->nnz = nnz;
    if (opt) P->o = *opt; else orc_default_opts(&P->o);
    if (P->o.check_every <= 0) P->o.check_every = 64;
    P->rp = xalloc(m + 1, sizeof(int32_t));
    P->ci = xalloc(nnz, sizeof(int32_t));
    double **dn[] = {&P->c, &P->l, &P->u, &P->Dc, &P->cs, &P->ls, &P->us, &P->x, &P->KTy, &P->xa,
                     &P->KTya, &P->x0, &P->xt, &P->KTyt, &P->xs, &P->xo, &P->KTyo};
    double **dm[] = {&P->q, &P->Dr, &P->qs, &P->y, &P->Kx, &P->ya, &P->Kxa, &P->y0, &P->yt,
                     &P->Kxt, &P->ys, &P->yo};
    for (size_t i = 0; i < sizeof(dn) / sizeof(dn[0]); ++i) *dn[i] = xalloc(n, sizeof(double));
    for (size_t i = 0; i < sizeof(dm) / sizeof(dm[0]); ++i) *dm[i] = xalloc(m, sizeof(double));
    P->v = xalloc(nnz, sizeof(double));
    P->kv = xalloc(nnz, sizeof(double));
    memcpy(P->rp, rp, sizeof(int32_t) * (size_t)(m + 1));
    if (nnz) {
        memcpy(P->ci, ci, sizeof(int32_t) * (size_t)nnz);
        memcpy(P->v, v, sizeof(double) * (size_t)nnz);
        memcpy(P->kv, v, sizeof(double) * (size_t)nnz);
    }
    if (n) {
        memcpy(P->c, c, sizeof(double) * (size_t)n);
        memcpy(P->l, l, sizeof(double) * (size_t)n);
        memcpy(P->u, u, sizeof(double) * (size_t)n);
    }
    if (m) memcpy(P->q, q, sizeof(double) * (size_t)m);
    scale_problem(P);
    P->Nq = norm2(P->q, m);
    P->Nc = norm2(P->c, n);
    P->status = ORC_NOT_SOLVED;
    *out = P;
    return ORC_OK;
}

int orc_set_start_weight(orc_t *P, double omega)
{
    if (!P) return ORC_ERR_ARG;
    P->omega_start = omega > 0.0 ? omega : 0.0;
    P->state_ready = 0;
    return ORC_OK;
}

int orc_set_start(orc_t *P, const double *x, const double *y)
{
    if (!P) return ORC_ERR_ARG;
    P->has_xs = x != NULL;
    P->has_ys = y != NULL;
    if (x) memcpy(P->xs, x, sizeof(double) * (size_t)P->n);
    if (y) memcpy(P->ys, y, sizeof(double) * (size_t)P->m);
    P->state_ready = 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* KKT quantities of one point (scaled space in, both scalings out)          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rp2_u, rp2_s, qy, dy2;       /* rows: unscaled/scaled primal residual^2, q'y, |y-y0|^2 */
    double rd2_u, rd2_s, cx, bnd, dx2;  /* cols: dual residual^2, c'x, l'lam+ - u'lam-, |x-x0|^2 */
    double rel_p, rel_d, rel_g, rel, pobj, dobj, gap;
} orc_eval_t;

static void eval_point(const orc_t *P, const double *x, const double *y, const double *Kx,
                       const double *KTy, orc_eval_t *e)
{
    memset(e, 0, sizeof(*e));
    for (int64_t i = 0; i < P->m; ++i) {
        double r = Kx[i] - P->qs[i];
        if (i >= P->m1) r = (P->qs[i] - Kx[i]) > 0.0 ? (P->qs[i] - Kx[i]) : 0.0;
        double ru = r * P->Dr[i];
        e->rp2_u += ru * ru;
        e->rp2_s += r * r;
        e->qy += P->qs[i] * y[i];
        double d = y[i] - P->y0[i];
        e->dy2 += d * d;
    }
    for (int64_t j = 0; j < P->n; ++j) {
        int lf = isfinite(P->ls[j]), uf = isfinite(P->us[j]);
        double g = P->cs[j] - KTy[j];
        double lam = proj_lambda(g, lf, uf);
        double rd = g - lam;
        double rdu = rd * P->Dc[j];
        e->rd2_u += rdu * rdu;
        e->rd2_s += rd * rd;
        e->cx += P->cs[j] * x[j];
        double b = 0.0;
        if (lf && lam > 0.0) b += P->ls[j] * lam;
        if (uf && lam < 0.0) b += (ORC_MUT == 4 ? -1.0 : 1.0) * P->us[j] * lam;   /* -u * lam-  with lam- = -lam */
        e->bnd += b;
        double d = x[j] - P->x0[j];
        e->dx2 += d * d;
    }
    e->pobj = e->cx;
    e->dobj = e->qy + e->bnd;
    e->gap = e->dobj - e->pobj;
    e->rel_p = sqrt(e->rp2_u) / (1.0 + P->Nq);
    e->rel_d = sqrt(e->rd2_u) / (1.0 + P->Nc);
    e->rel_g = fabs(e->gap) / (1.0 + fabs(e->dobj) + fabs(e->pobj));
    e->rel = e->rel_p;
    if (e->rel_d > e->rel) e->rel = e->rel_d;
    if (e->rel_g > e->rel) e->rel = e->rel_g;
    if (isnan(e->rel_p) || isnan(e->rel_d) || isnan(e->rel_g)) e->rel = NAN;
}

static double kkt_omega(const orc_t *P, const orc_eval_t *e, double omega)
{
    double wp = pow(omega, ORC_MUT == 8 ? 1.0 : P->o.kkt_p);
    return sqrt(wp * e->rp2_s + e->rd2_s / wp + e->gap * e->gap);
}

/* ------------------------------------------------------------------------ */
/* the solver                                                                */
/* ------------------------------------------------------------------------ */

static void set_output(orc_t *P, const double *x, const double *y, const double *KTy, const orc_eval_t *e)
{
    memcpy(P->xo, x, sizeof(double) * (size_t)P->n);
    memcpy(P->yo, y, sizeof(double) * (size_t)P->m);
    memcpy(P->KTyo, KTy, sizeof(double) * (size_t)P->n);
    P->out_rel_p = e->rel_p; P->out_rel_d = e->rel_d; P->out_rel_g = e->rel_g;
    P->out_pobj = e->pobj; P->out_dobj = e->dobj;
    P->has_output = 1;
}

static void init_state(orc_t *P)
{
    int64_t m = P->m, n = P->n;
    for (int64_t j = 0; j < n; ++j) {
        double v0 = P->has_xs ? P->xs[j] * P->Dc[j] : 0.0;
        P->x[j] = clampx(v0, P->ls[j], P->us[j]);
    }
    for (int64_t i = 0; i < m; ++i) {
        double v0 = P->has_ys ? P->ys[i] * P->Dr[i] : 0.0;
        P->y[i] = (i >= P->m1 && v0 < 0.0) ? 0.0 : v0;
    }
    double nc = norm2(P->cs, n), nq = norm2(P->qs, m);
    P->omega = (nc > 1e-10 && nq > 1e-10) ? nc / nq : 1.0;
    if (P->omega_start > 0.0) P->omega = P->omega_start;
    double kmax = 0.0;
    for (int64_t p = 0; p < P->nnz; ++p)
        if (fabs(P->kv[p]) > kmax) kmax = fabs(P->kv[p]);
    P->eta_hat = kmax > 0.0 ? 1.0 / kmax : 1.0;
    if (P->o.fixed_step) P->eta_hat = P->o.fixed_eta;
    P->k = P->t = P->attempts = P->restarts = 0;
    P->W = 0.0;
    P->eta_last = 0.0;
    spmv_K(P, P->x, P->Kx);
    spmv_KT(P, P->y, P->KTy);
    memcpy(P->x0, P->x, sizeof(double) * (size_t)n);
    memcpy(P->y0, P->y, sizeof(double) * (size_t)m);
    memcpy(P->xa, P->x, sizeof(double) * (size_t)n);
    memcpy(P->ya, P->y, sizeof(double) * (size_t)m);
    memcpy(P->Kxa, P->Kx, sizeof(double) * (size_t)m);
    memcpy(P->KTya, P->KTy, sizeof(double) * (size_t)n);
    orc_eval_t e;
    eval_point(P, P->x, P->y, P->Kx, P->KTy, &e);
    P->KKT0 = kkt_omega(P, &e, P->omega);
    P->KKT_prev = INFINITY;
    P->status = ORC_NOT_SOLVED;
    P->has_output = 0;
}

/* One accepted PDHG step (any number of rejected attempts before it).
 * Returns 0, or -1 when the step-size quantities became NaN. */
static int pdhg_step(orc_t *P)
{
    int64_t m = P->m, n = P->n;
    double eta = P->eta_hat, omega = P->omega;
    for (;;) {
        double tau = eta / omega, sigma = eta * omega;
        for (int64_t j = 0; j < n; ++j)
            P->xt[j] = clampx(P->x[j] - tau * (P->cs[j] - (ORC_MUT == 1 ? -1.0 : 1.0) * P->KTy[j]), P->ls[j], P->us[j]);
        spmv_K(P, P->xt, P->Kxt);
        for (int64_t i = 0; i < m; ++i) {
            double v = ORC_MUT == 2 ? P->y[i] + sigma * (P->qs[i] - P->Kxt[i])
                                    : P->y[i] + sigma * (P->qs[i] - 2.0 * P->Kxt[i] + P->Kx[i]);
            if (i >= P->m1 && v < 0.0) v = 0.0;
            P->yt[i] = v;
        }
        P->attempts += 1;
        if (P->o.fixed_step) {
            P->eta_hat = eta;
            break;
        }
        double dx2 = 0.0, dy2 = 0.0, inter = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double d = P->xt[j] - P->x[j];
            dx2 += d * d;
        }
        for (int64_t i = 0; i < m; ++i) {
            double d = P->yt[i] - P->y[i];
            dy2 += d * d;
            inter += d * (P->Kxt[i] - P->Kx[i]);
        }
        double N = omega * dx2 + dy2 / omega;
        double D = 2.0 * fabs(inter);
        if (isnan(N) || isnan(D)) return -1;
        double eta_bar = D > 0.0 ? N / D : INFINITY;
        double eta_new = orc_step_next(eta, eta_bar, P->k);
        if (eta <= eta_bar) {
            P->eta_hat = eta_new;
            break;
        }
        eta = eta_new;
    }
    spmv_KT(P, P->yt, P->KTyt);
    P->eta_last = eta;
    P->W += eta;
    double w = ORC_MUT == 7 ? 1.0 / (double)(P->t + 1) : eta / P->W;
    for (int64_t j = 0; j < n; ++j) {
        P->xa[j] += w * (P->xt[j] - P->xa[j]);
        P->KTya[j] += w * (P->KTyt[j] - P->KTya[j]);
    }
    for (int64_t i = 0; i < m; ++i) {
        P->ya[i] += w * (P->yt[i] - P->ya[i]);
        P->Kxa[i] += w * (P->Kxt[i] - P->Kxa[i]);
    }
    double *tmp;
    tmp = P->x; P->x = P->xt; P->xt = tmp;
    tmp = P->y; P->y = P->yt; P->yt = tmp;
    tmp = P->Kx; P->Kx = P->Kxt; P->Kxt = tmp;
    tmp = P->KTy; P->KTy = P->KTyt; P->KTyt = tmp;
    P->k += 1;
    P->t += 1;
    return 0;
}

/* Infeasibility certificates (Farkas' lemma for the LP pair), on the
 * unscaled problem.  Candidate rays are the differences of the current
 * iterate from the restart anchor: when the LP has no primal-dual solution
 * the iterates drift along a ray and these differences grow with it.
 *   Dual ray w = (y - y0)/Dr proves the primal infeasible when
 *     dobj = q'w + sum_j (l_j lam_j+ - u_j lam_j-) > 0, with lam = proj_Lambda(-K'w),
 *     and ||(-K'w - lam, min(w_G, 0))||_2 <= eps * dobj.
 *   Primal ray d = (x - x0)/Dc proves the dual infeasible (the primal
 *     unbounded, if feasible) when c'd < 0 and
 *     ||(A d, max(-G d, 0), v)||_2 <= eps * |c'd|, v_j = min(d_j, 0) if l_j is
 *     finite, plus max(d_j, 0) if u_j is finite (d must lie in the bounds'
 *     recession cone).
 * Returns the status (primal infeasibility first) or 0; on a certificate the
 * output holds the rays (x: d, y: w, and K'yo such that the returned lam is
 * proj_Lambda(-K'w)), with pobj = c'd and dobj as above. */
static int ray_status(orc_t *P, const orc_eval_t *ec)
{
    int64_t m = P->m, n = P->n;
    double eps = P->o.infeas_tol;
    double *d = xalloc(n, sizeof(double)), *w = xalloc(m, sizeof(double));
    double *Ad = xalloc(m, sizeof(double)), *KTw = xalloc(n, sizeof(double));
    for (int64_t j = 0; j < n; ++j) d[j] = (P->x[j] - P->x0[j]) / P->Dc[j];
    for (int64_t i = 0; i < m; ++i) w[i] = (P->y[i] - P->y0[i]) / P->Dr[i];
    spmv_K_unscaled(P, d, Ad);
    spmv_KT_unscaled(P, w, KTw);
    double cd = 0.0, pres2 = 0.0, qw = 0.0, bnd = 0.0, dres2 = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double r = Ad[i];
        if (i >= P->m1) r = -Ad[i] > 0.0 ? -Ad[i] : 0.0;
        pres2 += r * r;
        qw += P->q[i] * w[i];
        if (i >= P->m1 && w[i] < 0.0) dres2 += w[i] * w[i];
    }
    for (int64_t j = 0; j < n; ++j) {
        int lf = isfinite(P->l[j]), uf = isfinite(P->u[j]);
        cd += P->c[j] * d[j];
        if (ORC_MUT != 10 && lf && d[j] < 0.0) pres2 += d[j] * d[j];
        if (ORC_MUT != 10 && uf && d[j] > 0.0) pres2 += d[j] * d[j];
        double g = -KTw[j];
        double lam = proj_lambda(g, lf, uf);
        dres2 += (g - lam) * (g - lam);
        if (lf && lam > 0.0) bnd += P->l[j] * lam;
        if (uf && lam < 0.0) bnd += (ORC_MUT == 9 ? -1.0 : 1.0) * P->u[j] * lam;
    }
    double dobj = qw + bnd;
    int st = 0;
    if (dobj > 0.0 && sqrt(dres2) <= eps * dobj) st = ORC_PRIMAL_INFEASIBLE;
    else if (cd < 0.0 && sqrt(pres2) <= eps * -cd) st = ORC_DUAL_INFEASIBLE;
    if (st) {
        for (int64_t j = 0; j < n; ++j) P->xo[j] = P->x[j] - P->x0[j];
        for (int64_t i = 0; i < m; ++i) P->yo[i] = P->y[i] - P->y0[i];
        spmv_KT(P, P->yo, P->KTyo);   /* scaled K'(y - y0) */
        for (int64_t j = 0; j < n; ++j) P->KTyo[j] += P->cs[j];
        P->out_rel_p = ec->rel_p; P->out_rel_d = ec->rel_d; P->out_rel_g = ec->rel_g;
        P->out_pobj = cd; P->out_dobj = dobj;
        P->has_output = 1;
    }
    free(d); free(w); free(Ad); free(KTw);
    return st;
}

/* Termination test on current and average; restart test when `restart_ok`.
 * Returns 1 when the run must stop (status set). */
static int check(orc_t *P, double tol, int restart_ok, int at_limit)
{
    int64_t m = P->m, n = P->n;
    orc_eval_t ec, ea;
    eval_point(P, P->x, P->y, P->Kx, P->KTy, &ec);
    eval_point(P, P->xa, P->ya, P->Kxa, P->KTya, &ea);
    if (isnan(ec.rel) || isnan(ea.rel)) {
        P->status = ORC_NUMERICAL;
        set_output(P, P->x, P->y, P->KTy, &ec);
        return 1;
    }
    int use_avg = ea.rel < ec.rel;  /* ties go to the current iterate */
    if (ec.rel <= tol || ea.rel <= tol) {
        if (use_avg) set_output(P, P->xa, P->ya, P->KTya, &ea);
        else set_output(P, P->x, P->y, P->KTy, &ec);
        P->status = ORC_OPTIMAL;
        return 1;
    }
    if (P->o.infeas_tol > 0.0) {
        int st = ray_status(P, &ec);
        if (st) {
            P->status = st;
            return 1;
        }
    }
    if (at_limit) {
        if (use_avg) set_output(P, P->xa, P->ya, P->KTya, &ea);
        else set_output(P, P->x, P->y, P->KTy, &ec);
        P->status = at_limit;
    }
    if (restart_ok) {
        double kc = kkt_omega(P, &ec, P->omega), ka = kkt_omega(P, &ea, P->omega);
        int cand_cur = ORC_MUT == 11 ? 0 : kc < ka;
        double kz = cand_cur ? kc : ka;
        const orc_eval_t *ez = cand_cur ? &ec : &ea;
        int why = orc_restart_decision(kz, P->KKT0, P->KKT_prev, P->t, P->k);
        if (ORC_MUT != 12) P->KKT_prev = kz;
        if (why) {
            P->omega = orc_omega_update(P->omega, sqrt(ez->dx2), sqrt(ez->dy2));
            if (cand_cur) {
                memcpy(P->xa, P->x, sizeof(double) * (size_t)n);
                memcpy(P->ya, P->y, sizeof(double) * (size_t)m);
                memcpy(P->Kxa, P->Kx, sizeof(double) * (size_t)m);
                memcpy(P->KTya, P->KTy, sizeof(double) * (size_t)n);
            } else {
                memcpy(P->x, P->xa, sizeof(double) * (size_t)n);
                memcpy(P->y, P->ya, sizeof(double) * (size_t)m);
                memcpy(P->Kx, P->Kxa, sizeof(double) * (size_t)m);
                memcpy(P->KTy, P->KTya, sizeof(double) * (size_t)n);
            }
            memcpy(P->x0, P->x, sizeof(double) * (size_t)n);
            memcpy(P->y0, P->y, sizeof(double) * (size_t)m);
            P->KKT0 = kkt_omega(P, ez, P->omega);
            P->KKT_prev = INFINITY;
            P->W = 0.0;
            P->t = 0;
            P->restarts += 1;
        }
    }
    return at_limit ? 1 : 0;
}

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int orc_solve(orc_t *P, double tol, int64_t max_iters, double time_limit)
{
    if (!P || max_iters < 0) return ORC_ERR_ARG;
    double t0 = now_s();
    if (!P->state_ready) init_state(P);
    P->state_ready = 0;
    P->has_output = 0;
    P->status = ORC_NOT_SOLVED;
    for (;;) {
        if (P->k >= max_iters) {
            check(P, tol, 0, ORC_ITERATION_LIMIT);
            break;
        }
        if (pdhg_step(P) != 0) {
            orc_eval_t e;
            eval_point(P, P->x, P->y, P->Kx, P->KTy, &e);
            set_output(P, P->x, P->y, P->KTy, &e);
            P->status = ORC_NUMERICAL;
            break;
        }
        int at_check = (P->k % P->o.check_every) == 0;
        int at_limit = P->k >= max_iters ? ORC_ITERATION_LIMIT : 0;
        if (!at_limit && at_check && time_limit > 0.0 && now_s() - t0 > time_limit) at_limit = ORC_TIME_LIMIT;
        if (at_check || at_limit) {
            if (check(P, tol, at_check, at_limit)) break;
        }
    }
    P->seconds = now_s() - t0;
    return ORC_OK;
}

/* info: [status, pobj, dobj, rel_p, rel_d, rel_g, k, attempts, restarts, omega, eta_hat, seconds] */
int orc_result(const orc_t *P, double *x, double *y, double *lam, double *info)
{
    if (!P) return ORC_ERR_ARG;
    if (!P->has_output) return ORC_ERR_STATE;
    for (int64_t j = 0; j < P->n; ++j) {
        if (x) x[j] = P->xo[j] / P->Dc[j];
        if (lam) {
            double g = (P->cs[j] - P->KTyo[j]) * P->Dc[j];
            lam[j] = proj_lambda(g, isfinite(P->l[j]), isfinite(P->u[j]));
        }
    }
    for (int64_t i = 0; i < P->m; ++i)
        if (y) y[i] = P->yo[i] / P->Dr[i];
    if (info) {
        info[0] = P->status; info[1] = P->out_pobj; info[2] = P->out_dobj;
        info[3] = P->out_rel_p; info[4] = P->out_rel_d; info[5] = P->out_rel_g;
        info[6] = (double)P->k; info[7] = (double)P->attempts; info[8] = (double)P->restarts;
        info[9] = P->omega; info[10] = P->eta_hat; info[11] = P->seconds;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* state export / import (scaled space, original ordering)                   */
/* scalars[16]: eta_hat, omega, W, KKT0, KKT_prev, k, t, attempts, restarts, */
/*              status, eta_last, 0...                                       */
/* then x[n] y[m] Kx[m] KTy[n] xa[n] ya[m] Kxa[m] KTya[n] x0[n] y0[m]         */
/* ------------------------------------------------------------------------ */

int64_t orc_state_len(const orc_t *P) { return ORC_NSCALARS + 5 * P->n + 5 * P->m; }

int orc_get_state(const orc_t *P, double *buf)
{
    if (!P || !buf) return ORC_ERR_ARG;
    memset(buf, 0, sizeof(double) * ORC_NSCALARS);
    buf[0] = P->eta_hat; buf[1] = P->omega; buf[2] = P->W; buf[3] = P->KKT0; buf[4] = P->KKT_prev;
    buf[5] = (double)P->k; buf[6] = (double)P->t; buf[7] = (double)P->attempts;
    buf[8] = (double)P->restarts; buf[9] = P->status; buf[10] = P->eta_last;
    double *p = buf + ORC_NSCALARS;
    const double *src[] = {P->x, P->y, P->Kx, P->KTy, P->xa, P->ya, P->Kxa, P->KTya, P->x0, P->y0};
    const int64_t len[] = {P->n, P->m, P->m, P->n, P->n, P->m, P->m, P->n, P->n, P->m};
    for (int i = 0; i < 10; ++i) {
        memcpy(p, src[i], sizeof(double) * (size_t)len[i]);
        p += len[i];
    }
    return ORC_OK;
}

int orc_set_state(orc_t *P, const double *buf)
{
    if (!P || !buf) return ORC_ERR_ARG;
    P->eta_hat = buf[0]; P->omega = buf[1]; P->W = buf[2]; P->KKT0 = buf[3]; P->KKT_prev = buf[4];
    P->k = (int64_t)buf[5]; P->t = (int64_t)buf[6]; P->attempts = (int64_t)buf[7];
    P->restarts = (int64_t)buf[8]; P->eta_last = buf[10];
    const double *p = buf + ORC_NSCALARS;
    double *dst[] = {P->x, P->y, P->Kx, P->KTy, P->xa, P->ya, P->Kxa, P->KTya, P->x0, P->y0};
    const int64_t len[] = {P->n, P->m, P->m, P->n, P->n, P->m, P->m, P->n, P->n, P->m};
    for (int i = 0; i < 10; ++i) {
        memcpy(dst[i], p, sizeof(double) * (size_t)len[i]);
        p += len[i];
    }
    P->state_ready = 1;
    return ORC_OK;
}

/* KKT_omega of a point (x, y) of the scaled problem (restart criteria),
 * with the anchor at the point itself. */
double orc_kkt_omega(orc_t *P, const double *x, const double *y, double omega)
{
    double *Kx = xalloc(P->m, sizeof(double)), *KTy = xalloc(P->n, sizeof(double));
    double *x0s = xalloc(P->n, sizeof(double)), *y0s = xalloc(P->m, sizeof(double));
    spmv_K(P, x, Kx);
    spmv_KT(P, y, KTy);
    memcpy(x0s, P->x0, sizeof(double) * (size_t)P->n);
    memcpy(y0s, P->y0, sizeof(double) * (size_t)P->m);
    memcpy(P->x0, x, sizeof(double) * (size_t)P->n);
    memcpy(P->y0, y, sizeof(double) * (size_t)P->m);
    orc_eval_t e;
    eval_point(P, x, y, Kx, KTy, &e);
    memcpy(P->x0, x0s, sizeof(double) * (size_t)P->n);
    memcpy(P->y0, y0s, sizeof(double) * (size_t)P->m);
    free(Kx); free(KTy); free(x0s); free(y0s);
    return kkt_omega(P, &e, omega);
}

int orc_get_scaling(const orc_t *P, double *Dr, double *Dc, double *kv)
{
    if (!P) return ORC_ERR_ARG;
    if (Dr) memcpy(Dr, P->Dr, sizeof(double) * (size_t)P->m);
    if (Dc) memcpy(Dc, P->Dc, sizeof(double) * (size_t)P->n);
    if (kv && P->nnz) memcpy(kv, P->kv, sizeof(double) * (size_t)P->nnz);
    return ORC_OK;
}

/* K~ x and K~' y on the scaled matrix (original ordering) */
int orc_spmv(const orc_t *P, int transpose, const double *in, double *out)
{
    if (!P || !in || !out) return ORC_ERR_ARG;
    if (transpose) spmv_KT(P, in, out);
    else spmv_K(P, in, out);
    return ORC_OK;
}

/* Termination quantities of an unscaled point (x, y) on the original data:
 * out = [rel_p, rel_d, rel_g, pobj, dobj, max bound violation of x,
 *        max sign violation of y on the G rows] */
int orc_eval_unscaled(const orc_t *P, const double *x, const double *y, double *out)
{
    if (!P || !x || !y || !out) return ORC_ERR_ARG;
    int64_t m = P->m, n = P->n;
    double rp2 = 0.0, qy = 0.0, rd2 = 0.0, cx = 0.0, bnd = 0.0, bviol = 0.0, sviol = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) s += P->v[p] * x[P->ci[p]];
        double r = s - P->q[i];
        if (i >= P->m1) {
            r = (P->q[i] - s) > 0.0 ? (P->q[i] - s) : 0.0;
            if (-y[i] > sviol) sviol = -y[i];
        }
        rp2 += r * r;
        qy += P->q[i] * y[i];
    }
    double *g = xalloc(n, sizeof(double));
    for (int64_t j = 0; j < n; ++j) g[j] = P->c[j];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) g[P->ci[p]] -= P->v[p] * y[i];
    for (int64_t j = 0; j < n; ++j) {
        int lf = isfinite(P->l[j]), uf = isfinite(P->u[j]);
        double lam = proj_lambda(g[j], lf, uf);
        double rd = g[j] - lam;
        rd2 += rd * rd;
        cx += P->c[j] * x[j];
        if (lf && lam > 0.0) bnd += P->l[j] * lam;
        if (uf && lam < 0.0) bnd += (ORC_MUT == 4 ? -1.0 : 1.0) * P->u[j] * lam;
        double lo = P->l[j] - x[j], hi = x[j] - P->u[j];
        if (lo > bviol) bviol = lo;
        if (hi > bviol) bviol = hi;
    }
    free(g);
    double dobj = qy + bnd;
    out[0] = sqrt(rp2) / (1.0 + P->Nq);
    out[1] = sqrt(rd2) / (1.0 + P->Nc);
    out[2] = fabs(dobj - cx) / (1.0 + fabs(dobj) + fabs(cx));
    out[3] = cx;
    out[4] = dobj;
    out[5] = bviol;
    out[6] = sviol;
    return ORC_OK;
}
