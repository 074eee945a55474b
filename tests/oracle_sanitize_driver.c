/* Drives every entry point of the FP64 oracle on small LPs, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure;
 * compiled and run by tests/test_oracle_sanitize.py).  Prints "ok". */
#include "../oracle/pdhg_oracle.c"

#include <stdio.h>

static uint64_t lcg = 0x9e3779b97f4a7c15ull;
static double urand(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(c) do { if (!(c)) { printf("failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void)
{
    /* a random sparse LP with a feasible point x0 and dual y0 (bounded optimum) */
    enum { M = 60, M1 = 20, N = 90, PER = 4 };
    int32_t rp[M + 1], ci[M * PER];
    double v[M * PER], c[N], q[M], l[N], u[N], x0[N], y0[M];
    int64_t nnz = 0;
    for (int i = 0; i < M; ++i) {
        rp[i] = (int32_t)nnz;
        int used[PER];
        for (int k = 0; k < PER; ++k) {
            int j, dup;
            do {
                j = (int)(urand() * N);
                dup = 0;
                for (int t = 0; t < k; ++t) dup |= used[t] == j;
            } while (dup);
            used[k] = j;
            ci[nnz] = j;
            v[nnz] = 2.0 * urand() - 1.0;
            ++nnz;
        }
    }
    rp[M] = (int32_t)nnz;
    for (int j = 0; j < N; ++j) {
        const int kind = j % 4;
        l[j] = kind == 3 ? -INFINITY : 0.0;
        u[j] = kind == 0 || kind == 1 ? 10.0 : INFINITY;
        x0[j] = kind == 3 ? urand() * 4.0 - 2.0 : urand() * 5.0;
    }
    for (int i = 0; i < M; ++i) y0[i] = i < M1 ? 2.0 * urand() - 1.0 : urand();
    for (int i = 0; i < M; ++i) {
        double s = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * x0[ci[p]];
        q[i] = i < M1 ? s : s - urand();
    }
    for (int j = 0; j < N; ++j) c[j] = 0.0;
    for (int i = 0; i < M; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p) c[ci[p]] += v[p] * y0[i];
    for (int j = 0; j < N; ++j) c[j] += (j % 4 == 3) ? 0.0 : (j % 4 == 2 ? fabs(urand()) : urand() - 0.5);

    orc_opts o;
    orc_default_opts(&o);
    orc_t *P = NULL;
    CHECK(orc_load(&P, M, N, nnz, rp, ci, v, c, q, l, u, M1, &o) == ORC_OK);
    CHECK(orc_solve(P, 1e-8, 500000, 0.0) == ORC_OK);
    double x[N], y[M], lam[N], info[16], ev[16];
    CHECK(orc_result(P, x, y, lam, info) == ORC_OK);
    CHECK(orc_eval_unscaled(P, x, y, ev) == ORC_OK);
    const int64_t len = orc_state_len(P);
    double *st = malloc(sizeof(double) * (size_t)len);
    CHECK(orc_get_state(P, st) == ORC_OK);
    CHECK(orc_set_state(P, st) == ORC_OK);
    CHECK(orc_solve(P, 1e-8, 600000, 0.0) == ORC_OK);
    double Dr[M], Dc[N], kv[M * PER], in[N], out[M], back[N];
    CHECK(orc_get_scaling(P, Dr, Dc, kv) == ORC_OK);
    for (int j = 0; j < N; ++j) in[j] = urand();
    CHECK(orc_spmv(P, 0, in, out) == ORC_OK);
    CHECK(orc_spmv(P, 1, out, back) == ORC_OK);
    (void)orc_kkt_omega(P, x, y, 1.5);
    CHECK(orc_set_start(P, x0, y0) == ORC_OK);
    CHECK(orc_set_start_weight(P, 0.7) == ORC_OK);
    CHECK(orc_solve(P, 1e-6, 100000, 0.0) == ORC_OK);
    orc_free(P);
    free(st);

    /* constant step, no scaling, and a box-only LP (m = 0) */
    o.fixed_step = 1;
    o.fixed_eta = 0.1;
    o.ruiz_iters = 0;
    o.pc_alpha = -1.0;
    CHECK(orc_load(&P, M, N, nnz, rp, ci, v, c, q, l, u, M1, &o) == ORC_OK);
    CHECK(orc_solve(P, 1e-30, 300, 0.0) == ORC_OK);
    orc_free(P);
    orc_default_opts(&o);
    int32_t rp0[1] = {0};
    double lb[N];
    for (int j = 0; j < N; ++j) lb[j] = 0.0;
    CHECK(orc_load(&P, 0, N, 0, rp0, NULL, NULL, c, NULL, lb, u, 0, &o) == ORC_OK);
    CHECK(orc_solve(P, 1e-8, 1000, 0.0) == ORC_OK);
    orc_free(P);

    /* rejected inputs leave nothing behind */
    l[0] = 11.0;
    CHECK(orc_load(&P, M, N, nnz, rp, ci, v, c, q, l, u, M1, &o) != ORC_OK && P == NULL);
    l[0] = 0.0;
    ci[0] = N;
    CHECK(orc_load(&P, M, N, nnz, rp, ci, v, c, q, l, u, M1, &o) != ORC_OK && P == NULL);
    printf("ok\n");
    return 0;
}
