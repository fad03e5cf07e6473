/* Test driver: runs every function of the FP64 oracle on small stored-cost
 * and fused-cost problems, with every buffer allocated at its exact size,
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * reports any out-of-bounds access, leak or undefined operation.  Built and
 * run by tests/test_oracle_sanitized.py; prints "ok" at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t m, n;
    const double *C;
    const float *X;
    const float *Y;
    const double *a;
    const double *b;
    double w;
} or_problem;

double or_cost(const or_problem *P, int64_t i, int64_t j);
void or_cost_matrix(const or_problem *P, double *out);
void or_residual(const or_problem *P, const double *T, double *r);
double or_objective(const or_problem *P, const double *T, double *r_out);
void or_block_gradient(const or_problem *P, const double *r, int64_t i, double *grad);
int64_t or_lmo2(int64_t n, const double *grad, double *margin, int64_t *runner);
int64_t or_lmo(int64_t n, const double *grad, double *margin);
double or_step_dec(int64_t k, int64_t m);
double or_step_els(const or_problem *P, const double *t_i, const double *s_i, int64_t i, const double *r);
void or_gap(const or_problem *P, const double *T, double *G, int64_t *jstar, double *grow, double *out3);
void or_init_plan(const or_problem *P, double *T);
int or_bcfw_steps(const or_problem *P, double *T, double *r, int64_t *k, int rule, int64_t nsteps,
                  const int32_t *idx, int32_t *tr_j, double *tr_gamma, double *tr_margin, int32_t *tr_runner,
                  int32_t *tr_near, double near_tol);
int or_active_steps(const or_problem *P, double *T, double *r, int64_t *k, int pairwise, int64_t nsteps,
                    const int32_t *idx, int32_t *tr_j, int32_t *tr_away, double *tr_gamma, double *tr_margin,
                    int32_t *tr_near, double *tr_amargin, int32_t *tr_anear, double *tr_dslope, double near_tol);
double or_fw_iteration(const or_problem *P, double *T, int64_t k, int rule, double *gamma_out);
double or_row_gap(const or_problem *P, const double *T, const double *r, int64_t i);
int64_t or_ga_draw(int64_t m, const double *W, double u, double *margin);
void or_ga_steps(const or_problem *P, double *T, double *r, int64_t *k, int rule, int64_t nsteps, const double *u,
                 double *W, int32_t *tr_i, double *tr_umargin, int32_t *tr_j, double *tr_gamma, double *tr_margin,
                 int32_t *tr_near, double *tr_g, double near_tol);
void or_ga_refresh(const or_problem *P, const double *T, double *W);

static uint64_t state = 88172645463325252ull;
static double urand(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * 0x1.0p-53;
}

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

static void run(int64_t m, int64_t n, int fused, double w)
{
    double *C = NULL;
    float *X = NULL, *Y = NULL;
    double *a = xmalloc(sizeof(double) * m), *b = xmalloc(sizeof(double) * n);
    double sa = 0.0, sb = 0.0;
    for (int64_t i = 0; i < m; ++i) sa += (a[i] = 0.5 + urand());
    for (int64_t j = 0; j < n; ++j) sb += (b[j] = 0.5 + urand());
    for (int64_t i = 0; i < m; ++i) a[i] /= sa;
    for (int64_t j = 0; j < n; ++j) b[j] /= sb;
    if (fused) {
        X = xmalloc(sizeof(float) * 3 * m);
        Y = xmalloc(sizeof(float) * 3 * n);
        for (int64_t q = 0; q < 3 * m; ++q) X[q] = (float)urand();
        for (int64_t q = 0; q < 3 * n; ++q) Y[q] = (float)urand();
    } else {
        C = xmalloc(sizeof(double) * m * n);
        for (int64_t q = 0; q < m * n; ++q) C[q] = urand();
    }
    or_problem P = {m, n, C, X, Y, a, b, w};
    double *cm = xmalloc(sizeof(double) * m * n);
    or_cost_matrix(&P, cm);
    double *T = xmalloc(sizeof(double) * m * n), *r = xmalloc(sizeof(double) * n);
    or_init_plan(&P, T);
    or_residual(&P, T, r);
    double *r2 = xmalloc(sizeof(double) * n);
    (void)or_objective(&P, T, r2);
    double *grad = xmalloc(sizeof(double) * n), margin;
    int64_t runner;
    or_block_gradient(&P, r, m - 1, grad);
    (void)or_lmo2(n, grad, &margin, &runner);
    (void)or_lmo(n, grad, &margin);
    (void)or_step_dec(3, m);
    double *s = xmalloc(sizeof(double) * n);
    for (int64_t j = 0; j < n; ++j) s[j] = (j == n / 2) ? a[0] : 0.0;
    (void)or_step_els(&P, T, s, 0, r);

    const int64_t ns = 6 * m;
    int32_t *idx = xmalloc(sizeof(int32_t) * ns);
    for (int64_t q = 0; q < ns; ++q) idx[q] = (int32_t)(urand() * (double)m);
    int32_t *tj = xmalloc(sizeof(int32_t) * ns), *tr = xmalloc(sizeof(int32_t) * ns);
    int32_t *tn = xmalloc(sizeof(int32_t) * 4 * ns), *ta = xmalloc(sizeof(int32_t) * ns);
    int32_t *tan = xmalloc(sizeof(int32_t) * 4 * ns);
    double *tg = xmalloc(sizeof(double) * ns), *tm = xmalloc(sizeof(double) * ns);
    double *tam = xmalloc(sizeof(double) * ns), *tds = xmalloc(sizeof(double) * ns);
    int64_t k = 0;
    for (int rule = 0; rule < 2; ++rule) {
        or_init_plan(&P, T);
        or_residual(&P, T, r);
        k = 0;
        if (or_bcfw_steps(&P, T, r, &k, rule, ns, idx, tj, tg, tm, tr, tn, 1e-12) != 0) exit(3);
        if (or_bcfw_steps(&P, T, r, &k, rule, ns, idx, NULL, NULL, NULL, NULL, NULL, 1e-12) != 0) exit(3);
    }
    double *G = xmalloc(sizeof(double) * m), *grow = xmalloc(sizeof(double) * m), out3[3];
    int64_t *js = xmalloc(sizeof(int64_t) * m);
    or_gap(&P, T, G, js, grow, out3);
    for (int pairwise = 0; pairwise < 2; ++pairwise)
        if (or_active_steps(&P, T, r, &k, pairwise, ns, idx, tj, ta, tg, tm, tn, tam, tan, tds, 1e-12) != 0) exit(4);
    double gamma;
    for (int rule = 0; rule < 2; ++rule)
        for (int64_t it = 0; it < 4; ++it) (void)or_fw_iteration(&P, T, it, rule, &gamma);
    or_residual(&P, T, r);
    (void)or_row_gap(&P, T, r, 0);
    double *W = xmalloc(sizeof(double) * m), *u = xmalloc(sizeof(double) * ns);
    for (int64_t i = 0; i < m; ++i) W[i] = 0x1p300;
    for (int64_t q = 0; q < ns; ++q) u[q] = urand();
    (void)or_ga_draw(m, W, 0.5, &margin);
    int32_t *ti = xmalloc(sizeof(int32_t) * ns);
    double *tum = xmalloc(sizeof(double) * ns), *tgg = xmalloc(sizeof(double) * ns);
    or_ga_steps(&P, T, r, &k, 0, ns, u, W, ti, tum, tj, tg, tm, tn, tgg, 1e-12);
    or_ga_refresh(&P, T, W);

    free(C); free(X); free(Y); free(a); free(b); free(cm); free(T); free(r); free(r2); free(grad); free(s);
    free(idx); free(tj); free(tr); free(tn); free(ta); free(tan); free(tg); free(tm); free(tam); free(tds);
    free(G); free(grow); free(js); free(W); free(u); free(ti); free(tum); free(tgg);
}

int main(void)
{
    run(1, 1, 0, 1.0);
    run(5, 7, 0, 2.0);
    run(9, 4, 1, 0.5);
    run(16, 33, 1, 0.0);
    run(3, 64, 0, 10.0);
    printf("ok\n");
    return 0;
}
