/*
 * srot_oracle.c -- plain FP64 CPU oracle for block-coordinate Frank-Wolfe
 * (BCFW) on the quadratic semi-relaxed optimal-transport problem
 * (Fukunaga & Kasai, arXiv:2103.05857).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library; it is deliberately slow and written so that every
 * routine can be checked against the paper by eye.
 *
 * Orientation.  The paper keeps the column sums of T exact and relaxes the
 * row sums.  This oracle uses the transposed labelling: T is m x n,
 * row sums are exact (T 1_n = a), each block is a row t_i in a_i * simplex,
 * and the relaxed marginal is the column sum with residual
 *     r = T^T 1_m - b                     (length n).
 * The penalty weight w plays the role of the paper's 1/lambda, so the
 * objective (eq. EuculideanSquareRelaxedProblem, Sec. 3) reads
 *     f(T) = <T, C> + (w/2) ||T^T 1_m - b||^2 .
 *
 * All arithmetic is IEEE double; loops run in natural index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* -------------------------------------------------------------------------
 * Problem description.  Either C is given (row-major m x n, already widened
 * to double by the caller), or the cost is the squared Euclidean distance
 * between 3-D points X (m x 3) and Y (n x 3) stored as float, evaluated in
 * double (cost model of Sec. 5.1; squared as in the barycentric projection,
 * eq. barycentric_projection).
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t m, n;
    const double *C;   /* m*n row-major, or NULL when X,Y are used */
    const float *X;    /* m*3 source points */
    const float *Y;    /* n*3 target points */
    const double *a;   /* m  exact row sums  */
    const double *b;   /* n  relaxed column-sum target */
    double w;          /* penalty weight, the paper's 1/lambda */
} or_problem;

/* Cost c_ij: stored entry, or squared Euclidean distance in double. */
double or_cost(const or_problem *P, int64_t i, int64_t j)
{
    if (P->C) return P->C[i * P->n + j];
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double diff = (double)P->X[i * 3 + d] - (double)P->Y[j * 3 + d];
        s += diff * diff;
    }
    return s;
}

/* Materialise the whole cost matrix (for tests on small sizes). */
void or_cost_matrix(const or_problem *P, double *out)
{
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t j = 0; j < P->n; ++j)
            out[i * P->n + j] = or_cost(P, i, j);
}

/* Residual of the relaxed marginal, r = T^T 1_m - b, recomputed from T
 * (the quantity inside the penalty of eq. EuculideanSquareRelaxedProblem). */
void or_residual(const or_problem *P, const double *T, double *r)
{
    for (int64_t j = 0; j < P->n; ++j) r[j] = 0.0;
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t j = 0; j < P->n; ++j) r[j] += T[i * P->n + j];
    for (int64_t j = 0; j < P->n; ++j) r[j] -= P->b[j];
}

/* Objective f(T) = <T,C> + (w/2)||T^T 1 - b||^2
 * (eq. EuculideanSquareRelaxedProblem, Sec. 3).  r_out may be NULL. */
double or_objective(const or_problem *P, const double *T, double *r_out)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)P->n);
    or_residual(P, T, r);
    double lin = 0.0;
    for (int64_t i = 0; i < P->m; ++i)
        for (int64_t j = 0; j < P->n; ++j) lin += T[i * P->n + j] * or_cost(P, i, j);
    double pen = 0.0;
    for (int64_t j = 0; j < P->n; ++j) pen += r[j] * r[j];
    if (r_out) memcpy(r_out, r, sizeof(double) * (size_t)P->n);
    free(r);
    return lin + 0.5 * P->w * pen;
}

/* Gradient of f with respect to block i (eq. RelaxedGradient, Sec. 3.1):
 *     grad_i f = c_i + w * r ,  the same penalty part for every block. */
void or_block_gradient(const or_problem *P, const double *r, int64_t i, double *grad)
{
    for (int64_t j = 0; j < P->n; ++j) grad[j] = or_cost(P, i, j) + P->w * r[j];
}

/* Linear minimisation oracle on a_i * simplex
 * (eq. SemiRelaxedSubproblemImplement, Sec. 3.1): the minimising vertex is
 * a_i e_j with j the index of the smallest gradient entry.  Ties go to the
 * lowest index.  *margin receives (second smallest) - (smallest), the
 * distance to the nearest competing vertex (+inf when n == 1), and *runner
 * the lowest index attaining the second smallest value (-1 when n == 1). */
int64_t or_lmo2(int64_t n, const double *grad, double *margin, int64_t *runner)
{
    int64_t best = 0;
    for (int64_t j = 1; j < n; ++j)
        if (grad[j] < grad[best]) best = j;
    double second = INFINITY;
    int64_t second_j = -1;
    for (int64_t j = 0; j < n; ++j)
        if (j != best && grad[j] < second) { second = grad[j]; second_j = j; }
    if (margin) *margin = second - grad[best];
    if (runner) *runner = second_j;
    return best;
}

int64_t or_lmo(int64_t n, const double *grad, double *margin)
{
    return or_lmo2(n, grad, margin, NULL);
}

/* Decay step of Alg. 1 (Sec. 3.1), with m blocks and the global block-step
 * counter k starting at 0:  gamma = 2m / (k + 2m). */
double or_step_dec(int64_t k, int64_t m)
{
    return (2.0 * (double)m) / ((double)k + 2.0 * (double)m);
}

/* Exact line search for one block (eq. SemiRelaxedBCFWStep, Sec. 3.1), in
 * the penalty-weight form: with d = t_i - s_i,
 *     gamma = [ <d, c_i> + w <d, r> ] / ( w ||d||^2 ),
 * restricted to [0, 1] (the step range stated in Sec. 3.1).  When the
 * denominator vanishes (w == 0 or d == 0) the objective is linear along the
 * segment: take the far end if it decreases, else stay. */
double or_step_els(const or_problem *P, const double *t_i, const double *s_i,
                   int64_t i, const double *r)
{
    double num = 0.0, dd = 0.0;
    for (int64_t j = 0; j < P->n; ++j) {
        double d = t_i[j] - s_i[j];
        num += d * or_cost(P, i, j) + P->w * d * r[j];
        dd += d * d;
    }
    double den = P->w * dd;
    if (!(num > 0.0)) return 0.0;
    if (den == 0.0 || num >= den) return 1.0;
    return num / den;
}

/* Duality gap and certificates at a fixed plan T (Sec. 3.2.2).
 *   G_i    = min_j (grad_i f)_j, attained at jstar_i (lowest index)
 *   S      = the all-block LMO solution, s_i = a_i e_{jstar_i}
 *   g_i    = <t_i - s_i, c_i> + w <t_i - s_i, r>          (eq. AppenEq:Gi)
 *   g      = <T - S, C> + w <(T - S)^T 1, r>               (Thm 2)
 *   f      = objective
 *   D      = f - sum_i <t_i, grad_i f> + sum_i a_i G_i     (Lagrangian dual
 *            of App. D; the minimum over each block is the one written in
 *            the appendix derivation).
 * Any of G, jstar, grow may be NULL.  out3 = {g, f, D}. */
void or_gap(const or_problem *P, const double *T, double *G, int64_t *jstar,
            double *grow, double *out3)
{
    const int64_t m = P->m, n = P->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *grad = (double *)malloc(sizeof(double) * (size_t)n);
    double *S = (double *)calloc((size_t)(m * n), sizeof(double));
    double f = or_objective(P, T, r);

    /* all-block LMO */
    double sum_t_grad = 0.0, sum_a_min = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        or_block_gradient(P, r, i, grad);
        int64_t js = or_lmo(n, grad, NULL);
        S[i * n + js] = P->a[i];
        if (G) G[i] = grad[js];
        if (jstar) jstar[i] = js;
        for (int64_t j = 0; j < n; ++j) sum_t_grad += T[i * n + j] * grad[j];
        sum_a_min += P->a[i] * grad[js];
        if (grow) {
            double gi = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double d = T[i * n + j] - S[i * n + j];
                gi += d * or_cost(P, i, j) + P->w * d * r[j];
            }
            grow[i] = gi;
        }
    }
    /* Thm 2: g = <T - S, C> + w <(T - S)^T 1, r> */
    double lin = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) lin += (T[i * n + j] - S[i * n + j]) * or_cost(P, i, j);
    double pen = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double col = 0.0;
        for (int64_t i = 0; i < m; ++i) col += T[i * n + j] - S[i * n + j];
        pen += col * r[j];
    }
    out3[0] = lin + P->w * pen;
    out3[1] = f;
    out3[2] = f - sum_t_grad + sum_a_min;
    free(r); free(grad); free(S);
}

/* Initial plan used by the paper's experiments and by Thm 1: every block
 * at its first vertex, t_i = a_i e_1 (Sec. 5; Thm 1).  Zero-based: column 0. */
void or_init_plan(const or_problem *P, double *T)
{
    memset(T, 0, sizeof(double) * (size_t)(P->m * P->n));
    for (int64_t i = 0; i < P->m; ++i) T[i * P->n] = P->a[i];
}

/* BCFW block steps (Alg. 1, Sec. 3.1).  For each of nsteps iterations:
 * take the block index given for this iteration (the random draw is an
 * input), form the block gradient, solve the LMO, choose the step (ELS or
 * decay), move t_i toward s_i, and carry the relaxed marginal along.
 * T (m x n) and r (= T^T 1 - b) are updated in place; *k is the global
 * block-step counter used by the decay rule.  Per-step traces may be NULL:
 * the LMO vertex, the step, the margin to the runner-up vertex and the
 * runner-up's index; tr_near (nsteps x 4) lists the columns whose gradient
 * lies within near_tol of the minimum (lowest indices first, -1 padded), the
 * set of vertices that are LMO answers up to rounding.
 * rule: 0 = exact line search, 1 = decay.  Returns 0, or -1 on a bad index. */
int or_bcfw_steps(const or_problem *P, double *T, double *r, int64_t *k,
                  int rule, int64_t nsteps, const int32_t *idx,
                  int32_t *tr_j, double *tr_gamma, double *tr_margin,
                  int32_t *tr_runner, int32_t *tr_near, double near_tol)
{
    const int64_t m = P->m, n = P->n;
    double *grad = (double *)malloc(sizeof(double) * (size_t)n);
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    double *old = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t st = 0; st < nsteps; ++st) {
        int64_t i = idx[st];
        if (i < 0 || i >= m) { free(grad); free(s); free(old); return -1; }
        double *t_i = T + i * n;
        /* gradient of the selected block and its LMO vertex */
        or_block_gradient(P, r, i, grad);
        double margin;
        int64_t runner;
        int64_t js = or_lmo2(n, grad, &margin, &runner);
        for (int64_t j = 0; j < n; ++j) s[j] = 0.0;
        s[js] = P->a[i];
        /* step size */
        double gamma = (rule == 1) ? or_step_dec(*k, m) : or_step_els(P, t_i, s, i, r);
        /* block update t_i <- (1-gamma) t_i + gamma s_i; all other blocks kept */
        for (int64_t j = 0; j < n; ++j) old[j] = t_i[j];
        for (int64_t j = 0; j < n; ++j) t_i[j] = (1.0 - gamma) * t_i[j] + gamma * s[j];
        /* the column sums change only through the updated block */
        for (int64_t j = 0; j < n; ++j) r[j] += t_i[j] - old[j];
        if (tr_j) tr_j[st] = (int32_t)js;
        if (tr_gamma) tr_gamma[st] = gamma;
        if (tr_margin) tr_margin[st] = margin;
        if (tr_runner) tr_runner[st] = (int32_t)runner;
        if (tr_near) {
            int cnt = 0;
            for (int q = 0; q < 4; ++q) tr_near[st * 4 + q] = -1;
            for (int64_t j = 0; j < n && cnt < 4; ++j)
                if (grad[j] - grad[js] <= near_tol) tr_near[st * 4 + cnt++] = (int32_t)j;
        }
        *k += 1;
    }
    free(grad); free(s); free(old);
    return 0;
}

/* Block-coordinate Frank-Wolfe with away steps (Alg. A.2, BCAFW, pairwise =
 * 0) or pairwise steps (Alg. A.3, BCPFW, pairwise = 1), Sec. 4.1.  A block
 * t_i in a_i * simplex is the combination sum_j alpha_j (a_i e_j) with
 * alpha_j = t_ij / a_i; its active set is the support {j : t_ij > 0}.  Per
 * step, with g = grad_i f (eq. RelaxedGradient):
 *   FW vertex    s = a_i e_js,  js = lowest-index argmin of g;
 *   away vertex  v = a_i e_ja,  ja = argmax of g over the active set
 *                (lowest index on ties);
 *   BCAFW: d_FW = s - t_i, d_A = t_i - v; the FW direction is taken when
 *          <-g, d_FW> >= <-g, d_A>, with gamma_max = 1, else the away
 *          direction with gamma_max = alpha_ja / (1 - alpha_ja).  With a
 *          single atom, or ja = js, d_A is zero in exact arithmetic (alpha
 *          is 1 only up to rounding) and the FW direction is taken;
 *   BCPFW: d = s - v, gamma_max = alpha_ja.
 * Line search (eq. SemiRelaxedBCAFWStep in the penalty-weight form): f is
 * quadratic along d with curvature w ||d||^2, so gamma = -<g, d> / (w ||d||^2)
 * clipped to [0, gamma_max] (gamma_max when the curvature vanishes and the
 * slope is negative; 0 when the slope is not negative).  A step that reaches
 * gamma_max on an away or pairwise direction removes atom ja: its entry is
 * set to exactly 0.  Updates: FW direction (1 - gamma) t + gamma s (as
 * or_bcfw_steps), away direction (1 + gamma) t - gamma v, pairwise t_js +=
 * gamma a_i, t_ja -= gamma a_i; r follows the changed entries.
 * Traces (each optional): tr_j = js; tr_away = ja (BCAFW: -1 - ja when the
 * FW direction was taken); tr_gamma; tr_margin / tr_near as in
 * or_bcfw_steps; tr_amargin = largest minus second-largest gradient value on
 * the active set (INFINITY with one atom) and tr_anear = the first four
 * active columns within near_tol of the largest (-1 padded); tr_dslope =
 * <-g, d_FW> - <-g, d_A>, the margin of the BCAFW direction choice (NAN when
 * no choice is made: pairwise steps, one atom, or ja = js). */
int or_active_steps(const or_problem *P, double *T, double *r, int64_t *k, int pairwise,
                    int64_t nsteps, const int32_t *idx, int32_t *tr_j, int32_t *tr_away,
                    double *tr_gamma, double *tr_margin, int32_t *tr_near,
                    double *tr_amargin, int32_t *tr_anear, double *tr_dslope, double near_tol)
{
    const int64_t m = P->m, n = P->n;
    double *grad = (double *)malloc(sizeof(double) * (size_t)n);
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    double *old = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t st = 0; st < nsteps; ++st) {
        int64_t i = idx[st];
        if (i < 0 || i >= m) { free(grad); free(d); free(old); return -1; }
        double *t_i = T + i * n;
        const double ai = P->a[i];
        or_block_gradient(P, r, i, grad);
        double margin;
        int64_t runner;
        int64_t js = or_lmo2(n, grad, &margin, &runner);
        int64_t ja = -1, natoms = 0;
        for (int64_t j = 0; j < n; ++j)
            if (t_i[j] > 0.0) {
                ++natoms;
                if (ja < 0 || grad[j] > grad[ja]) ja = j;
            }
        double gamma = 0.0, dslope = NAN;
        int fw_dir = 0, drop = 0;
        for (int64_t j = 0; j < n; ++j) old[j] = t_i[j];
        if (ja >= 0) {
            const double alpha = t_i[ja] / ai;
            double gmax;
            if (pairwise) {
                for (int64_t j = 0; j < n; ++j) d[j] = (j == js ? ai : 0.0) - (j == ja ? ai : 0.0);
                gmax = alpha;
            } else {
                double slope_fw = 0.0, slope_aw = 0.0;   /* <-g, d_FW>, <-g, d_A> */
                for (int64_t j = 0; j < n; ++j) {
                    slope_fw -= grad[j] * ((j == js ? ai : 0.0) - t_i[j]);
                    slope_aw -= grad[j] * (t_i[j] - (j == ja ? ai : 0.0));
                }
                /* with one atom, or the away vertex at the FW vertex, the away
                 * direction is zero in exact arithmetic: take the FW one */
                fw_dir = natoms == 1 || ja == js || slope_fw >= slope_aw;
                if (natoms > 1 && ja != js) dslope = slope_fw - slope_aw;
                if (fw_dir) {
                    for (int64_t j = 0; j < n; ++j) d[j] = (j == js ? ai : 0.0) - t_i[j];
                    gmax = 1.0;
                } else {
                    for (int64_t j = 0; j < n; ++j) d[j] = t_i[j] - (j == ja ? ai : 0.0);
                    gmax = alpha / (1.0 - alpha);
                }
            }
            double num = 0.0, dd = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                num -= d[j] * grad[j];
                dd += d[j] * d[j];
            }
            const double den = P->w * dd;
            if (!(num > 0.0)) gamma = 0.0;
            else if (den == 0.0) gamma = gmax;
            else gamma = num / den < gmax ? num / den : gmax;
            drop = !fw_dir && gamma > 0.0 && gamma == gmax;
            if (fw_dir) {
                for (int64_t j = 0; j < n; ++j) t_i[j] = (1.0 - gamma) * t_i[j] + (j == js ? gamma * ai : 0.0);
            } else if (pairwise) {
                if (js != ja) {
                    t_i[js] = t_i[js] + gamma * ai;
                    t_i[ja] = t_i[ja] - gamma * ai;
                }
            } else {
                for (int64_t j = 0; j < n; ++j) t_i[j] = (1.0 + gamma) * t_i[j] - (j == ja ? gamma * ai : 0.0);
            }
            if (drop) t_i[ja] = 0.0;
        }
        for (int64_t j = 0; j < n; ++j) r[j] += t_i[j] - old[j];
        if (tr_j) tr_j[st] = (int32_t)js;
        if (tr_away) tr_away[st] = (int32_t)(fw_dir ? -1 - ja : ja);
        if (tr_gamma) tr_gamma[st] = gamma;
        if (tr_dslope) tr_dslope[st] = dslope;
        if (tr_margin) tr_margin[st] = margin;
        if (tr_near) {
            int cnt = 0;
            for (int q = 0; q < 4; ++q) tr_near[st * 4 + q] = -1;
            for (int64_t j = 0; j < n && cnt < 4; ++j)
                if (grad[j] - grad[js] <= near_tol) tr_near[st * 4 + cnt++] = (int32_t)j;
        }
        if (tr_amargin || tr_anear) {
            double second = -INFINITY;
            int cnt = 0;
            if (tr_anear) for (int q = 0; q < 4; ++q) tr_anear[st * 4 + q] = -1;
            for (int64_t j = 0; j < n; ++j) {
                if (!(old[j] > 0.0)) continue;
                if (j != ja && grad[j] > second) second = grad[j];
                if (tr_anear && ja >= 0 && grad[ja] - grad[j] <= near_tol && cnt < 4) tr_anear[st * 4 + cnt++] = (int32_t)j;
            }
            if (tr_amargin) tr_amargin[st] = (ja >= 0 && second > -INFINITY) ? grad[ja] - second : INFINITY;
        }
        *k += 1;
    }
    free(grad); free(d); free(old);
    return 0;
}

/* Full Frank-Wolfe iteration (Alg. A.1, App. A): LMO on every block, then
 * one step on the whole plan.  ELS per eq. AppenEq:SemiRelaxedFWStep in the
 * penalty-weight form, with D = T - S:
 *     gamma = [ <D, C> + w <D^T 1, r> ] / ( w ||D^T 1||^2 ),  in [0, 1];
 * decay rule gamma = 2/(k+2).  Returns the gap g(T) measured before the
 * step (the stopping quantity of Alg. A.1); *gamma_out receives the step. */
double or_fw_iteration(const or_problem *P, double *T, int64_t k, int rule,
                       double *gamma_out)
{
    const int64_t m = P->m, n = P->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *grad = (double *)malloc(sizeof(double) * (size_t)n);
    double *S = (double *)calloc((size_t)(m * n), sizeof(double));
    or_residual(P, T, r);
    for (int64_t i = 0; i < m; ++i) {
        or_block_gradient(P, r, i, grad);
        S[i * n + or_lmo(n, grad, NULL)] = P->a[i];
    }
    double lin = 0.0, pen = 0.0, dd = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) lin += (T[i * n + j] - S[i * n + j]) * or_cost(P, i, j);
    for (int64_t j = 0; j < n; ++j) {
        double col = 0.0;
        for (int64_t i = 0; i < m; ++i) col += T[i * n + j] - S[i * n + j];
        pen += col * r[j];
        dd += col * col;
    }
    double num = lin + P->w * pen;
    double gamma;
    if (rule == 1) {
        gamma = 2.0 / ((double)k + 2.0);
    } else {
        double den = P->w * dd;
        if (!(num > 0.0)) gamma = 0.0;
        else if (den == 0.0 || num >= den) gamma = 1.0;
        else gamma = num / den;
    }
    for (int64_t q = 0; q < m * n; ++q) T[q] = (1.0 - gamma) * T[q] + gamma * S[q];
    if (gamma_out) *gamma_out = gamma;
    free(r); free(grad); free(S);
    return num;
}

/* -------------------------------------------------------------------------
 * BCFW with gap-adaptive sampling (BCFW-GA, Alg. A.4, Sec. 4.2.1).
 * ---------------------------------------------------------------------- */

/* Gap of one block (eq. AppenEq:Gi) at plan T with residual r:
 *     g_i = <t_i - s_i, c_i> + w <t_i - s_i, r>,
 * s_i = a_i e_j* the block's LMO vertex at r.  The sum over the blocks is the
 * linearization gap g(T) (Thm 2). */
double or_row_gap(const or_problem *P, const double *T, const double *r, int64_t i)
{
    const int64_t n = P->n;
    double *grad = (double *)malloc(sizeof(double) * (size_t)n);
    or_block_gradient(P, r, i, grad);
    const int64_t js = or_lmo(n, grad, NULL);
    free(grad);
    double lin = 0.0, pen = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double d = T[i * n + j] - ((j == js) ? P->a[i] : 0.0);
        lin += d * or_cost(P, i, j);
        pen += d * r[j];
    }
    return lin + P->w * pen;
}

/* Block draw of Alg. A.4: block i with probability W_i / sum_q W_q, by
 * inversion.  The running sums S_i = W_0 + ... + W_i are formed in row
 * order, x = u * S_{m-1} with u in [0, 1), and i is the first block with
 * S_i > x; a block of zero weight is therefore never drawn.  Should
 * rounding leave x at or above the full sum, x is replaced by the largest
 * double below it.  When every weight is zero, i = floor(u m).
 * *margin receives the distance from x to the nearer end of the chosen
 * block's interval [S_{i-1}, S_i), relative to the full sum (+inf when
 * every weight is zero). */
int64_t or_ga_draw(int64_t m, const double *W, double u, double *margin)
{
    double total = 0.0;
    for (int64_t q = 0; q < m; ++q) total += W[q];
    if (!(total > 0.0)) {
        int64_t i = (int64_t)(u * (double)m);
        if (margin) *margin = INFINITY;
        return i < m ? i : m - 1;
    }
    double x = u * total;
    if (x >= total) x = nextafter(total, 0.0);
    double lo = 0.0, run = 0.0;
    for (int64_t q = 0; q < m; ++q) {
        const double hi = run + W[q];
        if (hi > x) {
            const double d1 = x - lo, d2 = hi - x;
            if (margin) *margin = (d1 < d2 ? d1 : d2) / total;
            return q;
        }
        lo = hi;
        run = hi;
    }
    if (margin) *margin = 0.0;   /* not reached: S_{m-1} = total > x */
    return m - 1;
}

/* nsteps iterations of Alg. A.4 in place on (T, r, *k, W): draw a block
 * from the stored gaps W (or_ga_draw with the given uniform u[s]), take
 * the BCFW block step of Alg. 1 on it (or_bcfw_steps: LMO, step rule, block
 * and marginal update), then store that block's gap at the new plan,
 * clamped at 0 (the exact value is non-negative; the clamp only removes a
 * rounding-level negative that would be no probability).  The global
 * update of all stored gaps is or_ga_refresh, called by the driver of the
 * outer iterations.  Traces (each optional): the drawn block, its draw
 * margin, the vertex, the step, the LMO margin and near set (as
 * or_bcfw_steps), and the stored gap. */
void or_ga_steps(const or_problem *P, double *T, double *r, int64_t *k, int rule, int64_t nsteps,
                 const double *u, double *W, int32_t *tr_i, double *tr_umargin, int32_t *tr_j,
                 double *tr_gamma, double *tr_margin, int32_t *tr_near, double *tr_g, double near_tol)
{
    for (int64_t s = 0; s < nsteps; ++s) {
        double um;
        const int32_t i = (int32_t)or_ga_draw(P->m, W, u[s], &um);
        or_bcfw_steps(P, T, r, k, rule, 1, &i, tr_j ? tr_j + s : NULL, tr_gamma ? tr_gamma + s : NULL,
                      tr_margin ? tr_margin + s : NULL, NULL, tr_near ? tr_near + 4 * s : NULL, near_tol);
        const double g = or_row_gap(P, T, r, i);
        W[i] = g > 0.0 ? g : 0.0;
        if (tr_i) tr_i[s] = i;
        if (tr_umargin) tr_umargin[s] = um;
        if (tr_g) tr_g[s] = W[i];
    }
}

/* Global update of Alg. A.4: every block's gap (eq. AppenEq:Gi) at plan T,
 * with the residual recomputed from T, clamped at 0 as in or_ga_steps. */
void or_ga_refresh(const or_problem *P, const double *T, double *W)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)P->n);
    or_residual(P, T, r);
    for (int64_t i = 0; i < P->m; ++i) {
        const double g = or_row_gap(P, T, r, i);
        W[i] = g > 0.0 ? g : 0.0;
    }
    free(r);
}
