/*
 * srot.h -- C ABI of the MI355X (gfx950) block-coordinate Frank-Wolfe solver
 * for quadratic semi-relaxed optimal transport
 * (Fukunaga & Kasai, arXiv:2103.05857).
 *
 * Problem (eq. EuculideanSquareRelaxedProblem, Sec. 3, written with blocks as
 * rows): given a cost C (m x n), exact row sums a (m) and a target b (n) for
 * the relaxed column sums,
 *
 *     minimise  f(T) = <T, C> + (w/2) || T^T 1_m - b ||^2
 *     over      T >= 0,  T 1_n = a          (a product of scaled simplices,
 *                                            eq. EuclideanRelaxedCartesian)
 *
 * w is the penalty weight (the paper's 1/lambda).  Each row t_i is one block
 * of the block-coordinate method (Alg. 1, Sec. 3.1); r = T^T 1 - b is the
 * residual of the relaxed marginal, kept on the device and updated in place.
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" are HIP device pointers, "host" are host
 *     pointers.  The caller owns every buffer it passes and keeps it alive
 *     until srot_destroy; the library allocates no device memory: all its
 *     state lives in the caller's workspace.
 *   - Matrices are row-major and dense, rows contiguous (leading dim = n).
 *   - All work is enqueued on the stream given to srot_init.  Entry points
 *     that return host scalars (srot_gap, srot_solve) synchronise that
 *     stream; the others return as soon as the work is enqueued.
 *   - Return value: SROT_OK (0), SROT_NOT_CONVERGED (> 0, soft), or a
 *     negative error code.  On error, srot_last_error() holds a message
 *     (per thread).  No C++ exception crosses this interface.
 *   - A handle is not thread-safe; calls on one handle must be serialised.
 */
#ifndef SROT_H
#define SROT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SROT_OK              0
#define SROT_NOT_CONVERGED   1   /* max_passes reached with gap > eps   */
#define SROT_EINVAL         -1   /* bad argument (shape, pointer, option) */
#define SROT_ENOMEM         -2   /* workspace smaller than srot_workspace_size */
#define SROT_ENONFINITE     -3   /* NaN/Inf or negative weight in the inputs  */
#define SROT_EHIP           -4   /* a HIP runtime call failed                  */
#define SROT_ECAPACITY      -5   /* an output buffer holds fewer entries than needed */

/* step rules (Alg. 1, Sec. 3.1) */
#define SROT_ELS  0   /* exact line search, eq. SemiRelaxedBCFWStep     */
#define SROT_DEC  1   /* decay step 2m/(k+2m), k = global block-step count */

/* block-step variants (Sec. 4.1) */
#define SROT_STEP_AWAY      1   /* away steps, Alg. A.2 (BCAFW)     */
#define SROT_STEP_PAIRWISE  2   /* pairwise steps, Alg. A.3 (BCPFW) */

/* block sampling (Sec. 3.1) */
#define SROT_UNIFORM  0   /* i.i.d. uniform rows (BCFW-U)             */
#define SROT_PERMUTE  1   /* a fresh random permutation per pass (BCFW-P) */

/* cost storage */
#define SROT_COST_F32      0   /* C stored as float  (m x n)                 */
#define SROT_COST_F64      1   /* C stored as double (m x n)                 */
#define SROT_COST_SQEUCLID 2   /* C never stored: c_ij = ||x_i - y_j||^2 from
                                  float points X (m x 3), Y (n x 3), evaluated
                                  in double (Sec. 5.1 cost, squared)         */

typedef struct srot_handle srot_handle;   /* opaque */

typedef struct {
    double   w;           /* penalty weight, >= 0 (the paper's 1/lambda)       */
    int32_t  step_rule;   /* SROT_ELS | SROT_DEC                               */
    int32_t  sampling;    /* SROT_UNIFORM | SROT_PERMUTE                       */
    uint64_t seed;        /* key of the Philox4x64-10 block-index stream       */
    double   eps;         /* stop when the duality gap g(T) <= eps (Sec. 3.1)  */
    int64_t  max_passes;  /* passes of m block steps before giving up          */
    int32_t  gap_every;   /* passes between gap evaluations (>= 1; the paper
                             measures the gap once per pass, Sec. 3.1)         */
    int32_t  cost;        /* SROT_COST_F32 | SROT_COST_F64 | SROT_COST_SQEUCLID */
} srot_options;

/* Fills *opt with: w = 1, ELS, uniform sampling, seed 0, eps = 1e-6,
 * max_passes = 1000 (the paper's default budget of 1000 epochs, Sec. 5),
 * gap_every = 1, cost = SROT_COST_F32. */
void srot_default_options(srot_options *opt);

/* Bytes of device workspace needed for an m x n problem with these options
 * (dense FP64 plan, residual, index and reduction buffers; 256-byte aligned
 * sub-buffers).  Returns 0 for invalid sizes. */
size_t srot_workspace_size(int64_t m, int64_t n, const srot_options *opt);

/* Creates a solver for one problem and sets the initial plan used by the
 * paper's experiments and Thm 1: every row at its first vertex,
 * t_i = a_i e_0, with the residual r computed from it; k = 0.
 *   C         device; m x n float or double (opt->cost), or NULL for
 *             SROT_COST_SQEUCLID.  Read at every step; must stay unchanged.
 *   X, Y      device; m x 3 and n x 3 float.  Required for SROT_COST_SQEUCLID
 *             and by srot_backward for point gradients; otherwise may be NULL.
 *   a, b      device; m and n doubles, finite and >= 0.
 *   workspace device; at least srot_workspace_size(m, n, opt) bytes, 256-byte
 *             aligned.  Owned by the caller, used exclusively by this handle.
 *   opt       host; copied.
 *   stream    a hipStream_t (NULL = the default stream).
 * Validates the inputs on the device (SROT_ENONFINITE on NaN/Inf anywhere in
 * C/X/Y/a/b or a negative weight) and synchronises once.
 * Errors: SROT_EINVAL (m, n < 1, m or n > 2^31 - 1, bad option, NULL pointer
 * where one is required), SROT_ENOMEM, SROT_ENONFINITE, SROT_EHIP. */
int srot_init(srot_handle **out, int64_t m, int64_t n, const void *C,
              const float *X, const float *Y, const double *a, const double *b,
              void *workspace, size_t ws_bytes, const srot_options *opt,
              void *stream);

/* Runs nsteps BCFW block steps (Alg. 1): for each step take block i, form the
 * block gradient c_i + w r (eq. RelaxedGradient), pick the LMO vertex
 * a_i e_j* with j* the lowest index of the smallest gradient entry
 * (eq. SemiRelaxedSubproblemImplement), take the ELS step
 * (eq. SemiRelaxedBCFWStep, clipped to [0,1]) or the decay step, and update
 * t_i and r in place.
 *   idx          device, nsteps int32 block indices in [0, m), or NULL to draw
 *                them from the handle's Philox stream (opt->sampling, seed)
 *                at the handle's step counter.  Out-of-range indices give
 *                SROT_EINVAL (checked on the device before any update).
 *   trace_j      device, nsteps int32 (optional): the LMO vertex j* per step.
 *   trace_gamma  device, nsteps double (optional): the step size per step.
 * Enqueues the work and returns (one validation synchronisation when idx is
 * given by the caller). */
int srot_step(srot_handle *h, int64_t nsteps, const int32_t *idx,
              int32_t *trace_j, double *trace_gamma);

/* Duality gap at the current plan (Thm 2, Sec. 3.2.2) with its certificates:
 *   out3[0] = g(T) = sum_i g_i,  g_i = <t_i - s_i, c_i + w r>  (eq. AppenEq:Gi)
 *   out3[1] = f(T)
 *   out3[2] = D(T), the Lagrangian dual value of App. D, = f - g
 * out3 is host memory.  row_gap (device, m doubles) and row_argmin (device,
 * m int32) are optional per-row outputs g_i and j*_i.  Synchronises. */
int srot_gap(srot_handle *h, double *out3, double *row_gap, int32_t *row_argmin);

/* The same sweep as srot_gap, enqueued without synchronising: when the
 * stream reaches it, out5 (device or pinned host memory, 5 doubles) receives
 * {g, f, D, <T, C>, ||r||^2}.  Per-row outputs stay in the workspace. */
int srot_gap_async(srot_handle *h, double *out5);

/* Runs passes of m block steps, measuring the gap every opt->gap_every passes
 * and stopping at the first measurement with g <= opt->eps, or after
 * opt->max_passes passes (Sec. 3.1 stopping rule).  The stop test runs on
 * the device: passes are queued four at a time, the next four before the
 * host reads the last ones' stop word (copied to pinned host memory the
 * handle holds from its first solve), so the GPU does not wait for the
 * host between them; passes queued after the stopping one do nothing, so the
 * state left is that of the stopping pass (the same as testing after every
 * pass on the host).
 *   out3    host, {g, f, D} at the last measurement.
 *   passes  host, number of passes run by this call.
 * Returns SROT_OK when converged, SROT_NOT_CONVERGED otherwise, SROT_EHIP
 * when a team-chain member (rows of 4097-65536 columns) gave up waiting for
 * the others (the plan is then inconsistent; the failure stays recorded
 * until srot_set_state loads a state). */
int srot_solve(srot_handle *h, double *out3, int64_t *passes);

/* Copies the dense plan T (device, m x n double) and the residual
 * r = T^T 1 - b (device, n double) out; either may be NULL. */
int srot_get_plan(srot_handle *h, double *T_out, double *r_out);

/* The plan in compressed sparse rows: row i's support (its active set,
 * Sec. 4.1, eq. ActiveSet: the columns with t_ij > 0) in ascending column
 * order, with the plan entries; read from the support masks, so only the
 * support of T is touched.
 *   row_ptr  device, m + 1 int32: row i's entries are
 *            [row_ptr[i], row_ptr[i + 1]); always written.
 *   col      device, cap int32 column indices, or NULL with cap = 0.
 *   val      device, cap double plan entries, or NULL with cap = 0.
 *   cap      entries col and val can hold (>= 0).
 *   nnz      host: the number of entries, also when it exceeds cap.
 * col and val are written only when nnz <= cap, on the handle's stream
 * (asynchronously); reading the count synchronises.
 * Errors: SROT_EINVAL (NULL h, row_ptr or nnz, cap < 0, col or val NULL
 * with cap > 0, more than 2^31 - 1 entries), SROT_ECAPACITY (nnz > cap:
 * call again with a larger buffer), SROT_EHIP. */
int srot_get_plan_csr(srot_handle *h, int32_t *row_ptr, int32_t *col, double *val, int64_t cap, int64_t *nnz);

/* Checkpoint / resume: the state is (T, r, k).  srot_get_state writes the
 * block-step counter to *k (host); srot_get_plan copies T and r.
 * srot_set_state loads a plan T (device, m x n double; rows must lie on
 * a_i * simplex up to rounding, not checked), rebuilds the support masks, and
 * either copies the residual r_in (device, n double) or, when r_in is NULL,
 * recomputes it from T; the counter becomes k.  With r_in taken from the
 * same run, a resumed run repeats the uninterrupted one bit for bit (the
 * block-index stream is counter based). */
int srot_get_state(srot_handle *h, int64_t *k);
int srot_set_state(srot_handle *h, const double *T_in, const double *r_in, int64_t k);

/* Diagnostics of the last block-step launch (srot_step, or the steps of a
 * pass of srot_solve), written to out4 (host, 4 int64; synchronises):
 *   out4[0]  steps whose LMO (eq. SemiRelaxedSubproblemImplement) scanned the
 *            full row outside the chain's fast path: with the screened LMO
 *            (stored FP32 cost, 513-4096 columns), steps where the
 *            candidates could not be certified; otherwise steps taken by the
 *            one-at-a-time tail path;
 *   out4[1]  screened LMO only: steps whose support was re-read from the plan
 *            (rows updated within the last 8 steps, or rows with more
 *            nonzeros per screener lane than prepared);
 *   out4[2]  which chain kernel ran the last launch, written by the kernel
 *            itself: SROT_CHAIN_PREFETCH, SROT_CHAIN_SCREENED,
 *            SROT_CHAIN_TEAM (the default beyond 4096 columns), or
 *            SROT_CHAIN_GLOBAL / SROT_CHAIN_WIDE (one workgroup, selected by
 *            SROT_TEAM_CHAIN=0 in the environment) (0 before any launch);
 *   out4[3]  0 (reserved).
 * The chains for rows of up to 4096 columns with a register-resident
 * residual write out4[0] and out4[1] at every launch; the wide-row chains
 * (more than 4096 columns) leave them as they were (0 after srot_init).
 * Neither changes any result: every path takes the same exact step.
 * Setting SROT_LMO_SCREEN=0 in the environment before srot_init selects the
 * unscreened chain for that handle. */
int srot_chain_stats(srot_handle *h, int64_t *out4);
#define SROT_CHAIN_PREFETCH  1   /* one workgroup, rows prefetched, r in LDS   */
#define SROT_CHAIN_SCREENED  2   /* stepper wave over FP32-screened candidates */
#define SROT_CHAIN_GLOBAL    3   /* stored cost wider than 4096 columns        */
#define SROT_CHAIN_WIDE      4   /* fused cost wider than 4096 columns (one workgroup) */
#define SROT_CHAIN_TEAM      5   /* rows of 4097-65536 columns over a team of workgroups */

/* Gradients of the optimal value V = min f (the problem above) with respect
 * to the inputs, evaluated at the handle's current plan T and scaled by
 * grad_out (dL/dV of a caller's loss L).  The paper does not differentiate
 * V; these are the envelope-theorem derivatives, i.e. the partial
 * derivatives of the Lagrangian of App. D with the plan held fixed:
 *     dC_ij = g t_ij,            db_j = -g w r_j,
 *     da_i  = g min_j (c_ij + w r_j)   (the row multiplier at the optimum),
 *     dX_i  = 2 g sum_j t_ij (x_i - y_j),   dY_j = 2 g sum_i t_ij (y_j - x_i),
 * with g = grad_out.  They are exact at an optimal plan; at an iterate with
 * duality gap G (srot_gap) the residual, hence db, is within
 * sqrt(2 w G) * |g| in Euclidean norm of its optimal value.  dX and dY take
 * c_ij = ||x_i - y_j||^2, the fused cost, and need X and Y at srot_init.
 *   dC   device, m x n, float for SROT_COST_F32, double for SROT_COST_F64;
 *        NULL to skip; must be NULL for SROT_COST_SQEUCLID.  Written densely
 *        (zeros off the plan's support).
 *   dX   device, m x 3 float, or NULL.      dY  device, n x 3 float, or NULL.
 *   da   device, m double, or NULL (costs one gap sweep).
 *   db   device, n double, or NULL.
 * Sums run in FP64 in a fixed order (bit-reproducible).  Enqueues the work
 * and returns without synchronising.
 * Errors: SROT_EINVAL (NULL handle, non-finite grad_out, dC with the fused
 * cost, dX/dY without points), SROT_EHIP. */
int srot_backward(srot_handle *h, double grad_out, void *dC, float *dX, float *dY,
                  double *da, double *db);

/* srot_backward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, outputs (bit for bit) and errors as srot_backward, and it
 * calls no hipMalloc, hipFree or allocating library routine.  The scratch
 * of its kernels -- the gap sweep's arrival counter, per-workgroup partial
 * sums and final sums (when da is requested) and the per-row-slice column
 * sums of dY -- is not taken from the workspace but from a static device
 * array of SROT_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends; its address is looked up at srot_init with
 * the handle's device current.  All calls on one GPU share that array and
 * it keeps the last call's contents (the counter is cleared by a kernel at
 * every call): calls that overlap on one GPU (several streams or threads)
 * race and give wrong results, so serialise them.  The handle's per-row gap
 * arrays are updated as srot_backward updates them.
 * Limit: 512 bytes, plus 64 x min(2048, ceil(m / 8)) bytes with da, plus
 * 24 n s bytes with dY (s <= min(m, 32) row slices) must fit in
 * SROT_NOALLOC_SCRATCH_BYTES; with every output that holds for any m when
 * n <= 10751.
 * Errors: those of srot_backward; SROT_EINVAL when the scratch needed
 * exceeds the limit (srot_backward has none); SROT_EHIP when the static
 * array had no device address at srot_init. */
#define SROT_NOALLOC_SCRATCH_BYTES (8u << 20)
int srot_backward_noalloc(srot_handle *h, double grad_out, void *dC, float *dX, float *dY,
                          double *da, double *db);

/* Block steps with away or pairwise directions (Sec. 4.1, Alg. A.2 / A.3)
 * on the handle's plan, in place of srot_step's FW direction.  A row's
 * active set is its support; per step, with g = c_i + w r:
 *   FW vertex js = lowest-index argmin of g; away vertex ja = lowest-index
 *   argmax of g over the support, alpha = t_ija / a_i;
 *   SROT_STEP_AWAY: FW direction a_i e_js - t_i (gamma_max = 1) when its
 *     slope is at least that of the away direction t_i - a_i e_ja (gamma_max
 *     = alpha / (1 - alpha)), and always with a single atom or ja = js;
 *   SROT_STEP_PAIRWISE: d = a_i (e_js - e_ja), gamma_max = alpha;
 *   gamma = clip(-<g, d> / (w ||d||^2), 0, gamma_max)
 *   (eq. SemiRelaxedBCAFWStep); reaching gamma_max on an away or pairwise
 *   direction empties atom ja exactly.
 * Needs opt->step_rule == SROT_ELS and rows of at most 8192 columns.
 * Stored FP32 rows of 513-4096 columns take the steps on the screened LMO
 * chain of srot_step (SROT_CHAIN_SCREENED): the same steps, with the support
 * sums added in another order.
 *   idx          device block indices, or NULL for the handle's sampler.
 *   trace_j      device int32 per step (optional): js.
 *   trace_away   device int32 per step (optional): ja, or -1 - ja when the
 *                FW direction was taken.
 *   trace_gamma  device double per step (optional).
 * Errors: SROT_EINVAL (variant, step rule, row width, index), SROT_EHIP. */
int srot_step_variant(srot_handle *h, int variant, int64_t nsteps, const int32_t *idx,
                      int32_t *trace_j, int32_t *trace_away, double *trace_gamma);

/* srot_solve with srot_step_variant's steps. */
int srot_solve_variant(srot_handle *h, int variant, double *out3, int64_t *passes);

/* Block-coordinate Frank-Wolfe with gap-adaptive sampling (BCFW-GA,
 * Alg. A.4, Sec. 4.2.1).  The handle keeps a stored gap W_i per row (block);
 * srot_init sets every W_i to SROT_GA_INIT.  An inner iteration draws row i
 * with probability W_i / sum W by inversion of x = u sum W (a row of zero
 * weight is never drawn; with every weight zero, i = floor(u m)), takes the
 * BCFW block step of srot_step on it (opt->step_rule), and stores the row's
 * gap at the new plan, g_i = <t_i - s_i, c_i + w r> (eq. AppenEq:Gi, >= 0).
 * The global update recomputes every W_i at the current plan.
 * Rows of at most 8192 columns and at most 16384 rows.
 * The initial constant 2^300 is exact under addition and absorbs every real
 * row gap, so rows not yet visited are drawn (uniformly) before any other. */
#define SROT_GA_INIT 0x1p300

/* Every stored row gap <- init (> 0 and finite, m * init finite). */
int srot_ga_reset(srot_handle *h, double init);

/* Global update: every stored row gap <- the gap sweep's g_i at the current
 * plan (one sweep; enqueued, no synchronisation). */
int srot_ga_refresh(srot_handle *h);

/* Copies the m stored row gaps to W_out (device, m doubles); enqueued. */
int srot_ga_weights(srot_handle *h, double *W_out);

/* nsteps inner iterations (enqueued, no synchronisation).
 *   u            device, nsteps uniforms in [0, 1) (others count as 0), or
 *                NULL: u_s = floor(x / 2^11) 2^-53 with x the output k + s
 *                of the handle's block-index stream (Philox4x64-10, key
 *                (seed, 0)), k the global block-step counter.
 *   trace_i      device int32 per step (optional): the drawn row.
 *   trace_j      device int32 per step (optional): its LMO vertex.
 *   trace_gamma  device double per step (optional): the step size.
 *   trace_g      device double per step (optional): the stored row gap.
 * Errors: SROT_EINVAL (NULL handle, nsteps < 0, problem too large), SROT_EHIP. */
int srot_step_ga(srot_handle *h, int64_t nsteps, const double *u, int32_t *trace_i, int32_t *trace_j,
                 double *trace_gamma, double *trace_g);

/* Outer iterations of Alg. A.4 from the current plan: every stored gap set
 * to init (init <= 0: SROT_GA_INIT), then passes of m inner iterations
 * (u from the handle's stream); the gap is measured every opt->gap_every
 * passes (stop at g <= opt->eps) and every `period` passes (>= 1) the
 * global update runs (reusing that pass's sweep).  out3 (host) = {g, f, D};
 * *passes (host).  Returns SROT_OK or SROT_NOT_CONVERGED. */
int srot_solve_ga(srot_handle *h, double init, int64_t period, double *out3, int64_t *passes);

/* Full Frank-Wolfe (Alg. A.1) on the handle's plan: each iteration takes
 * every row's LMO vertex at once (S = (a_i e_{j*_i})_i, from the gap sweep),
 * and moves T <- (1 - gamma) T + gamma S with the decay step 2/(k+2) (k =
 * FW iteration counter of the handle, from 0) or the exact line search of
 * eq. AppenEq:SemiRelaxedFWStep, gamma = clip(<T - S, grad f> /
 * (w ||(T - S)^T 1||^2), 0, 1), as opt->step_rule says.  Shares the plan,
 * residual and masks with the block-coordinate entry points.  Each
 * iteration is one launch of the gap sweep, which applies the previous
 * iteration's step to each row as it reaches it and sums the vertex columns
 * in fixed point (order-independent: runs are reproducible); a last
 * launch applies the final step, so the plan is complete when the call's
 * work has run.
 *   iters        number of iterations (enqueued; no synchronisation).
 *   trace_gamma  device, iters doubles (optional): the step sizes. */
int srot_fw_steps(srot_handle *h, int64_t iters, double *trace_gamma);

/* Full Frank-Wolfe until the gap measured at an iterate is <= opt->eps or
 * opt->max_passes iterations have run.  out3 (host) = {g, f, D} at the last
 * iterate; *iters (host) = iterations run.  The stop test runs on the
 * device (a sweep that finds the run converged does nothing), so
 * iterations are queued in batches of 4, the next batch before the host
 * reads the last one's run state (as srot_solve).  Returns SROT_OK or
 * SROT_NOT_CONVERGED. */
int srot_fw_solve(srot_handle *h, double *out3, int64_t *iters);

/* Barycentric projection of the source points through the plan
 * (eq. barycentric_projection): Xhat_i = sum_j t_ij y_j / sum_j t_ij
 * (device, m x 3 float; a row without mass keeps x_i).  Needs X and Y at
 * srot_init.  Enqueued on the stream. */
int srot_barycentric(srot_handle *h, float *Xhat);

/* ------------------------------------------------------------------------
 * Batched solver: many independent problems of uneven sizes, each solved
 * from the initial plan to g <= eps (or max_passes) by Alg. 1 with the
 * per-pass gap test of Sec. 3.1, all in one graph launch.  Every problem
 * uses the options given (w, step rule, seed, eps, max_passes, gap_every);
 * problem p follows the trajectory srot_solve would take on it alone with
 * the same tile shape.  Stored FP32 cost and uniform sampling only; rows of
 * at most 4096 columns.
 * ------------------------------------------------------------------------ */
typedef struct srot_batch srot_batch;   /* opaque */

/* Bytes of device workspace for `count` problems of sizes m[p] x n[p]
 * (host arrays); 0 for invalid sizes. */
size_t srot_workspace_size_batched(int32_t count, const int64_t *m, const int64_t *n,
                                   const srot_options *opt);

/* Creates the batch.
 *   m, n     host, count sizes (1 <= m[p] <= 2^31 - 1, 1 <= n[p] <= 4096).
 *   c_off    host, count element offsets of each cost matrix in C, or NULL
 *            for matrices stored back to back.  An offset that is a
 *            multiple of 4 (with n[p] % 4 == 0) allows 16-byte cost loads.
 *   C        device, float: problem p's m x n cost matrix at C + c_off[p].
 *   a, b     device, doubles: the problems' weights back to back (problem
 *            p's a at offset sum_{q<p} m[q], its b at sum_{q<p} n[q]).
 *   workspace  device, >= srot_workspace_size_batched bytes, 256-byte aligned.
 *   opt      host; cost must be SROT_COST_F32, sampling SROT_UNIFORM.
 *   tune     0: each problem gets the tile shape srot_init would choose;
 *            1: per group of problems sharing that shape, every compiled
 *            candidate shape is timed on the group's widest problem with
 *            the fewest rows (one pass, second of two runs) and the
 *            fastest is kept.  Choices
 *            are cached per size class (default shape, widest row,
 *            16-byte rows) for the process, and in the file of JSON lines
 *            named by the environment variable SROT_TUNE_CACHE, if set
 *            (read once, appended to); a cached class is not timed again.
 *   stream   hipStream_t for all work of the batch.
 * Validates the inputs on the device, builds and instantiates the graph,
 * and synchronises.  Errors: SROT_EINVAL, SROT_ENOMEM, SROT_ENONFINITE,
 * SROT_EHIP. */
int srot_init_batched(srot_batch **out, int32_t count, const int64_t *m, const int64_t *n,
                      const int64_t *c_off, const float *C, const double *a, const double *b,
                      void *workspace, size_t ws_bytes, const srot_options *opt, int32_t tune,
                      void *stream);

/* Solves every problem from its initial plan (one graph launch: at most
 * four concurrent kernel launches, one per launch class of tile shapes) and
 * synchronises.  Host outputs, each optional: out3 (count x 3: g, f, D at
 * the last gap sweep), passes (count), status (count: SROT_OK or
 * SROT_NOT_CONVERGED).  Returns SROT_OK when every problem converged,
 * SROT_NOT_CONVERGED otherwise (SROT_EINVAL if a problem's kernel did not
 * match its tile shape, an internal error that leaves its results unset).  Each call also reorders the problems'
 * start order for the next call (longest measured run time first); a
 * problem's results do not depend on that order. */
int srot_solve_batched(srot_batch *h, double *out3, int64_t *passes, int32_t *status);

/* Copies problem p's plan (device, m x n double, zeros off the support) and
 * residual (device, n double); either may be NULL.  Enqueued on the stream. */
int srot_get_plan_batched(srot_batch *h, int32_t p, double *T_out, double *r_out);

/* Tile shape of every problem (host, count x 3: threads, columns per
 * thread, vector width) and, when tuned, the measured milliseconds per
 * block step of its group's shape (host, count floats, or NULL). */
int srot_get_tiles_batched(srot_batch *h, int32_t *tiles, float *ms_per_step);

void srot_destroy_batched(srot_batch *h);

/* Destroys the handle: its host memory, and the pinned readback words and
 * events of the solve loops (after the handle's stream has drained); the
 * caller frees its buffers. */
void srot_destroy(srot_handle *h);

const char *srot_strerror(int status);
const char *srot_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SROT_H */
