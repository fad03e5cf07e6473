// Internal declarations shared by the kernel and API translation units of
// libsrot.  Not part of the public interface (include/srot.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace srot {

// Everything a launch needs about one problem.  Device pointers only.
struct ProblemView {
    int32_t m, n;
    int32_t cost;          // SROT_COST_F32 / F64 / SQEUCLID
    const void *C;         // m x n (float or double), or nullptr
    const float *X;        // m x 3
    const float *Y;        // n x 3
    const float4 *Y4;      // y4n entries: Y padded to 16 bytes, then sentinel points (workspace), or nullptr
    int32_t y4n;           // entries of Y4 (y4_entries(n))
    const double *a;       // m
    const double *b;       // n
    double w;
    // When set, a device word: block-step and gap-sweep kernels return at
    // once while it is nonzero (set by the final sum of a sweep that found
    // g <= eps, so passes queued after it do nothing).
    const int32_t *stop = nullptr;
};

// Column ownership shared by the step and gap kernels of one handle: thread
// `tid` of an nt-thread workgroup owns columns
//   j(u) = ((u / vec) * nt + tid) * vec + u % vec,   u < cpt,
// i.e. groups of vec adjacent columns strided by nt groups.  The support of
// row i is kept as bitmasks: bit (u % 32) of word
//   mask[(i * words + u / 32) * nt + tid]
// is set iff T[i][j(u)] != 0, so kernels touch only nonzero entries.
struct Ownership {
    int32_t nt;     // threads per workgroup
    int32_t cpt;    // columns per thread
    int32_t vec;    // adjacent columns per group (1, 2 or 4)
    int32_t words;  // ceil(cpt / 32)
    int32_t reg;    // 1: register-resident residual variant (cpt <= 32)
};

// Device state carved out of the caller's workspace.
struct DeviceState {
    double *T;             // m x n dense plan
    double *r;             // n, residual T^T 1 - b
    uint32_t *mask;        // m x words x nt support bitmasks
    Ownership own;
    int32_t *idx;          // index buffer (idx_cap entries)
    int64_t idx_cap;
    double *row_G;         // m, min_j of the block gradient (gap sweep)
    int32_t *row_j;        // m, its lowest argmin
    double *row_g;         // m, per-row gap g_i
    double *partials;      // gap_blocks x 8 (gap sweep), or the FW step-size partials
    int32_t gap_blocks;
    double *scalars;       // 8: g, f, D, ...
    double *meas;          // 8: {g, f, D, <T,C>, ||r||^2} of a solve's last measuring sweep
    int32_t *flags;        // 8: [0] validation/index error flags, [1..3] FW run state, [4..5] solve stop word and
                           // pass, [6] team-chain error
    int64_t *slow_steps;   // 4: slow-path step counts of the last chain launch (diagnostic)
    double *adj_part;      // adjoint_slices_cap(m) x 3 x n per-slice column sums
    unsigned long long *team_rec;  // 2 x TEAM_MAX_MEMBERS x TEAM_REC_STRIDE exchange words of the team chain
    int32_t team;          // 1: block steps run on the team chain (chosen at init)
    double screen_delta2;  // 2 x error bound of the FP32 LMO screen (wide fused rows), 0 = unused
    double screen_err;     // error bound of the FP32 LMO screen of the screened chain, 0 = chain unused
    double *ga_w;          // m, stored block gaps of the gap-adaptive sampler
};

// Records a printf-style message as the calling thread's last error
// (srot_last_error) and returns code.
int fail(int code, const char *fmt, ...);

// Ownership chosen for an n-column problem with the given cost storage;
// aligned16: the cost matrix base is 16-byte aligned (honours
// SROT_CHAIN_VARIANT).
Ownership choose_ownership(int64_t n, int cost, bool aligned16);

// Launch wrappers (srot_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
hipError_t launch_validate(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_check_indices(const int32_t *idx, int64_t count, int32_t m, int32_t *flag,
                                hipStream_t stream);
hipError_t launch_init_plan(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_residual(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_mask_build(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_pad_points(const ProblemView &P, hipStream_t stream);
hipError_t launch_sample_uniform(uint64_t seed, int64_t k0, int64_t count, int32_t m,
                                 int32_t *out, hipStream_t stream);
hipError_t launch_sample_permute(uint64_t seed, int64_t p0, int64_t npasses, int32_t m,
                                 int32_t *out, hipStream_t stream);
hipError_t launch_chain(const ProblemView &P, const DeviceState &S, const int32_t *idx,
                        int64_t k0, int64_t nsteps, int rule, int32_t *trace_j,
                        double *trace_gamma, hipStream_t stream);
// The sweep and its final sums into S.scalars[0..4] (and out_dev[0..4],
// device memory, when given).
hipError_t launch_gap(const ProblemView &P, const DeviceState &S, hipStream_t stream, double *out_dev = nullptr);
// The same within a solve whose P.stop is stop_w (the sums also into
// S.meas): g <= eps sets stop_w[0] = 1 and stop_w[1] = pass; nothing runs
// once stop_w[0] is set.
hipError_t launch_gap_stop(const ProblemView &P, const DeviceState &S, hipStream_t stream, int32_t *stop_w, double eps,
                           int32_t pass);

// Screened-LMO chain (srot_screen.hip): stored FP32 cost in the 256 x {8,16}
// x 4 ownership.  launch_cost_bounds writes {max |c_ij|, max(sum a, max b)}
// to out2 (device; uses the gap partial buffer); the chain needs
// S.screen_err > 0.  SROT_LMO_SCREEN=0 in the environment turns it off.
bool screened_chain_supported(const ProblemView &P, const DeviceState &S);
bool screened_chain_enabled();
hipError_t launch_cost_bounds(const ProblemView &P, const DeviceState &S, double *out2, hipStream_t stream);
hipError_t launch_chain_screened(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                                 int64_t nsteps, int rule, int32_t *trace_j, double *trace_gamma,
                                 hipStream_t stream);
// Away (pairwise = 0) or pairwise (pairwise = 1) block steps on the screened
// chain (same conditions as above; ELS).
hipError_t launch_active_screened(const ProblemView &P, const DeviceState &S, int pairwise, const int32_t *idx,
                                  int64_t nsteps, int32_t *trace_j, int32_t *trace_away, double *trace_gamma,
                                  hipStream_t stream);
// {squared diameter of the points' bounding box, max(sum a, max b)} into out2.
hipError_t launch_screen_bounds(const ProblemView &P, double *out2, hipStream_t stream);

// Entries of the padded target points: n real points followed by sentinel
// points, at least one, and up to the columns the wide-row chain touches
// (8192, 16384 or 32768 when n exceeds 4096).
inline int64_t y4_entries(int64_t n)
{
    if (n <= 4096) return n + 1;
    int64_t cols = 8192;
    while (cols < n) cols *= 2;
    return cols > n ? cols : n + 1;
}

// Number of workgroups used by the gap sweep for an m-row problem.
int32_t gap_blocks_for(int64_t m);

// Block-step chain over a team of workgroups (srot_team.hip), rows of
// 4097 .. 1024 * TEAM_MAX_MEMBERS columns, any cost; the default there
// unless SROT_TEAM_CHAIN=0 is set in the environment at init.
// Gap sweep: threads per workgroup and the most workgroups (partials) of one
// sweep.
constexpr int GAP_NT = 256;
constexpr int GAP_NW = GAP_NT / 64;
constexpr int GAP_MAX_BLOCKS = 2048;

constexpr int TEAM_MAX_MEMBERS = 64;
constexpr int TEAM_REC_STRIDE = 16;  // 64-bit words per member record (one 128-byte line)
int team_members(int64_t n);
bool team_chain_supported(const ProblemView &P);
hipError_t launch_chain_team(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                             int64_t nsteps, int rule, int32_t *trace_j, double *trace_gamma,
                             hipStream_t stream);

// Adjoint at the current plan (srot_adjoint.hip): dC (m x n, float or double
// as the stored cost), dX (m x 3), dY (n x 3), da (m, reads row_G of the last
// gap sweep), db (n); each may be null.  g scales every output.
hipError_t launch_adjoint(const ProblemView &P, const DeviceState &S, double g, void *dC,
                          float *dX, float *dY, double *da, double *db, hipStream_t stream);
// Row slices of the adjoint's column sums (sizes DeviceState::adj_part).
int32_t adjoint_slices_cap(int64_t m);
// doubles of per-slice dY column sums (adj_part) that launch_adjoint uses
size_t adjoint_part_doubles(const ProblemView &P, const Ownership &own);

// Full Frank-Wolfe (Alg. A.1): per iteration the sweep and the step (one
// launch up to 4096 columns, two beyond).  The sweep of
// iteration k first applies the step of iteration k - 1 to each row as it
// reaches it (t_i <- (1 - gamma) t_i + gamma a_i e_{j*_i}, gamma in
// scalars[5], j*_i in row_j), then measures the row's vertex and gap at the
// new plan and adds a_i to the vertex column sum s = S^T 1 (fixed point,
// device-scope integer atomics: order-free, so the sums are reproducible).
// The step (srot_fw.hip) then either stops (gap <= eps, or a
// measuring-only sweep) or takes the line search on d = r + b - s, writes
// gamma and the new residual r <- (1 - gamma)(r + b) + gamma s - b, and
// leaves the row updates pending for the next sweep.  Once the done flag
// is set the sweep returns at once and the step takes the same stop again,
// so the host can queue iterations and read the flag once per batch.
struct FwSweep {
    int32_t *state;                 // [0] done, [1] a step is pending, [2] steps taken
    unsigned long long *s_fixed;    // n vertex column sums, zero between sweeps
    const double *scale;            // fixed-point scale of a (device, one double)
    double eps;                     // stop once the measured gap is <= eps (negative: never)
    int32_t rule;                   // SROT_ELS / SROT_DEC
    int32_t allow_step;             // 0: measure only
    int64_t k;                      // FW iteration counter (decay rule 2/(k+2))
    double *trace_gamma;            // device, one entry, or null
    int32_t *rb_words;              // pinned host memory, or null: the run state [0..2] after the step
    double *rb_sums;                // pinned host memory, or null: g, f, D of the sweep
};
// The sweep alone (its nb workgroup partials are left for gap_total).
hipError_t launch_gap_fw(const ProblemView &P, const DeviceState &S, const FwSweep &fw, hipStream_t stream, int *nb);
// One FW iteration: the FW sweep and the step kernel.
hipError_t launch_fw_iteration(const ProblemView &P, const DeviceState &S, const FwSweep &fw, hipStream_t stream);
// Before a run of FW sweeps: done / pending / steps cleared, s zeroed, the
// fixed-point scale of a computed (srot_fw.hip).
hipError_t launch_fw_reset(const ProblemView &P, const DeviceState &S, hipStream_t stream);
// After a run: applies a pending step to every row (srot_fw.hip).
hipError_t launch_fw_flush(const ProblemView &P, const DeviceState &S, hipStream_t stream);

// The plan in compressed sparse rows (srot_plan.hip): row counts from the
// support masks scanned into row_ptr (m + 1 entries; -1 from the first
// offset past 2^31 - 1 on), then each row's columns and entries.
hipError_t launch_plan_count(const ProblemView &P, const DeviceState &S, int32_t *row_ptr, hipStream_t stream);
hipError_t launch_plan_fill(const ProblemView &P, const DeviceState &S, const int32_t *row_ptr, int32_t *col,
                            double *val, hipStream_t stream);
// Device words of the FW run state inside DeviceState (flags[1..3]) and the
// scale (scalars[7]); s lives in adj_part.
inline FwSweep fw_sweep_args(const DeviceState &S, double eps, int rule, int allow_step, int64_t k,
                             double *trace_gamma)
{
    FwSweep f;
    f.state = S.flags + 1;
    f.s_fixed = reinterpret_cast<unsigned long long *>(S.adj_part);
    f.scale = S.scalars + 7;
    f.eps = eps;
    f.rule = rule;
    f.allow_step = allow_step;
    f.k = k;
    f.trace_gamma = trace_gamma;
    f.rb_words = nullptr;
    f.rb_sums = nullptr;
    return f;
}

// Block steps with away (pairwise = 0, Alg. A.2) or pairwise (pairwise = 1,
// Alg. A.3) directions (srot_variants.hip); rows of at most 4096 columns.
bool active_steps_supported(const DeviceState &S);
hipError_t launch_active_steps(const ProblemView &P, const DeviceState &S, int pairwise, const int32_t *idx,
                               int64_t nsteps, int32_t *trace_j, int32_t *trace_away, double *trace_gamma,
                               hipStream_t stream);

// Gap-adaptive sampling (srot_ga.hip, Alg. A.4): W lives in LDS during the
// inner iterations, so at most GA_MAX_ROWS rows; rows of at most 4096 columns.
constexpr int32_t GA_MAX_ROWS = 16384;
bool ga_supported(const ProblemView &P, const DeviceState &S);
// nsteps inner iterations; u (device, nsteps uniforms in [0, 1)) or, when
// null, u_s from output k0 + s of the block-index stream with key (seed, 0).
hipError_t launch_ga_steps(const ProblemView &P, const DeviceState &S, const double *u, uint64_t seed, int64_t k0,
                           int64_t nsteps, int rule, int32_t *trace_i, int32_t *trace_j, double *trace_gamma,
                           double *trace_g, hipStream_t stream);
// W_i <- max(src_i, 0) (src: device, m doubles), or W_i <- value when src is null.
hipError_t launch_ga_fill(const ProblemView &P, const DeviceState &S, const double *src, double value,
                          hipStream_t stream);

// Barycentric projection (srot_adjoint.hip): Xhat_i = sum_j t_ij y_j / sum_j t_ij.
hipError_t launch_barycentric(const ProblemView &P, const DeviceState &S, float *Xhat, hipStream_t stream);

}  // namespace srot
