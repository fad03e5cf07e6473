// Full Frank-Wolfe (Alg. A.1, step eq. AppenEq:SemiRelaxedFWStep) on the
// handle's plan, for gfx950.  An iteration is three launches.  The gap sweep
// in its FW form (srot_kernels.hip) applies the previous iteration's step
// to each row as it reaches it, measures every row's LMO vertex j*_i and
// its part of the gap g = <T - S, grad f> at the new plan, and adds a_i to
// the vertex column sum s_{j*_i} in fixed point (integer atomics, so the
// sums do not depend on the order the rows finish in).  Two launches over
// the columns then add the sweep's partial sums and ||d||^2 with
// d = r + b - s, take the line search (or the decay rule), write the
// residual of the new plan and leave the row updates to the next sweep, or
// stop when g <= eps.
// Here also: the reset before a run (state, s, the fixed-point scale of a)
// and the flush after it (a pending step applied to every row).  The host
// is not involved between iterations.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/srot.h"
#include "srot_device.h"
#include "srot_internal.h"

namespace srot {

namespace {

constexpr int FW_NT = 256;

// One workgroup: done / pending / steps cleared, s zeroed, and the scale
// 2^(62 - e) with sum a < 2^e, so that every fixed-point vertex sum (at most
// sum a scaled) stays below 2^62 while a_i keeps its rounding error of
// 2^-63 sum a or less.
__global__ __launch_bounds__(FW_NT) void fw_reset_kernel(int32_t m, int32_t n, const double *__restrict__ a,
                                                         int32_t *__restrict__ state,
                                                         unsigned long long *__restrict__ s_fixed,
                                                         double *__restrict__ scale)
{
    __shared__ double sh[FW_NT / 64];
    const int tid = threadIdx.x;
    for (int j = tid; j < n; j += FW_NT) s_fixed[j] = 0ull;
    double x[1] = {0.0};
    for (int i = tid; i < m; i += FW_NT) x[0] += a[i];
    wave_sum<1>(x);
    if ((tid & 63) == 0) sh[tid >> 6] = x[0];
    __syncthreads();
    if (tid == 0) {
        double t = sh[0];
#pragma unroll
        for (int q = 1; q < FW_NT / 64; ++q) t += sh[q];
        int e = 0;
        if (t > 0.0) frexp(t, &e);
        *scale = ldexp(1.0, 62 - e);
        state[0] = 0;
        state[1] = 0;
        state[2] = 0;
    }
}

// The step of Alg. A.1 after an FW sweep: up to 4096 columns one
// workgroup holding every column in registers; wider rows in two launches
// spread over the columns (one workgroup could not keep enough loads in
// flight: 25 us at 16384 columns).
//
// fw_dd_kernel: ||d||^2 of one slice of columns per workgroup, d = r + b - s
// (T^T 1 - S^T 1, s the vertex column sums in fixed point), into
// dd_part[blockIdx.x]; nothing once the run is done.
//
// fw_update_kernel: every workgroup adds the sweep's nb partials
// (gap_total) and the dd partials in the same fixed order, so all take the
// same decision: the stop of the run (gap <= eps, or a measuring-only
// sweep) or the exact line search gamma = clip(g / (w ||d||^2), 0, 1)
// (eq. AppenEq:SemiRelaxedFWStep) or the decay rule 2/(k+2); then each
// updates its columns, r <- (1 - gamma)(r + b) + gamma s - b, and zeroes s
// there.  Workgroup 0 alone writes the final sums and the run state.  Once
// the run is done the sweep and fw_dd_kernel leave their partials as they
// were, so a later fw_update_kernel takes the same stop again.  The rows
// take the step in the next sweep (or the flush).
constexpr int FW_DD_NT = 256, FW_DD_PER = 4;                // columns per thread and batch
constexpr int FW_DD_COLS = FW_DD_NT * FW_DD_PER;            // columns per workgroup and batch
constexpr int FW_DD_MAX_BLOCKS = 256;
constexpr int FW_STEP_NT = 1024, FW_UP_MAX_BLOCKS = 64;
constexpr int FW_SELF_PER = 4, FW_SELF_COLS = FW_STEP_NT * FW_SELF_PER;  // one launch up to 4096 columns

struct FwStepArgs {
    double eps;
    int32_t rule, allow_step;
    int64_t k;
    double *trace_gamma;
    int32_t *rb_words;  // pinned host memory (the run's readback slot), or null
    double *rb_sums;
};

int fw_dd_blocks(int32_t n) { return (int)std::min<int64_t>(((int64_t)n + FW_DD_COLS - 1) / FW_DD_COLS, FW_DD_MAX_BLOCKS); }
int fw_up_blocks(int32_t n) { return (int)std::min<int64_t>(((int64_t)n + FW_STEP_NT - 1) / FW_STEP_NT, FW_UP_MAX_BLOCKS); }

__global__ __launch_bounds__(FW_DD_NT) void fw_dd_kernel(int32_t n, const double *__restrict__ b,
                                                         const double *__restrict__ r,
                                                         const unsigned long long *__restrict__ s_fixed,
                                                         const double *__restrict__ scale_p,
                                                         const int32_t *__restrict__ state,
                                                         double *__restrict__ dd_part)
{
    if (state[0]) return;  // the run has reached its gap
    constexpr int NW = FW_DD_NT / 64;
    __shared__ double sh[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const double inv = 1.0 / *scale_p;  // a power of two: exact
    const int64_t stride = (int64_t)gridDim.x * FW_DD_NT;
    double x[1] = {0.0};
    for (int64_t j0 = (int64_t)blockIdx.x * FW_DD_NT + tid; j0 < n; j0 += stride * FW_DD_PER) {
        double rv[FW_DD_PER], bv[FW_DD_PER], sv[FW_DD_PER];
#pragma unroll
        for (int u = 0; u < FW_DD_PER; ++u) {
            const int64_t j = j0 + u * stride;
            const bool in = j < n;
            rv[u] = in ? r[j] : 0.0;
            bv[u] = in ? b[j] : 0.0;
            sv[u] = in ? (double)s_fixed[j] * inv : 0.0;
        }
#pragma unroll
        for (int u = 0; u < FW_DD_PER; ++u) {
            const double d = (rv[u] + bv[u]) - sv[u];
            x[0] += d * d;
        }
    }
    wave_sum<1>(x);
    if (lane == 0) sh[wid] = x[0];
    __syncthreads();
    if (tid == 0) {
        double t = sh[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) t += sh[q];
        dd_part[blockIdx.x] = t;
    }
}

template <bool SELF>
__global__ __launch_bounds__(FW_STEP_NT) void fw_update_kernel(int32_t n, double w, const double *__restrict__ b,
                                                               double *__restrict__ r,
                                                               unsigned long long *__restrict__ s_fixed,
                                                               const double *__restrict__ scale_p,
                                                               double *__restrict__ scal, int32_t *__restrict__ state,
                                                               const double *__restrict__ partials, int32_t nb,
                                                               const double *__restrict__ dd_part, int32_t nbd,
                                                               FwStepArgs A)
{
    constexpr int PER = SELF ? FW_SELF_PER : 1;  // columns per thread held in registers
    constexpr int NW = FW_STEP_NT / 64;
    __shared__ double s_sums[5];
    __shared__ double s_dd[NW];
    __shared__ double s_gam;
    __shared__ int s_stop;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool lead = blockIdx.x == 0;
    const double inv = 1.0 / *scale_p;
    // the first columns and the dd partials (wave 0, fixed order) are
    // requested before the sweep's partials are added
    const int64_t stride = (int64_t)gridDim.x * FW_STEP_NT;
    const int64_t jf = (int64_t)blockIdx.x * FW_STEP_NT + tid;
    double rv[PER], bv[PER], sv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int64_t j = jf + u * stride;
        const bool in = j < n;
        rv[u] = in ? r[j] : 0.0;
        bv[u] = in ? b[j] : 0.0;
        sv[u] = in ? (double)s_fixed[j] * inv : 0.0;
    }
    double dd[1] = {0.0};
    if constexpr (SELF) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const double d = (rv[u] + bv[u]) - sv[u];
            dd[0] += d * d;
        }
    } else if (tid < 64) {
        for (int k = lane; k < nbd; k += 64) dd[0] += dd_part[k];
    }
    static_assert(FW_STEP_NT == GAP_FINAL_NT, "the final sums take the whole workgroup");
    gap_total(w, partials, nb, lead ? scal : s_sums);
    if (SELF || tid < 64) wave_sum<1>(dd);
    if (SELF && lane == 0) s_dd[wid] = dd[0];
    __syncthreads();  // thread 0 has written the final sums
    if (tid == 0) {
        if constexpr (SELF) {
            dd[0] = s_dd[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) dd[0] += s_dd[q];
        }
        const double g = lead ? scal[0] : s_sums[0];
        const int stop = (!A.allow_step || g <= A.eps) ? 1 : 0;
        double gamma = 0.0;
        if (!stop) {
            const double num = g, den = w * dd[0];
            if (A.rule == SROT_DEC) gamma = 2.0 / ((double)A.k + 2.0);
            else if (!(num > 0.0)) gamma = 0.0;
            else if (den == 0.0 || num >= den) gamma = 1.0;
            else gamma = num / den;
        }
        if (lead) {
            if (!stop) {
                scal[5] = gamma;
                scal[6] = dd[0];
                if (A.trace_gamma) A.trace_gamma[0] = gamma;
                state[1] = 1;
                state[2] += 1;
            } else {
                state[1] = 0;
                if (g <= A.eps) state[0] = 1;
            }
            // the run state and the sums straight into the host's readback
            // slot (visible to the host once the launch has completed)
            if (A.rb_words) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A.rb_words[c] = state[c];
                    A.rb_sums[c] = scal[c];
                }
            }
        }
        s_stop = stop;
        s_gam = gamma;
    }
    __syncthreads();
    const int stop = s_stop;
    const double gamma = s_gam;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int64_t j = jf + u * stride;
        if (j < n) {
            if (!stop) r[j] = (1.0 - gamma) * (rv[u] + bv[u]) + gamma * sv[u] - bv[u];
            s_fixed[j] = 0ull;
        }
    }
    if constexpr (!SELF) {
        for (int64_t j = jf + stride; j < n; j += stride) {
            const double rj = r[j], bj = b[j], sj = (double)s_fixed[j] * inv;
            if (!stop) r[j] = (1.0 - gamma) * (rj + bj) + gamma * sj - bj;
            s_fixed[j] = 0ull;
        }
    }
}

// A step left pending by the last sweep of a run, on every row.
__global__ __launch_bounds__(FW_NT) void fw_flush_kernel(int32_t m, int32_t n, const double *__restrict__ a,
                                                         const int32_t *__restrict__ row_j,
                                                         const double *__restrict__ scal,
                                                         const int32_t *__restrict__ state, Ownership own,
                                                         double *__restrict__ T, uint32_t *__restrict__ M)
{
    if (!state[1]) return;
    const double gamma = scal[5];
    for (int i = blockIdx.x; i < m; i += gridDim.x) fw_apply_row(i, n, gamma, a[i], row_j[i], own, T, M, threadIdx.x, FW_NT);
}

}  // namespace

hipError_t launch_fw_reset(const ProblemView &P, const DeviceState &S, hipStream_t st)
{
    const FwSweep f = fw_sweep_args(S, 0.0, 0, 0, 0, nullptr);
    hipLaunchKernelGGL(fw_reset_kernel, dim3(1), dim3(FW_NT), 0, st, P.m, P.n, P.a, f.state, f.s_fixed,
                       S.scalars + 7);
    return hipGetLastError();
}

hipError_t launch_fw_iteration(const ProblemView &P, const DeviceState &S, const FwSweep &fw, hipStream_t st)
{
    int nb = 0;
    hipError_t e = launch_gap_fw(P, S, fw, st, &nb);
    if (e != hipSuccess) return e;
    FwStepArgs A;
    A.eps = fw.eps;
    A.rule = fw.rule;
    A.allow_step = fw.allow_step;
    A.k = fw.k;
    A.trace_gamma = fw.trace_gamma;
    A.rb_words = fw.rb_words;
    A.rb_sums = fw.rb_sums;
    if (P.n <= FW_SELF_COLS) {
        // one workgroup holds every column: ||d||^2 and the update in one launch
        hipLaunchKernelGGL(fw_update_kernel<true>, dim3(1), dim3(FW_STEP_NT), 0, st, P.n, P.w, P.b, S.r, fw.s_fixed,
                           fw.scale, S.scalars, fw.state, (const double *)S.partials, nb, (const double *)nullptr,
                           0, A);
        return hipGetLastError();
    }
    // the dd partials sit behind s (n + n / 1024 entries at most of the 3n
    // the region holds)
    double *dd_part = S.adj_part + P.n;
    const int nbd = fw_dd_blocks(P.n);
    hipLaunchKernelGGL(fw_dd_kernel, dim3(nbd), dim3(FW_DD_NT), 0, st, P.n, P.b, (const double *)S.r,
                       (const unsigned long long *)fw.s_fixed, fw.scale, (const int32_t *)fw.state, dd_part);
    hipLaunchKernelGGL(fw_update_kernel<false>, dim3(fw_up_blocks(P.n)), dim3(FW_STEP_NT), 0, st, P.n, P.w, P.b,
                       S.r, fw.s_fixed, fw.scale, S.scalars, fw.state, (const double *)S.partials, nb,
                       (const double *)dd_part, nbd, A);
    return hipGetLastError();
}

hipError_t launch_fw_flush(const ProblemView &P, const DeviceState &S, hipStream_t st)
{
    const int rb = (int)std::min<int64_t>(P.m, 4096);
    hipLaunchKernelGGL(fw_flush_kernel, dim3(rb), dim3(FW_NT), 0, st, P.m, P.n, P.a, (const int32_t *)S.row_j,
                       (const double *)S.scalars, (const int32_t *)(S.flags + 1), S.own, S.T, S.mask);
    return hipGetLastError();
}

}  // namespace srot
