// Full Frank-Wolfe (Alg. A.1, step eq. AppenEq:SemiRelaxedFWStep) on the
// handle's plan, for gfx950.  An iteration is two launches.  The gap sweep
// in its FW form (srot_kernels.hip) applies the previous iteration's step
// to each row as it reaches it, measures every row's LMO vertex j*_i and
// its part of the gap g = <T - S, grad f> at the new plan, and adds a_i to
// the vertex column sum s_{j*_i} in fixed point (integer atomics, so the
// sums do not depend on the order the rows finish in).  The step kernel
// (one workgroup) adds the sweep's partial sums, then takes the line search
// on d = r + b - s (or the decay rule), writes the residual of the new plan
// and leaves the row updates to the next sweep, or stops when g <= eps.
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

// The step of Alg. A.1 after an FW sweep (that sweep's nb workgroup
// partials, the vertex column sums s in fixed point), by one workgroup: the
// sweep's final sums into scal[0..4] (gap_total), ||d||^2 with
// d = r + b - s (T^T 1 - S^T 1) in a fixed order, then either the stop of
// the run (gap <= eps, or a measuring-only sweep) or the exact line search
// gamma = clip(g / (w ||d||^2), 0, 1) (eq. AppenEq:SemiRelaxedFWStep) or the
// decay rule 2/(k+2), and r <- (1 - gamma)(r + b) + gamma s - b; the rows
// take the step in the next sweep (or the flush).  s is zeroed.
constexpr int FW_STEP_NT = 1024;

struct FwStepArgs {
    double eps;
    int32_t rule, allow_step;
    int64_t k;
    double *trace_gamma;
};

__global__ __launch_bounds__(FW_STEP_NT) void fw_step_kernel(int32_t n, double w, const double *__restrict__ b,
                                                             double *__restrict__ r,
                                                             unsigned long long *__restrict__ s_fixed,
                                                             const double *__restrict__ scale_p,
                                                             double *__restrict__ scal, int32_t *__restrict__ state,
                                                             const double *__restrict__ partials, int32_t nb,
                                                             FwStepArgs A)
{
    // up to FW_STEP_NT * TB columns the values stay in registers between
    // the two passes; wider rows read them again
    constexpr int NW = FW_STEP_NT / 64, TB = 8;
    __shared__ double sh[NW];
    __shared__ double s_gam;
    __shared__ int s_stop;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int done = state[0];
    const double inv = 1.0 / *scale_p;  // a power of two: exact
    double rv[TB], bv[TB], sv[TB];
    auto load = [&](int j0) {
#pragma unroll
        for (int u = 0; u < TB; ++u) {
            const int j = j0 + u * FW_STEP_NT;
            rv[u] = 0.0;
            bv[u] = 0.0;
            sv[u] = 0.0;
            if (j < n) {  // the same for every thread but the last chunk's
                rv[u] = r[j];
                bv[u] = b[j];
                sv[u] = (double)s_fixed[j] * inv;
            }
        }
    };
    load(tid);
    if (done) return;  // the run has reached its gap
    static_assert(FW_STEP_NT == GAP_FINAL_NT, "the final sums take the whole workgroup");
    gap_total(w, partials, nb, scal);  // thread 0 reads scal[0] below
    double x[1] = {0.0};
    for (int j0 = tid; j0 < n; j0 += FW_STEP_NT * TB) {
        if (j0 != tid) load(j0);
#pragma unroll
        for (int u = 0; u < TB; ++u) {
            const double d = (rv[u] + bv[u]) - sv[u];
            x[0] += (j0 + u * FW_STEP_NT < n) ? d * d : 0.0;
        }
    }
    wave_sum<1>(x);
    if (lane == 0) sh[wid] = x[0];
    __syncthreads();
    if (tid == 0) {
        double dd = sh[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) dd += sh[q];
        const double g = scal[0];
        const int stop = (!A.allow_step || g <= A.eps) ? 1 : 0;
        double gamma = 0.0;
        if (!stop) {
            const double num = g, den = w * dd;
            if (A.rule == SROT_DEC) gamma = 2.0 / ((double)A.k + 2.0);
            else if (!(num > 0.0)) gamma = 0.0;
            else if (den == 0.0 || num >= den) gamma = 1.0;
            else gamma = num / den;
            scal[5] = gamma;
            scal[6] = dd;
            if (A.trace_gamma) A.trace_gamma[0] = gamma;
            state[1] = 1;
            state[2] += 1;
        } else {
            state[1] = 0;
            if (g <= A.eps) state[0] = 1;
        }
        s_stop = stop;
        s_gam = gamma;
    }
    __syncthreads();
    const int stop = s_stop;
    const double gamma = s_gam;
    for (int j0 = tid; j0 < n; j0 += FW_STEP_NT * TB) {
        if (n > FW_STEP_NT * TB) load(j0);
#pragma unroll
        for (int u = 0; u < TB; ++u) {
            const int j = j0 + u * FW_STEP_NT;
            if (j < n) {
                if (!stop) r[j] = (1.0 - gamma) * (rv[u] + bv[u]) + gamma * sv[u] - bv[u];
                s_fixed[j] = 0ull;
            }
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
    hipLaunchKernelGGL(fw_step_kernel, dim3(1), dim3(FW_STEP_NT), 0, st, P.n, P.w, P.b, S.r, fw.s_fixed, fw.scale,
                       S.scalars, fw.state, (const double *)S.partials, nb, A);
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
