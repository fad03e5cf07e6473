// Block steps with away steps (Alg. A.2, BCAFW) and pairwise steps
// (Alg. A.3, BCPFW) of Sec. 4.1, for gfx950.  A row t_i in a_i * simplex is
// the combination of the vertices a_i e_j with coefficients alpha_j =
// t_ij / a_i; its active set is the support, which the support bitmasks of
// the block-coordinate kernels already hold.  Per step, with g = c_i + w r:
//   FW vertex   js = lowest-index argmin of g (all columns);
//   away vertex ja = lowest-index argmax of g over the support;
//   BCAFW: the FW direction a_i e_js - t_i (gamma_max = 1) when its slope
//          sum t (g - g_js) is at least that of the away direction
//          t_i - a_i e_ja, sum t (g_ja - g) (gamma_max = alpha/(1 - alpha)),
//          and always with one atom or ja = js (the away direction is then
//          zero; alpha is 1 only up to rounding);
//   BCPFW: d = a_i (e_js - e_ja), gamma_max = alpha_ja;
// gamma = clip(-<g, d> / (w ||d||^2), 0, gamma_max) (eq. SemiRelaxedBCAFWStep);
// a step reaching gamma_max on an away or pairwise direction empties atom ja
// exactly.  One workgroup runs the steps in order with the column ownership
// of the handle (r in registers); a step is three workgroup reductions: the
// FW vertex, the away vertex, and seven sums over the support.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/srot.h"
#include "srot_device.h"
#include "srot_internal.h"

namespace srot {

namespace {

// OR of a 32-bit word over the wave, the same in every lane.
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v)
{
    v |= (uint32_t)dpp_i32<DPP_QUAD_XOR1>((int)v);
    v |= (uint32_t)dpp_i32<DPP_QUAD_XOR2>((int)v);
    v |= (uint32_t)dpp_i32<DPP_HALF_MIRROR>((int)v);
    v |= (uint32_t)dpp_i32<DPP_MIRROR>((int)v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) | (uint32_t)__builtin_amdgcn_readlane((int)v, 16) |
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) | (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

template <int NT, int CPT, int VEC, int COST, int PAIR>
__global__ __launch_bounds__(NT) void active_step_kernel(ProblemView P, double *__restrict__ T,
                                                         double *__restrict__ rg, uint32_t *__restrict__ M,
                                                         const int32_t *__restrict__ idx, int64_t nsteps,
                                                         int32_t *__restrict__ trace_j,
                                                         int32_t *__restrict__ trace_away,
                                                         double *__restrict__ trace_gamma)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NW = NT / 64;
    __shared__ double s_v[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_v2[2][NW];
    __shared__ int s_j2[2][NW];
    __shared__ double s_sum[2][NW][7];
    const int tid = threadIdx.x;
    const int n = P.n;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;

    double r[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        r[u] = (j < n) ? rg[j] : 0.0;
    }
    // One step ahead: the next row's cost entries, mask word and a_i are
    // requested at the start of a step, its plan entries once the mask has
    // arrived (after the step's first reductions); when the next step
    // revisits the row, the entries come from the update instead.
    auto load_row = [&](int i, CT (&cv)[CPT], float (&x)[3], uint32_t &mk, double &ai) {
        ai = P.a[i];
        mk = M[(size_t)i * NT + tid];
        if constexpr (FUSED) { x[0] = P.X[3 * i]; x[1] = P.X[3 * i + 1]; x[2] = P.X[3 * i + 2]; }
        else load_cost_row<NT, CPT, VEC, CT>(C + (size_t)i * (size_t)n, n, tid, cv);
    };
    auto gather = [&](int i, uint32_t mk, double (&t)[CPT]) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = owned_col<NT, VEC>(u, tid);
            t[u] = (mk & (1u << u)) ? T[(size_t)i * (size_t)n + j] : 0.0;
        }
    };
    int i = idx[0];
    CT cv[CPT];
    float x[3] = {0.f, 0.f, 0.f};
    uint32_t mk;
    double ai, t[CPT];
    load_row(i, cv, x, mk, ai);
    gather(i, mk, t);
    int inext = nsteps > 1 ? idx[1] : i;

    for (int64_t s = 0; s < nsteps; ++s) {
        CT cvn[CPT];
        float xn[3] = {0.f, 0.f, 0.f};
        uint32_t mkn;
        double an, tnx[CPT];
        load_row(inext, cvn, xn, mkn, an);
        const int inext2 = (s + 2 < nsteps) ? idx[s + 2] : inext;
        const size_t base = (size_t)i * (size_t)n;

        double vv[CPT];
        double best = INFINITY, nb = INFINITY;
        int bj = 0x7fffffff, nj = 0x7fffffff;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = owned_col<NT, VEC>(u, tid);
            const int jc = j < n ? j : n - 1;
            double c;
            if constexpr (FUSED) c = sqdist(x[0], x[1], x[2], P.Y[3 * jc], P.Y[3 * jc + 1], P.Y[3 * jc + 2]);
            else c = (double)cv[u];
            vv[u] = c + w * r[u];
            const double v = (j < n) ? vv[u] : INFINITY;
            if (v < best) { best = v; bj = j; }
            if (t[u] > 0.0 && -vv[u] < nb) { nb = -vv[u]; nj = j; }
        }
        block_argmin<NW>(best, bj, s_v[s & 1], s_j[s & 1]);
        block_argmin<NW>(nb, nj, s_v2[s & 1], s_j2[s & 1]);
        const double G = best, V = -nb;
        const int js = bj, ja = nj;
        if (inext != i) gather(inext, mkn, tnx);

        // P1 = sum t (g - G), P2 = sum t (V - g), Q1 = sum_{j != js} t^2,
        // Q2 = sum_{j != ja} t^2, t_js, t_ja, number of atoms
        // Only the support contributes (t >= 0 and every sum starts at +0, so
        // leaving out columns with t = 0 changes no bit); a column index u no
        // lane of the wave holds in its support is skipped by the whole wave.
        uint32_t nz = 0u, touch = 0u;  // support; support, FW and away vertex
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = owned_col<NT, VEC>(u, tid);
            nz |= (t[u] != 0.0 ? 1u : 0u) << u;
            touch |= (t[u] != 0.0 || j == js || j == ja ? 1u : 0u) << u;
        }
        const uint32_t wnz = wave_or_u32(nz), wtouch = wave_or_u32(touch);
        double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            if (!((wnz >> u) & 1u)) continue;  // uniform over the wave
            const int j = owned_col<NT, VEC>(u, tid);
            const bool on = t[u] > 0.0;
            acc[0] += t[u] * (vv[u] - G);
            acc[1] += on ? t[u] * (V - vv[u]) : 0.0;
            acc[2] += (j == js) ? 0.0 : t[u] * t[u];
            acc[3] += (j == ja) ? 0.0 : t[u] * t[u];
            acc[4] = (j == js) ? t[u] : acc[4];
            acc[5] = (j == ja) ? t[u] : acc[5];
            acc[6] += on ? 1.0 : 0.0;
        }
        block_sum<NW, 7>(acc, s_sum[s & 1]);
        const double tjs = acc[4], tja = acc[5];
        const double alpha = tja / ai;
        bool fw_dir = false;
        double num, den, gmax;
        if constexpr (PAIR) {
            num = (js != ja) ? ai * (V - G) : 0.0;
            den = (js != ja) ? w * (2.0 * ai * ai) : 0.0;
            gmax = alpha;
        } else {
            fw_dir = acc[6] == 1.0 || ja == js || acc[0] >= acc[1];
            if (fw_dir) {
                num = acc[0];
                den = w * (acc[2] + (tjs - ai) * (tjs - ai));
                gmax = 1.0;
            } else {
                num = acc[1];
                den = w * (acc[3] + (tja - ai) * (tja - ai));
                gmax = alpha / (1.0 - alpha);
            }
        }
        double gamma;
        if (!(num > 0.0)) gamma = 0.0;
        else if (den == 0.0) gamma = gmax;
        else gamma = num / den < gmax ? num / den : gmax;
        const bool drop = !fw_dir && gamma > 0.0 && gamma == gmax;

        // update this thread's entries, r and the support bits (only the
        // support and the two vertices can change)
        uint32_t nm = mk;
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            if (!((wtouch >> u) & 1u)) continue;  // uniform over the wave
            const int j = owned_col<NT, VEC>(u, tid);
            double tn;
            if (fw_dir) tn = (1.0 - gamma) * t[u] + ((j == js) ? gamma * ai : 0.0);
            else if constexpr (PAIR) tn = (js == ja) ? t[u] : ((j == js) ? t[u] + gamma * ai : ((j == ja) ? t[u] - gamma * ai : t[u]));
            else tn = (1.0 + gamma) * t[u] - ((j == ja) ? gamma * ai : 0.0);
            if (drop && j == ja) tn = 0.0;
            if (j < n && tn != t[u]) T[base + j] = tn;
            r[u] += tn - t[u];
            nm = (tn != 0.0) ? (nm | (1u << u)) : (nm & ~(1u << u));
            t[u] = tn;
        }
        if (nm != mk) M[(size_t)i * NT + tid] = nm;
        if (tid == 0) {
            if (trace_j) trace_j[s] = js;
            if (trace_away) trace_away[s] = fw_dir ? -1 - ja : ja;
            if (trace_gamma) trace_gamma[s] = gamma;
        }

        // the next step's row
        if (inext == i) {
            mkn = nm;
#pragma unroll
            for (int u = 0; u < CPT; ++u) tnx[u] = t[u];
        }
        i = inext;
        inext = inext2;
        mk = mkn;
        ai = an;
#pragma unroll
        for (int u = 0; u < CPT; ++u) { cv[u] = cvn[u]; t[u] = tnx[u]; }
        x[0] = xn[0]; x[1] = xn[1]; x[2] = xn[2];
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        if (j < n) rg[j] = r[u];
    }
}

#define SROT_VAR_V1(X) \
    X(64, 2, 1) X(64, 4, 1) X(128, 4, 1) X(256, 4, 1) X(256, 8, 1) X(256, 16, 1)
#define SROT_VAR_V2(X) \
    X(64, 2, 2) X(64, 4, 2) X(128, 4, 2) X(256, 4, 2) X(256, 8, 2) X(256, 16, 2)
#define SROT_VAR_V4(X) \
    X(64, 4, 4) X(128, 4, 4) X(256, 4, 4) X(256, 8, 4) X(256, 16, 4)

// The wide-row ownership of a handle for 4097-8192 columns.
bool wide_active_layout(const Ownership &o) { return !o.reg && o.nt == 512 && o.vec == 1 && o.words == 1 && o.cpt <= 16; }

template <int COST, int PAIR>
hipError_t launch_active_cost(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t nsteps,
                              int32_t *tj, int32_t *ta, double *tg, hipStream_t st)
{
    const Ownership &o = S.own;
#define SROT_ACT(NT_, CPT_, VEC_)                                                                  \
    if (o.nt == NT_ && o.cpt == CPT_ && o.vec == VEC_) {                                           \
        hipLaunchKernelGGL((active_step_kernel<NT_, CPT_, VEC_, COST, PAIR>), dim3(1), dim3(NT_), 0, st, \
                           P, S.T, S.r, S.mask, idx, nsteps, tj, ta, tg);                          \
        return hipGetLastError();                                                                  \
    }
    SROT_VAR_V1(SROT_ACT)
    if constexpr (COST == SROT_COST_F32) { SROT_VAR_V4(SROT_ACT) }
    if constexpr (COST == SROT_COST_F64) { SROT_VAR_V2(SROT_ACT) }
#undef SROT_ACT
    // rows of 4097-8192 columns: the handle's wide ownership (512 threads,
    // at most 16 single columns each, one mask word) is the layout of the
    // 512 x 16 x 1 kernel; slots past the row's width lie beyond column n
    if (wide_active_layout(o)) {
        hipLaunchKernelGGL((active_step_kernel<512, 16, 1, COST, PAIR>), dim3(1), dim3(512), 0, st, P, S.T, S.r,
                           S.mask, idx, nsteps, tj, ta, tg);
        return hipGetLastError();
    }
    return hipErrorInvalidConfiguration;
}

}  // namespace

bool active_steps_supported(const DeviceState &S)
{
    const Ownership &o = S.own;
    return (o.reg && o.nt <= 256) || wide_active_layout(o);
}

hipError_t launch_active_steps(const ProblemView &P, const DeviceState &S, int pairwise, const int32_t *idx,
                               int64_t nsteps, int32_t *trace_j, int32_t *trace_away, double *trace_gamma,
                               hipStream_t stream)
{
    if (nsteps <= 0) return hipSuccess;
    // stored FP32 cost of 513-4096 columns: the screened chain's stepper
    if (S.screen_err > 0.0 && screened_chain_supported(P, S))
        return launch_active_screened(P, S, pairwise, idx, nsteps, trace_j, trace_away, trace_gamma, stream);
    switch (P.cost) {
    case SROT_COST_F32:
        return pairwise ? launch_active_cost<SROT_COST_F32, 1>(P, S, idx, nsteps, trace_j, trace_away, trace_gamma, stream)
                        : launch_active_cost<SROT_COST_F32, 0>(P, S, idx, nsteps, trace_j, trace_away, trace_gamma, stream);
    case SROT_COST_F64:
        return pairwise ? launch_active_cost<SROT_COST_F64, 1>(P, S, idx, nsteps, trace_j, trace_away, trace_gamma, stream)
                        : launch_active_cost<SROT_COST_F64, 0>(P, S, idx, nsteps, trace_j, trace_away, trace_gamma, stream);
    default:
        return pairwise ? launch_active_cost<SROT_COST_SQEUCLID, 1>(P, S, idx, nsteps, trace_j, trace_away, trace_gamma, stream)
                        : launch_active_cost<SROT_COST_SQEUCLID, 0>(P, S, idx, nsteps, trace_j, trace_away, trace_gamma, stream);
    }
}

}  // namespace srot
