// Block-coordinate Frank-Wolfe with gap-adaptive sampling (BCFW-GA,
// Alg. A.4, Sec. 4.2.1) for gfx950.  Every block keeps a stored gap W_i
// (eq. AppenEq:Gi, a large constant until the block is first visited); an
// inner iteration draws block i with probability W_i / sum W, takes the
// BCFW block step of Alg. 1 on it and stores that block's gap at the new
// plan; the global update (every block's gap recomputed) is the gap sweep's
// per-row output copied into W.
//
// One workgroup runs the inner iterations in order, with the column
// ownership of the handle (r in registers) and W in LDS: thread t owns the
// contiguous rows [t L, (t + 1) L), L = ceil(m / NT), and keeps their sum.
// The draw, for x = u * (sum of W):
//   * the chunk sums are scanned (inclusive) in thread order: within a wave
//     by a log-step scan, across waves by a running sum in wave order, so
//     every thread knows its chunk's upper end and the total;
//   * the drawn chunk is the lowest thread with a positive sum whose upper
//     end exceeds x (or, should rounding leave none, the last positive one),
//     and its wave walks its rows from the chunk's lower end to the first
//     positive weight whose running end exceeds x (else its last positive
//     weight), 64 rows at a time with the running ends from a wave scan.
// This is inversion of W / sum W with sums formed in another order than a
// plain running sum, so a draw can differ from one made with a running sum
// only where x lies within rounding of an interval end.  A block with zero
// weight is never drawn; with every weight zero, i = floor(u m).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
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

// Inclusive sum of x over the wave in lane order: log-step adds of the row
// shifts by 1, 2, 4, 8 within each row of 16 lanes (DPP; lanes with no
// source read 0), then each row adds the totals of the rows before it, in
// row order.  *prev gets the sum of the lanes below (0 in lane 0).
__device__ __forceinline__ double wave_incl_scan(double x, double *prev)
{
    x += dpp_f64<0x111>(x);  // row_shr:1
    x += dpp_f64<0x112>(x);  // row_shr:2
    x += dpp_f64<0x114>(x);  // row_shr:4
    x += dpp_f64<0x118>(x);  // row_shr:8
    const double r0 = readlane_f64(x, 15), r1 = readlane_f64(x, 31), r2 = readlane_f64(x, 47);
    const double o1 = r0, o2 = o1 + r1, o3 = o2 + r2;
    const int row = (threadIdx.x & 63) >> 4;
    x = row == 0 ? x : x + (row == 1 ? o1 : (row == 2 ? o2 : o3));
    *prev = dpp_f64<0x138>(x);  // wave_shr:1
    return x;
}

// Uniform double in [0, 1) from output k of the block-index stream.
__device__ __forceinline__ double philox_unit(uint64_t seed, int64_t k)
{
    return (double)(philox_output(seed, (uint64_t)k) >> 11) * 0x1.0p-53;
}

template <int NT, int CPT, int VEC, int COST>
__global__ __launch_bounds__(NT) void ga_step_kernel(ProblemView P, double *__restrict__ T,
                                                     double *__restrict__ rg, uint32_t *__restrict__ M,
                                                     double *__restrict__ Wg, const double *__restrict__ u_in,
                                                     uint64_t seed, int64_t k0, int64_t nsteps, int rule,
                                                     int32_t *__restrict__ tr_i, int32_t *__restrict__ tr_j,
                                                     double *__restrict__ tr_gamma, double *__restrict__ tr_g)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NW = NT / 64;
    extern __shared__ double s_W[];  // the m stored block gaps
    __shared__ double s_tot[2][NW];
    __shared__ int s_cand[2][NW], s_last[2][NW];
    __shared__ double s_v[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_sum[2][NW][3];
    __shared__ double s_v2[2][NW];
    __shared__ int s_j2[2][NW];
    __shared__ double s_sum2[2][NW][1];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int m = P.m, n = P.n;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;
    const int L = (m + NT - 1) / NT;
    const int q0 = min(m, tid * L), q1 = min(m, q0 + L);

    // this thread's chunk of W: copy, sum (row order), last positive row
    double cs = 0.0;
    int lastpos = -1;
    for (int q = q0; q < q1; ++q) {
        const double v = Wg[q];
        s_W[q] = v;
        cs += v;
        lastpos = v > 0.0 ? q : lastpos;
    }
    double r[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        r[u] = (j < n) ? rg[j] : 0.0;
    }

    // the uniform of each step is formed during the step before (while
    // that step's row is in flight)
    double u_next = nsteps > 0 ? (u_in ? u_in[0] : philox_unit(seed, k0)) : 0.0;
    for (int64_t s = 0; s < nsteps; ++s) {
        const int par = (int)(s & 1);
        double u = u_next;
        u = (u >= 0.0 && u < 1.0) ? u : 0.0;

        // ---- draw i with probability W_i / sum W ----
        double below;
        const double inc = wave_incl_scan(cs, &below);
        if (lane == 63) s_tot[par][wid] = inc;
        __syncthreads();
        double run = 0.0, off = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q == wid) off = run;
            run += s_tot[par][q];
        }
        const double total = run;  // the same bits in every thread
        int i;
        if (!(total > 0.0)) {
            const int q = (int)(u * (double)m);
            i = q < m ? q : m - 1;
        } else {
            double x = u * total;
            if (x >= total) x = __longlong_as_double(__double_as_longlong(total) - 1);
            const double hi = off + inc;
            const double lo = off + (lane ? below : 0.0);
            const unsigned long long fb = __ballot(cs > 0.0 && hi > x);
            const unsigned long long pb = __ballot(cs > 0.0);
            int cand = -1;
            if (fb) {
                // the chunk of the wave's first lane with hi > x, walked by
                // the whole wave 64 rows at a time: each lane takes one row,
                // the running ends come from a wave scan added to the
                // chunk's lower end; the first positive weight whose end
                // exceeds x, else the chunk's last positive weight
                const int fl = __ffsll((long long)fb) - 1;
                const int q0f = min(m, (wid * 64 + fl) * L), q1f = min(m, q0f + L);
                double base = readlane_f64(lo, fl);
                int lp = -1;
                for (int qb = q0f; qb < q1f && cand < 0; qb += 64) {  // uniform over the wave
                    const int q = qb + lane;
                    const double wq = q < q1f ? s_W[q] : 0.0;
                    double prev;
                    const double end = base + wave_incl_scan(wq, &prev);
                    const unsigned long long hit = __ballot(wq > 0.0 && end > x);
                    const unsigned long long pos = __ballot(wq > 0.0);
                    if (hit) cand = qb + __ffsll((long long)hit) - 1;
                    if (pos) lp = qb + 63 - __clzll((long long)pos);
                    base = readlane_f64(end, 63);
                }
                if (cand < 0) cand = lp;
            }
            int lastw = -1;
            if (pb) lastw = __builtin_amdgcn_readlane(lastpos, 63 - __clzll((long long)pb));
            if (lane == 0) { s_cand[par][wid] = cand; s_last[par][wid] = lastw; }
            __syncthreads();
            i = -1;
#pragma unroll
            for (int q = 0; q < NW; ++q) i = (i < 0) ? s_cand[par][q] : i;
#pragma unroll
            for (int q = NW - 1; q >= 0; --q) i = (i < 0) ? s_last[par][q] : i;
            i = i < 0 ? 0 : i;  // not reached: a positive total has a positive chunk
        }

        // ---- BCFW block step on row i (Alg. 1) ----
        const double ai = P.a[i];
        const size_t base = (size_t)i * (size_t)n;
        const uint32_t mk = M[(size_t)i * NT + tid];
        CT cv[CPT];
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if constexpr (FUSED) { x0 = P.X[3 * i]; x1 = P.X[3 * i + 1]; x2 = P.X[3 * i + 2]; }
        else load_cost_row<NT, CPT, VEC, CT>(C + base, n, tid, cv);
        double t[CPT], cc[CPT];
        // the row's plan entries are requested with its mask word and cost
        // (one round trip instead of two) and kept where the mask has a bit
        double tl[CPT];
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) {
            const int j = owned_col<NT, VEC>(u2, tid);
            tl[u2] = T[base + (j < n ? j : n - 1)];
        }
        if (s + 1 < nsteps) u_next = u_in ? u_in[s + 1] : philox_unit(seed, k0 + s + 1);
        double best = INFINITY;
        int bj = 0x7fffffff;
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) {
            const int j = owned_col<NT, VEC>(u2, tid);
            const int jc = j < n ? j : n - 1;
            t[u2] = (mk & (1u << u2)) ? tl[u2] : 0.0;
            if constexpr (FUSED) cc[u2] = sqdist(x0, x1, x2, P.Y[3 * jc], P.Y[3 * jc + 1], P.Y[3 * jc + 2]);
            else cc[u2] = (double)cv[u2];
            const double v = (j < n) ? cc[u2] + w * r[u2] : INFINITY;
            if (v < best) { best = v; bj = j; }
        }
        block_argmin<NW>(best, bj, s_v[par], s_j[par]);
        const double G = best;
        const int jstar = bj;
        // only the support contributes (t >= 0, sums from +0: leaving out
        // t = 0 changes no bit); column slots no lane holds are skipped by
        // the whole wave, and only the support and j* can change
        const int jg = jstar / VEC;
        const int us = ((jg % NT) == tid) ? (jg / NT) * VEC + (jstar % VEC) : -1;
        uint32_t nz = 0u;
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) nz |= (t[u2] != 0.0 ? 1u : 0u) << u2;
        const uint32_t wnz = wave_or_u32(nz);
        const uint32_t wtouch = wave_or_u32(nz | (us >= 0 ? 1u << us : 0u));
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) {
            if (!((wnz >> u2) & 1u)) continue;  // uniform over the wave
            const bool st = (owned_col<NT, VEC>(u2, tid) == jstar);
            acc[0] += t[u2] * ((cc[u2] + w * r[u2]) - G);
            acc[1] += st ? 0.0 : t[u2] * t[u2];
            acc[2] = st ? t[u2] : acc[2];
        }
        block_sum<NW, 3>(acc, s_sum[par]);
        const double gamma = step_size(rule, k0 + s, m, w, acc[0], acc[1], acc[2], ai);
        const double gadd = gamma * ai;
        uint32_t nm = mk;
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) {
            if (!((wtouch >> u2) & 1u)) continue;  // uniform over the wave
            const double tn = blend(t[u2], gamma, (u2 == us) ? gadd : 0.0);
            if (tn != t[u2]) T[base + owned_col<NT, VEC>(u2, tid)] = tn;
            r[u2] += tn - t[u2];
            t[u2] = tn;
            nm = (tn != 0.0) ? (nm | (1u << u2)) : (nm & ~(1u << u2));
        }
        if (nm != mk) M[(size_t)i * NT + tid] = nm;

        // ---- the block's gap at the new plan (eq. AppenEq:Gi) ----
        double best2 = INFINITY;
        int bj2 = 0x7fffffff;
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) {
            const int j = owned_col<NT, VEC>(u2, tid);
            const double v = (j < n) ? cc[u2] + w * r[u2] : INFINITY;
            if (v < best2) { best2 = v; bj2 = j; }
        }
        block_argmin<NW>(best2, bj2, s_v2[par], s_j2[par]);
        double gs[1] = {0.0};
        const uint32_t wnm = wave_or_u32(nm);
#pragma unroll
        for (int u2 = 0; u2 < CPT; ++u2) {
            if (!((wnm >> u2) & 1u)) continue;  // uniform over the wave
            gs[0] += t[u2] * ((cc[u2] + w * r[u2]) - best2);
        }
        block_sum<NW, 1>(gs, s_sum2[par]);
        const double gi = gs[0];
        if (tid == i / L) {
            s_W[i] = gi;
            Wg[i] = gi;
            cs = 0.0;
            lastpos = -1;
            // the chunk sum again in row order; the reads are independent,
            // so unrolling lets them be requested together
#pragma unroll 8
            for (int q = q0; q < q1; ++q) {
                const double v = s_W[q];
                cs += v;
                lastpos = v > 0.0 ? q : lastpos;
            }
        }
        if (tid == 0) {
            if (tr_i) tr_i[s] = i;
            if (tr_j) tr_j[s] = jstar;
            if (tr_gamma) tr_gamma[s] = gamma;
            if (tr_g) tr_g[s] = gi;
        }
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int j = owned_col<NT, VEC>(u, tid);
        if (j < n) rg[j] = r[u];
    }
}

// W_i <- max(g_i, 0) from the gap sweep (global update), or W_i <- value;
// nothing once a solve has stopped (stop set).
__global__ void ga_fill_kernel(int32_t m, const double *__restrict__ src, double value, double *__restrict__ W,
                               const int32_t *__restrict__ stop)
{
    if (stop && *stop) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        W[i] = src ? fmax(src[i], 0.0) : value;
}

#define SROT_GA_V1(X) \
    X(64, 2, 1) X(64, 4, 1) X(128, 4, 1) X(256, 4, 1) X(256, 8, 1) X(256, 16, 1)
#define SROT_GA_V2(X) \
    X(64, 2, 2) X(64, 4, 2) X(128, 4, 2) X(256, 4, 2) X(256, 8, 2) X(256, 16, 2)
#define SROT_GA_V4(X) \
    X(64, 4, 4) X(128, 4, 4) X(256, 4, 4) X(256, 8, 4) X(256, 16, 4)

// The wide-row ownership of a handle for 4097-8192 columns.
bool wide_ga_layout(const Ownership &o) { return !o.reg && o.nt == 512 && o.vec == 1 && o.words == 1 && o.cpt <= 16; }

template <int COST>
hipError_t launch_ga_cost(const ProblemView &P, const DeviceState &S, const double *u, uint64_t seed, int64_t k0,
                          int64_t nsteps, int rule, int32_t *ti, int32_t *tj, double *tg, double *tgi,
                          hipStream_t st)
{
    const Ownership &o = S.own;
    const size_t lds = sizeof(double) * (size_t)P.m;
#define SROT_GAK(NT_, CPT_, VEC_)                                                                   \
    if (o.nt == NT_ && o.cpt == CPT_ && o.vec == VEC_) {                                            \
        const void *fn = (const void *)&ga_step_kernel<NT_, CPT_, VEC_, COST>;                      \
        hipError_t e_ = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        if (e_ != hipSuccess) return e_;                                                            \
        hipLaunchKernelGGL((ga_step_kernel<NT_, CPT_, VEC_, COST>), dim3(1), dim3(NT_), lds, st, P, S.T, \
                           S.r, S.mask, S.ga_w, u, seed, k0, nsteps, rule, ti, tj, tg, tgi);        \
        return hipGetLastError();                                                                   \
    }
    SROT_GA_V1(SROT_GAK)
    if constexpr (COST == SROT_COST_F32) { SROT_GA_V4(SROT_GAK) }
    if constexpr (COST == SROT_COST_F64) { SROT_GA_V2(SROT_GAK) }
#undef SROT_GAK
    // rows of 4097-8192 columns: the handle's wide ownership (512 threads,
    // at most 16 single columns each, one mask word) as a 512 x 16 x 1 tile;
    // slots past the row's width lie beyond column n
    if (wide_ga_layout(o)) {
        const void *fn = (const void *)&ga_step_kernel<512, 16, 1, COST>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((ga_step_kernel<512, 16, 1, COST>), dim3(1), dim3(512), lds, st, P, S.T, S.r, S.mask,
                           S.ga_w, u, seed, k0, nsteps, rule, ti, tj, tg, tgi);
        return hipGetLastError();
    }
    return hipErrorInvalidConfiguration;
}

}  // namespace

bool ga_supported(const ProblemView &P, const DeviceState &S)
{
    return ((S.own.reg && S.own.nt <= 256) || wide_ga_layout(S.own)) && P.m <= GA_MAX_ROWS;
}

hipError_t launch_ga_steps(const ProblemView &P, const DeviceState &S, const double *u, uint64_t seed, int64_t k0,
                           int64_t nsteps, int rule, int32_t *trace_i, int32_t *trace_j, double *trace_gamma,
                           double *trace_g, hipStream_t stream)
{
    if (nsteps <= 0) return hipSuccess;
    switch (P.cost) {
    case SROT_COST_F32:
        return launch_ga_cost<SROT_COST_F32>(P, S, u, seed, k0, nsteps, rule, trace_i, trace_j, trace_gamma,
                                             trace_g, stream);
    case SROT_COST_F64:
        return launch_ga_cost<SROT_COST_F64>(P, S, u, seed, k0, nsteps, rule, trace_i, trace_j, trace_gamma,
                                             trace_g, stream);
    default:
        return launch_ga_cost<SROT_COST_SQEUCLID>(P, S, u, seed, k0, nsteps, rule, trace_i, trace_j,
                                                  trace_gamma, trace_g, stream);
    }
}

hipError_t launch_ga_fill(const ProblemView &P, const DeviceState &S, const double *src, double value,
                          hipStream_t stream)
{
    const int blocks = (int)std::min<int64_t>((P.m + 255) / 256, 1024);
    hipLaunchKernelGGL(ga_fill_kernel, dim3(blocks), dim3(256), 0, stream, P.m, src, value, S.ga_w, P.stop);
    return hipGetLastError();
}

}  // namespace srot
