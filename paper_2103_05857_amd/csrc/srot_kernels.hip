// HIP kernels for block-coordinate Frank-Wolfe on quadratic semi-relaxed OT
// (Fukunaga & Kasai, arXiv:2103.05857), written for gfx950 (CDNA4, wave64).
//
// Orientation: T is m x n, rows are the blocks (T 1 = a exact), the relaxed
// marginal is the column sum with residual r = T^T 1 - b, and w is the
// penalty weight (the paper's 1/lambda).
//
// Column ownership: thread tid of an NT-thread workgroup owns columns
// j = u * NT + tid.  Loads of a cost row are then coalesced, the residual
// entries r_j a thread owns never move, and every update of t_ij and r_j is
// done by its owner: no atomics, no cross-thread hazards on T or r.  The
// support of each row is a bitmask per (row, thread) (see Ownership), so a
// step reads the cost row plus only the nonzero plan entries (a BCFW row
// without away steps holds a handful of atoms).
//
// Kernels
//   chain_kernel      one workgroup runs a sequence of BCFW block steps
//                     (Alg. 1) with r in registers (n <= NT * 32).  The next
//                     four rows (cost row, mask, a_i) and the next two rows'
//                     plan entries are prefetched: the row sequence is known
//                     in advance.  A step is two workgroup reductions: the
//                     LMO argmin, then the line-search sums over the support.
//   chain_glb_kernel  same step for wider rows: r in global memory (L2).
//   gap_sweep_kernel  per-pass duality-gap sweep (Thm 2): each wave streams
//                     whole cost rows (HBM bound); the last workgroup adds
//                     the partials in a fixed order.
//   sample kernels    counter-based Philox4x64-10 block indices.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <algorithm>
#include <type_traits>

#include "../../include/srot.h"
#include "srot_internal.h"
#include "srot_device.h"

namespace srot {

template <int NT, int CPT, int VEC, int COST, bool TRACE>
__global__ __launch_bounds__(NT) void chain_kernel(ProblemView P, double *__restrict__ T,
                                                   double *__restrict__ rg,
                                                   uint32_t *__restrict__ M,
                                                   const int32_t *__restrict__ idx, int64_t k0,
                                                   int64_t nsteps, int rule,
                                                   int32_t *__restrict__ trace_j,
                                                   double *__restrict__ trace_gamma,
                                                   int64_t *__restrict__ slow_steps)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    const int64_t slow = chain_run<NT, CPT, VEC, COST, TRACE>(P, T, rg, M, idx, k0, nsteps, rule,
                                                             trace_j, trace_gamma);
    if (threadIdx.x == 0) {
        slow_steps[0] = slow;
        slow_steps[2] = SROT_CHAIN_PREFETCH;
    }
}

// ---------------------------------------------------------------------------
// Block-step chain for wide rows: r in global memory; thread tid owns columns
// j = u * GLB_NT + tid for all u, reads and writes only those entries of r,
// T and its mask words.
// ---------------------------------------------------------------------------
constexpr int GLB_NT = 512;

template <int COST>
__global__ __launch_bounds__(GLB_NT) void chain_glb_kernel(ProblemView P, double *__restrict__ T,
                                                           double *__restrict__ rg,
                                                           uint32_t *__restrict__ M, int words,
                                                           const int32_t *__restrict__ idx,
                                                           int64_t k0, int64_t nsteps, int rule,
                                                           int32_t *__restrict__ trace_j,
                                                           double *__restrict__ trace_gamma,
                                                           int64_t *__restrict__ stats)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NT = GLB_NT, NW = NT / 64;
    if (threadIdx.x == 0) stats[2] = SROT_CHAIN_GLOBAL;
    __shared__ double s_v[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_sum[2][NW][4];
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;

    auto cost = [&](int i, int j, float x0, float x1, float x2) -> double {
        if constexpr (FUSED) return sqdist(x0, x1, x2, P.Y[3 * j], P.Y[3 * j + 1], P.Y[3 * j + 2]);
        else return (double)C[(size_t)i * (size_t)n + j];
    };

    for (int64_t s = 0; s < nsteps; ++s) {
        const int i = idx[s];
        const double ai = P.a[i];
        const size_t base = (size_t)i * (size_t)n;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if constexpr (FUSED) { x0 = P.X[3 * i]; x1 = P.X[3 * i + 1]; x2 = P.X[3 * i + 2]; }
        double best = INFINITY;
        int bj = 0x7fffffff;
        for (int j = tid; j < n; j += NT) {
            const double v = cost(i, j, x0, x1, x2) + w * rg[j];
            if (v < best) { best = v; bj = j; }
        }
        block_argmin<NW>(best, bj, s_v[s & 1], s_j[s & 1]);
        const double G = best;
        const int jstar = bj;

        uint32_t *Mi = M + (size_t)i * words * NT + tid;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int wd = 0; wd < words; ++wd) {
            uint32_t mk = Mi[(size_t)wd * NT];
            while (mk) {
                const int b = __ffs(mk) - 1;
                mk &= mk - 1u;
                const int j = (wd * 32 + b) * NT + tid;
                const double t = T[base + j];
                const double v = cost(i, j, x0, x1, x2) + w * rg[j];
                acc[0] += t * (v - G);
                if (j == jstar) acc[2] = t;
                else acc[1] += t * t;
            }
        }
        block_sum<NW, 4>(acc, s_sum[s & 1]);
        const double gamma = step_size(rule, k0 + s, m, w, acc[0], acc[1], acc[2], ai);

        for (int wd = 0; wd < words; ++wd) {
            const uint32_t mk = Mi[(size_t)wd * NT];
            uint32_t nm = mk, todo = mk;
            const int ustar = jstar / NT - wd * 32;
            const bool st_here = (jstar % NT) == tid && ustar >= 0 && ustar < 32;
            if (st_here) todo |= (1u << ustar);
            while (todo) {
                const int b = __ffs(todo) - 1;
                todo &= todo - 1u;
                const int j = (wd * 32 + b) * NT + tid;
                const bool on = (mk >> b) & 1u;
                const double told = on ? T[base + j] : 0.0;
                const double tn = (1.0 - gamma) * told + ((j == jstar) ? gamma * ai : 0.0);
                if (tn != told) {
                    T[base + j] = tn;
                    rg[j] += tn - told;
                }
                nm = (tn != 0.0) ? (nm | (1u << b)) : (nm & ~(1u << b));
            }
            if (nm != mk) Mi[(size_t)wd * NT] = nm;
        }
        if (tid == 0) {
            if (trace_j) trace_j[s] = jstar;
            if (trace_gamma) trace_gamma[s] = gamma;
        }
    }
}

// ---------------------------------------------------------------------------
// Block-step chain for wide rows with the fused cost (4096 < n <= 32768).
// One 512-thread workgroup; thread tid owns columns j = u * 512 + tid and
// keeps their target points in registers.  The LMO is found in two stages:
//   1. a screen in FP32: v'_j = fl(c'_j + w r32_j) with c'_j the FP32 squared
//      distance and r32 an FP32 copy of r kept in LDS (owner-only access);
//      every |v'_j - v_j| <= delta (bound below), so with m' = min_j v'_j
//      every column whose exact value can reach the exact minimum satisfies
//      v'_j <= m' + 2 delta;
//   2. those candidates (typically one or two) are evaluated exactly in FP64
//      (squared distance of the FP32 points in double, r_j from the FP64
//      residual in global memory) and the lowest-index exact minimum wins.
// The step is therefore exactly the FP64 BCFW step of Alg. 1.  Error bound
// (u = 2^-24, round to nearest): the FP32 distance carries at most 5.01 u c,
// the product w r at most 2.01 u |w r|, the final fused add u |v|; delta is
// taken as 8 u (Cmax + |w| Rmax) with Cmax the squared diameter of the
// points' bounding box and Rmax = max(sum a, max b) >= |r_j|, and the
// threshold is rounded upwards.  The line search and the update run on the
// row's support (bitmasks), as in the other chain kernels; r is updated in
// FP64 (global) and its FP32 copy alongside.
// ---------------------------------------------------------------------------
constexpr int WIDE_NT = 512;
constexpr int WIDE_KA = 2;
constexpr int WIDE_MAX_N = WIDE_NT * 64;
constexpr int WIDE_B = 16;  // columns per streamed batch of target points

__device__ __forceinline__ float wave_min_f32(float v)
{
    v = fminf(v, __int_as_float(dpp_i32<DPP_QUAD_XOR1>(__float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_i32<DPP_QUAD_XOR2>(__float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_i32<DPP_HALF_MIRROR>(__float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_i32<DPP_MIRROR>(__float_as_int(v))));
    float m = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    m = fminf(m, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16)));
    m = fminf(m, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32)));
    m = fminf(m, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48)));
    return m;
}

template <int CPTK, int YMODE, bool TRACE>
__global__ __launch_bounds__(WIDE_NT) void chain_wide_kernel(ProblemView P, double *__restrict__ T,
                                                             double *__restrict__ rg,
                                                             uint32_t *__restrict__ M, int words,
                                                             const int32_t *__restrict__ idx, int64_t k0,
                                                             int64_t nsteps, int rule,
                                                             int32_t *__restrict__ trace_j,
                                                             double *__restrict__ trace_gamma,
                                                             double delta2, int64_t *__restrict__ stats)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    constexpr int NW = WIDE_NT / 64;
    if (threadIdx.x == 0) stats[2] = SROT_CHAIN_WIDE;
    extern __shared__ float r32[];
    __shared__ float s_m[2][NW];
    __shared__ double s_v[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_sum[2][NW][3];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const float w32 = (float)w;
    const float4 *__restrict__ Y4 = P.Y4;

    // r32 holds CPTK * WIDE_NT entries (zero past column n - 1), so the
    // screen reads it at constant offsets; a column past n - 1 gets a point
    // 3e18 away from every coordinate, whose screen value (~2.7e37, finite)
    // never reaches the minimum of the real columns (every thread owns at
    // least one real column: n > WIDE_NT)
    // YMODE 1: the thread's target points in registers; 0: streamed from L2
    constexpr int YR = YMODE == 1 ? CPTK : 1;
    float y0[YR], y1[YR], y2[YR];
#pragma unroll
    for (int u = 0; u < CPTK; ++u) {
        const int j = u * WIDE_NT + tid;
        if constexpr (YMODE == 1) {
            const float4 yv = Y4[j < n ? j : n - 1];
            y0[u] = (j < n) ? yv.x : 3e18f;
            y1[u] = (j < n) ? yv.y : 3e18f;
            y2[u] = (j < n) ? yv.z : 3e18f;
        }
        r32[j] = (j < n) ? (float)rg[j] : 0.0f;
    }

    // YMODE 0: the thread's points are streamed in batches of WIDE_B
    // columns, double buffered; the batches repeat every step (the points do
    // not depend on the row), so the last batch of a step requests the
    // first batch of the next one.
    constexpr int YB = YMODE == 0 ? WIDE_B : 1;
    static_assert(YMODE == 1 || CPTK % (2 * WIDE_B) == 0, "whole pairs of batches");
    float4 ya[YB], yb2[YB];
    // raw buffer loads: the lane's offset in a vector register, the batch's
    // column offset in a scalar one; entries past n hold sentinel points
    const __amdgpu_buffer_rsrc_t rs_y = buf_rsrc(Y4, (unsigned)P.y4n * 16u);
    auto issue_batch = [&](float4 (&q)[YB], int ub) {
#pragma unroll
        for (int e = 0; e < YB; ++e)
            q[e] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  rs_y, tid * 16, (ub + e) * WIDE_NT * 16, 0));
    };
    if constexpr (YMODE == 0) issue_batch(ya, 0);

    // row data of the next step (index, point, weight, this thread's mask
    // words) is requested one step ahead; a mask is forwarded when the next
    // step revisits the row just updated
    const int64_t last = nsteps - 1;
    int i_nx = idx[0];
    int i_nn = idx[last > 0 ? 1 : 0];
    double a_nx = P.a[i_nx];
    float x_nx[3] = {P.X[3 * i_nx], P.X[3 * i_nx + 1], P.X[3 * i_nx + 2]};
    uint32_t m_nx0 = M[(size_t)i_nx * words * WIDE_NT + tid];
    uint32_t m_nx1 = words > 1 ? M[((size_t)i_nx * words + 1) * WIDE_NT + tid] : 0u;
    for (int64_t s = 0; s < nsteps; ++s) {
        const int i = i_nx;
        const double ai = a_nx;
        const size_t base = (size_t)i * (size_t)n;
        const float x0 = x_nx[0], x1 = x_nx[1], x2 = x_nx[2];
        uint32_t *Mi = M + (size_t)i * words * WIDE_NT + tid;
        const uint32_t mk0 = m_nx0;
        const uint32_t mk1 = m_nx1;

        // support entries at the WIDE_KA lowest mask bits: plan value, FP64
        // residual and target point, requested before the screen
        int aj[WIDE_KA];
        double at[WIDE_KA], ar[WIDE_KA];
        float ay[WIDE_KA][3];
        uint32_t rest0 = mk0, rest1 = mk1;
#pragma unroll
        for (int k = 0; k < WIDE_KA; ++k) {
            int u = -1;
            if (rest0) { u = __ffs(rest0) - 1; rest0 &= rest0 - 1u; }
            else if (rest1) { u = 32 + __ffs(rest1) - 1; rest1 &= rest1 - 1u; }
            aj[k] = u >= 0 ? u * WIDE_NT + tid : -1;
            const int jj = aj[k] >= 0 ? aj[k] : 0;
            const double tv = T[base + jj];
            at[k] = aj[k] >= 0 ? tv : 0.0;
            ar[k] = rg[jj];
            const float4 yv = Y4[jj];
            ay[k][0] = yv.x; ay[k][1] = yv.y; ay[k][2] = yv.z;
        }
        const bool more = (rest0 | rest1) != 0u;

        i_nx = i_nn;
        i_nn = idx[s + 2 < last ? s + 2 : last];
        a_nx = P.a[i_nx];
        x_nx[0] = P.X[3 * i_nx]; x_nx[1] = P.X[3 * i_nx + 1]; x_nx[2] = P.X[3 * i_nx + 2];
        m_nx0 = M[(size_t)i_nx * words * WIDE_NT + tid];
        m_nx1 = words > 1 ? M[((size_t)i_nx * words + 1) * WIDE_NT + tid] : 0u;

        // stage 1: FP32 screen, smallest and second smallest value per thread
        float b1 = INFINITY, b2 = INFINITY;
        int u1 = 0;
        // running smallest (b1, at column u1; ties keep the lower column) and
        // second smallest b2: with b1 <= b2 the median of {b1, b2, v} is the
        // new second smallest
        auto screen = [&](int u, float v) {
            u1 = (v < b1) ? u : u1;
            b2 = __builtin_amdgcn_fmed3f(b1, b2, v);
            b1 = fminf(b1, v);
        };
        if constexpr (YMODE == 1) {
#pragma unroll
            for (int u = 0; u < CPTK; ++u) {
                const float d0 = x0 - y0[u], d1 = x1 - y1[u], d2 = x2 - y2[u];
                const float c = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
                screen(u, fmaf(w32, r32[u * WIDE_NT + tid], c));
                __builtin_amdgcn_sched_barrier(0);  // the point registers stay the only per-column state
            }
        } else {
            auto consume = [&](const float4 (&q)[YB], int ub) {
                const float *rb = r32 + ub * WIDE_NT + tid;
                float rr[YB];
#pragma unroll
                for (int e = 0; e < YB; ++e) rr[e] = rb[e * WIDE_NT];
#pragma unroll
                for (int e = 0; e < YB; ++e) {
                    const float d0 = x0 - q[e].x, d1 = x1 - q[e].y, d2 = x2 - q[e].z;
                    const float c = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
                    screen(ub + e, fmaf(w32, rr[e], c));
                }
            };
            // one pair of batches per iteration; the scheduling barriers keep
            // each batch's loads one batch ahead of its use (hoisting them all
            // would need registers for every point of the step)
#pragma unroll 1
            for (int ub = 0; ub < CPTK; ub += 2 * WIDE_B) {
                issue_batch(yb2, ub + WIDE_B);
                __builtin_amdgcn_sched_barrier(0);
                consume(ya, ub);
                __builtin_amdgcn_sched_barrier(0);
                issue_batch(ya, (ub + 2 * WIDE_B) % CPTK);
                __builtin_amdgcn_sched_barrier(0);
                consume(yb2, ub + WIDE_B);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        const int j1 = u1 * WIDE_NT + tid;
        const double r1 = rg[j1];
        const float4 yb = Y4[j1];
        float mw = wave_min_f32(b1);
        if (lane == 0) s_m[s & 1][wid] = mw;
        __syncthreads();
        float mb = s_m[s & 1][0];
#pragma unroll
        for (int k = 1; k < NW; ++k) mb = fminf(mb, s_m[s & 1][k]);
        const float thr = __double2float_ru((double)mb + delta2);

        // stage 2: exact FP64 values of the candidates.  A thread with a single
        // candidate evaluates it; one with several (rare) takes the exact
        // minimum over all its columns, which contains them.
        double best = INFINITY;
        int bj = 0x7fffffff;
        if (b1 <= thr) {
            if (b2 <= thr) {
                for (int j = tid; j < n; j += WIDE_NT) {
                    const float4 yv = Y4[j];
                    const double v = sqdist(x0, x1, x2, yv.x, yv.y, yv.z) + w * rg[j];
                    if (v < best) { best = v; bj = j; }
                }
            } else {
                best = sqdist(x0, x1, x2, yb.x, yb.y, yb.z) + w * r1;
                bj = j1;
            }
        }
        block_argmin<NW>(best, bj, s_v[s & 1], s_j[s & 1]);
        const double G = best;
        const int jstar = bj;

        // line-search sums over this thread's support (Alg. 1 step size)
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < WIDE_KA; ++k) {
            if (aj[k] >= 0) {
                const double v = sqdist(x0, x1, x2, ay[k][0], ay[k][1], ay[k][2]) + w * ar[k];
                const bool st = aj[k] == jstar;
                acc[0] += at[k] * (v - G);
                acc[1] += st ? 0.0 : at[k] * at[k];
                acc[2] = st ? at[k] : acc[2];
            }
        }
        if (more) {
            uint32_t q0 = rest0, q1 = rest1;
            while (q0 | q1) {
                int u;
                if (q0) { u = __ffs(q0) - 1; q0 &= q0 - 1u; }
                else { u = 32 + __ffs(q1) - 1; q1 &= q1 - 1u; }
                const int j = u * WIDE_NT + tid;
                const double t = T[base + j];
                const float4 yv = Y4[j];
                const double v = sqdist(x0, x1, x2, yv.x, yv.y, yv.z) + w * rg[j];
                const bool st = j == jstar;
                acc[0] += t * (v - G);
                acc[1] += st ? 0.0 : t * t;
                acc[2] = st ? t : acc[2];
            }
        }
        block_sum<NW, 3>(acc, s_sum[s & 1]);
        const double gamma = step_size(rule, k0 + s, m, w, acc[0], acc[1], acc[2], ai);
        const double gadd = gamma * ai;

        // t_i <- (1 - gamma) t_i + gamma a_i e_j*, r <- r + (t_i new - t_i old)
        uint32_t nm0 = mk0, nm1 = mk1;
        bool star_in = false;
        auto set_bit = [&](int u, bool on) {
            if (u < 32) nm0 = on ? (nm0 | (1u << u)) : (nm0 & ~(1u << u));
            else nm1 = on ? (nm1 | (1u << (u - 32))) : (nm1 & ~(1u << (u - 32)));
        };
#pragma unroll
        for (int k = 0; k < WIDE_KA; ++k) {
            if (aj[k] >= 0) {
                const bool st = aj[k] == jstar;
                star_in |= st;
                const double tn = blend(at[k], gamma, st ? gadd : 0.0);
                if (tn != at[k]) {
                    T[base + aj[k]] = tn;
                    const double rn = ar[k] + (tn - at[k]);
                    rg[aj[k]] = rn;
                    r32[aj[k]] = (float)rn;
                }
                set_bit(aj[k] / WIDE_NT, tn != 0.0);
            }
        }
        if (more) {
            uint32_t q0 = rest0, q1 = rest1;
            while (q0 | q1) {
                int u;
                if (q0) { u = __ffs(q0) - 1; q0 &= q0 - 1u; }
                else { u = 32 + __ffs(q1) - 1; q1 &= q1 - 1u; }
                const int j = u * WIDE_NT + tid;
                const double t = T[base + j];
                const bool st = j == jstar;
                star_in |= st;
                const double tn = blend(t, gamma, st ? gadd : 0.0);
                if (tn != t) {
                    T[base + j] = tn;
                    const double rn = rg[j] + (tn - t);
                    rg[j] = rn;
                    r32[j] = (float)rn;
                }
                set_bit(u, tn != 0.0);
            }
        }
        if ((jstar % WIDE_NT) == tid && !star_in) {
            const double tsn = blend(0.0, gamma, gadd);
            if (tsn != 0.0) {
                T[base + jstar] = tsn;
                const double rn = rg[jstar] + tsn;
                rg[jstar] = rn;
                r32[jstar] = (float)rn;
                set_bit(jstar / WIDE_NT, true);
            }
        }
        if (nm0 != mk0) Mi[0] = nm0;
        if (words > 1 && nm1 != mk1) Mi[WIDE_NT] = nm1;
        if (i_nx == i) { m_nx0 = nm0; m_nx1 = nm1; }
        if constexpr (TRACE) {
            if (tid == 0) {
                if (trace_j) trace_j[s] = jstar;
                if (trace_gamma) trace_gamma[s] = gamma;
            }
        }
    }
}

// Bounds used by the wide-row screen: bounding box of all points and
// max(sum a, max b).  One workgroup; out = {sq. box diameter, Rmax}.
__global__ __launch_bounds__(256) void screen_bounds_kernel(ProblemView P, double *__restrict__ out)
{
    __shared__ double sh[256];
    double lo[3], hi[3], sa = 0.0, mb = 0.0;
    for (int d = 0; d < 3; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; }
    for (int i = threadIdx.x; i < P.m; i += 256) {
        for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], (double)P.X[3 * i + d]); hi[d] = fmax(hi[d], (double)P.X[3 * i + d]); }
        sa += P.a[i];
    }
    for (int j = threadIdx.x; j < P.n; j += 256) {
        for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], (double)P.Y[3 * j + d]); hi[d] = fmax(hi[d], (double)P.Y[3 * j + d]); }
        mb = fmax(mb, P.b[j]);
    }
    auto reduce = [&](double v, int op) -> double {  // 0: min, 1: max, 2: sum
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                const double o = sh[threadIdx.x + s];
                sh[threadIdx.x] = op == 0 ? fmin(sh[threadIdx.x], o) : (op == 1 ? fmax(sh[threadIdx.x], o) : sh[threadIdx.x] + o);
            }
            __syncthreads();
        }
        const double r = sh[0];
        __syncthreads();
        return r;
    };
    double diam2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double l = reduce(lo[d], 0), h = reduce(hi[d], 1);
        diam2 += (h - l) * (h - l);
    }
    const double suma = reduce(sa, 2), maxb = reduce(mb, 1);
    if (threadIdx.x == 0) {
        out[0] = diam2;
        out[1] = fmax(suma, maxb);
    }
}

// ---------------------------------------------------------------------------
// Gap sweep (Thm 2, eq. AppenEq:Gi, dual of App. D), streaming the cost once.
// A wave takes R rows at a time (row groups strided over the grid), with no
// workgroup barrier per row:
//   G_i = min_j v_ij, v_ij = c_ij + w r_j (lowest argmin j*_i),
//   g_i = sum_j t_ij (v_ij - G_i),  lin_i = sum_j t_ij c_ij  (support only).
// Lane l meets columns j = (q * 64 + l) * VEC + e in increasing order, so '<'
// keeps the lowest index; 16 columns per lane are requested at once for each
// of the R rows, and each r_j (read through L2, vectorised) serves the R
// rows.  Per-row outputs go to row_G / row_j / row_g.  Row sums are added in
// row order within a wave and waves in order within a workgroup; each
// workgroup stores its partials, and gap_total (a one-workgroup kernel
// after the sweep, or the first part of the full-FW step kernel) adds them
// in a fixed tree order and writes
//   out[0] = g = sum g_i,  out[1] = f = <T,C> + (w/2)||r||^2,
//   out[2] = D = sum a_i G_i - w <b, r> - (w/2)||r||^2,  out[3] = <T,C>,
//   out[4] = ||r||^2
// (sum_i <t_i, grad_i f> = <T,C> + w <r + b, r> gives D = f - g).
// ---------------------------------------------------------------------------
constexpr int GAP_KS = 2;  // support entries per lane and row gathered ahead of the scan

// Workgroup partials of a gap sweep.  Each workgroup adds its rows'
// (a_i G_i, lin_i, g_i) and, for its slice of ceil(n / grid) columns,
// ||r||^2 and <b, r>, and stores the five component-major (component c of
// workgroup b at partials[c * grid + b], so the final sum reads each
// component contiguously); the sweep kernel ends there, and gap_total (the
// next kernel) adds them.
__device__ __forceinline__ void gap_partials(const ProblemView &P, const double *__restrict__ rg, double aG,
                                             double lin, double gs, double *__restrict__ partials)
{
    __shared__ double s_w[GAP_NW][5];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = P.n;
    const int nb = (int)gridDim.x;
    const int cols = (n + nb - 1) / nb;
    const int j0 = min(n, (int)blockIdx.x * cols), j1 = min(n, j0 + cols);
    double x[2] = {0.0, 0.0};  // ||r||^2, <b, r> over this workgroup's columns
    for (int j = j0 + tid; j < j1; j += GAP_NT) {
        const double rj = rg[j];
        x[0] += rj * rj;
        x[1] += P.b[j] * rj;
    }
    wave_sum<2>(x);
    if (lane == 0) { s_w[wid][0] = aG; s_w[wid][1] = lin; s_w[wid][2] = gs; s_w[wid][3] = x[0]; s_w[wid][4] = x[1]; }
    __syncthreads();
    if (tid < 5) {
        double t = s_w[0][tid];
#pragma unroll
        for (int k = 1; k < GAP_NW; ++k) t += s_w[k][tid];
        partials[tid * nb + (int)blockIdx.x] = t;
    }
}

// The final sums of a sweep; in a solve (stop_w set) also the stop test of
// Sec. 3.1: g <= eps sets stop_w[0] and records the pass in stop_w[1].
__global__ __launch_bounds__(GAP_FINAL_NT) void gap_final_kernel(ProblemView P, const double *__restrict__ partials,
                                                                 int nb, double *__restrict__ out,
                                                                 double *__restrict__ out2, int32_t *__restrict__ stop_w,
                                                                 double eps, int32_t pass)
{
    if (P.stop && *P.stop) return;  // the solve has stopped: the last sums stay
    gap_total(P.w, partials, nb, out, out2);
    if (stop_w && threadIdx.x == 0 && out[0] <= eps) {
        stop_w[1] = pass;
        stop_w[0] = 1;
    }
}

template <int COST, int VEC, int R, bool FW>
__global__ __launch_bounds__(GAP_NT) void gap_sweep_kernel(ProblemView P, double *__restrict__ T,
                                                           double *__restrict__ rg,
                                                           uint32_t *__restrict__ M, Ownership own,
                                                           double *__restrict__ row_G,
                                                           int32_t *__restrict__ row_j,
                                                           double *__restrict__ row_g,
                                                           double *__restrict__ partials,
                                                           double *__restrict__ out, FwSweep fw, double delta2)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int GU = (FUSED && R > 2) ? 8 : 16 / VEC;  // vectors per lane per group
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = P.m, n = P.n;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;
    const int slots = own.words * own.nt;
    const int nq = (n + 64 * VEC - 1) / (64 * VEC);

    bool pending = false;
    double gprev = 0.0, scale = 0.0;
    if constexpr (FW) {
        if (fw.state[0]) return;  // the run has reached its gap: every workgroup leaves
        pending = fw.state[1] != 0;
        gprev = out[5];
        scale = *fw.scale;
    }
    double aG = 0.0, lin = 0.0, gs = 0.0;
    const int stride = gridDim.x * GAP_NW * R;
    for (int i0 = (blockIdx.x * GAP_NW + wid) * R; i0 < m; i0 += stride) {
        if constexpr (FW) {
            // the previous iteration's step on these rows (their old vertices)
            if (pending) {
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (i0 + k < m) fw_apply_row(i0 + k, n, gprev, P.a[i0 + k], row_j[i0 + k], own, T, M, lane, 64);
            }
        }
        int ir[R];
        float xr[R][3];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            ir[k] = (i0 + k < m) ? i0 + k : m - 1;
            if constexpr (FUSED) {
                xr[k][0] = P.X[3 * ir[k]]; xr[k][1] = P.X[3 * ir[k] + 1]; xr[k][2] = P.X[3 * ir[k] + 2];
            }
        }
        // The first GAP_KS support entries of each row in this lane's mask
        // slots are requested before the cost rows, so their gathers overlap
        // the stream; further entries (rare) are read after the scan.
        int sj[R][GAP_KS];
        double st[R][GAP_KS], sc[R][GAP_KS], sr[R][GAP_KS];
        bool more[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            more[k] = false;
            int found = 0;
#pragma unroll
            for (int e = 0; e < GAP_KS; ++e) sj[k][e] = -1;
            if (i0 + k < m) {
                for (int s = lane; s < slots; s += 64) {
                    uint32_t mk = M[(size_t)ir[k] * slots + s];
                    const int wd = s / own.nt, ts = s - wd * own.nt;
                    while (mk) {
                        const int b = __ffs(mk) - 1;
                        mk &= mk - 1u;
                        const int u = wd * 32 + b;
                        const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                        if (found < GAP_KS) {
#pragma unroll
                            for (int e = 0; e < GAP_KS; ++e) sj[k][e] = (e == found) ? j : sj[k][e];
                            ++found;
                        } else {
                            more[k] = true;
                        }
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < GAP_KS; ++e) {
                const int j = sj[k][e] >= 0 ? sj[k][e] : 0;
                st[k][e] = T[(size_t)ir[k] * (size_t)n + j];
                sr[k][e] = rg[j];
                if constexpr (FUSED) {
                    const float4 yj = P.Y4[j];
                    sc[k][e] = sqdist(xr[k][0], xr[k][1], xr[k][2], yj.x, yj.y, yj.z);
                } else {
                    sc[k][e] = (double)C[(size_t)ir[k] * (size_t)n + j];
                }
            }
        }
        double best[R];
        int bj[R];
#pragma unroll
        for (int k = 0; k < R; ++k) { best[k] = INFINITY; bj[k] = 0x7fffffff; }
        auto plain_scan = [&]() {
            for (int q0 = 0; q0 < nq; q0 += GU) {
                CT cv[R][GU][VEC];
                if constexpr (!FUSED) {
    #pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const CT *__restrict__ crow = C + (size_t)ir[k] * (size_t)n;
    #pragma unroll
                        for (int u = 0; u < GU; ++u) {
                            const int jb = ((q0 + u) * 64 + lane) * VEC;
                            const int jc = jb < n ? jb : 0;
                            if constexpr (VEC == 4) {
                                const float4 v = *reinterpret_cast<const float4 *>(crow + jc);
                                cv[k][u][0] = v.x; cv[k][u][1] = v.y; cv[k][u][2] = v.z; cv[k][u][3] = v.w;
                            } else if constexpr (VEC == 2) {
                                const double2 v = *reinterpret_cast<const double2 *>(crow + jc);
                                cv[k][u][0] = v.x; cv[k][u][1] = v.y;
                            } else {
                                cv[k][u][0] = crow[jc];
                            }
                        }
                    }
                }
    #pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const int jb = ((q0 + u) * 64 + lane) * VEC;
                    if (jb >= n) continue;
                    double rv[VEC];
                    if constexpr (VEC == 4) {
                        const double2 ra = *reinterpret_cast<const double2 *>(rg + jb);
                        const double2 rb = *reinterpret_cast<const double2 *>(rg + jb + 2);
                        rv[0] = ra.x; rv[1] = ra.y; rv[2] = rb.x; rv[3] = rb.y;
                    } else if constexpr (VEC == 2) {
                        const double2 ra = *reinterpret_cast<const double2 *>(rg + jb);
                        rv[0] = ra.x; rv[1] = ra.y;
                    } else {
                        rv[0] = rg[jb];
                    }
                    float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
                    if constexpr (FUSED) y = P.Y4[jb];
    #pragma unroll
                    for (int k = 0; k < R; ++k) {
    #pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            double c;
                            if constexpr (FUSED) c = sqdist(xr[k][0], xr[k][1], xr[k][2], y.x, y.y, y.z);
                            else c = (double)cv[k][u][e];
                            const double v = c + w * rv[e];
                            if (v < best[k]) { best[k] = v; bj[k] = jb + e; }
                        }
                    }
                }
            }
        };
        bool scanned = false;
        if constexpr (FUSED) {
            if (delta2 > 0.0) {
                // FP32 screen (the bound of the wide-row chain: every
                // |v'_j - v_j| <= delta2 / 2): a column is evaluated exactly
                // when its screen value is within delta2 of the smallest
                // screen value met so far by the wave, a set that holds every
                // exact minimiser (its screen value is within delta2 of every
                // other column's); lanes meet their columns in increasing
                // order, so '<' keeps the lowest index.
                const float w32 = (float)w;
                float bw[R];
#pragma unroll
                for (int k = 0; k < R; ++k) bw[k] = INFINITY;
                for (int q0 = 0; q0 < nq; q0 += GU) {
                    double rvv[GU];
                    float4 yy[GU];
#pragma unroll
                    for (int u = 0; u < GU; ++u) {
                        const int jb = (q0 + u) * 64 + lane;
                        const int jc = jb < n ? jb : 0;
                        rvv[u] = rg[jc];
                        yy[u] = P.Y4[jc];
                    }
                    float vp[R][GU];
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        float bl = bw[k];
#pragma unroll
                        for (int u = 0; u < GU; ++u) {
                            const float d0 = xr[k][0] - yy[u].x, d1 = xr[k][1] - yy[u].y, d2 = xr[k][2] - yy[u].z;
                            const float c = fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
                            const float v = fmaf(w32, (float)rvv[u], c);
                            vp[k][u] = ((q0 + u) * 64 + lane < n) ? v : INFINITY;
                            bl = fminf(bl, vp[k][u]);
                        }
                        bw[k] = wave_min_f32(bl);
                    }
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const float thr = __double2float_ru((double)bw[k] + delta2);
#pragma unroll
                        for (int u = 0; u < GU; ++u) {
                            if (vp[k][u] <= thr) {
                                const int jb = (q0 + u) * 64 + lane;
                                const double v = sqdist(xr[k][0], xr[k][1], xr[k][2], yy[u].x, yy[u].y, yy[u].z) +
                                                 w * rvv[u];
                                if (v < best[k]) { best[k] = v; bj[k] = jb; }
                            }
                        }
                    }
                }
                scanned = true;
            }
        }
        if (!scanned) plain_scan();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (i0 + k >= m) break;  // uniform over the wave
            const int i = i0 + k;
            double G = best[k];
            int J = bj[k];
            wave_argmin(G, J);
            double x[2] = {0.0, 0.0};
#pragma unroll
            for (int e = 0; e < GAP_KS; ++e) {
                if (sj[k][e] >= 0) {
                    x[0] += st[k][e] * (sc[k][e] + w * sr[k][e] - G);
                    x[1] += st[k][e] * sc[k][e];
                }
            }
            if (__any(more[k])) {
                int seen = 0;  // entries of this lane already added
                for (int s = lane; s < slots; s += 64) {
                    const int wd = s / own.nt, ts = s - wd * own.nt;
                    uint32_t mk = more[k] ? M[(size_t)i * slots + s] : 0u;
                    while (mk) {
                        const int b = __ffs(mk) - 1;
                        mk &= mk - 1u;
                        if (seen++ < GAP_KS) continue;
                        const int u = wd * 32 + b;
                        const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                        const double t = T[(size_t)i * (size_t)n + j];
                        double c;
                        if constexpr (FUSED) {
                            const float4 yj = P.Y4[j];
                            c = sqdist(xr[k][0], xr[k][1], xr[k][2], yj.x, yj.y, yj.z);
                        } else {
                            c = (double)C[(size_t)i * (size_t)n + j];
                        }
                        x[0] += t * (c + w * rg[j] - G);
                        x[1] += t * c;
                    }
                }
            }
            wave_sum<2>(x);
            if (lane == 0) {
                row_G[i] = G;
                row_j[i] = J;
                row_g[i] = x[0];
                // full FW: a_i joins its vertex column's sum (the atomics
                // have completed when the kernel ends)
                if constexpr (FW)
                    __hip_atomic_fetch_add(fw.s_fixed + J, (unsigned long long)__double2ull_rn(P.a[i] * scale),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            aG += P.a[i] * G;
            lin += x[1];
            gs += x[0];
        }
    }
    gap_partials(P, rg, aG, lin, gs, partials);
}

// Stored-cost gap sweep with the memory operations ordered for latency:
// per group of R rows a wave issues the rows' support-mask words (up to
// GAP_MW per lane and row), then the first batch of GU 16-byte cost vectors
// per row together with the matching entries of r, and only then waits for
// the masks; the support gathers follow, and the batches run double
// buffered (batch q + 1 requested before batch q is consumed).  Loads are
// raw buffer loads whose out-of-range offsets return zero without touching
// memory, so every batch is one fixed, branch-free group of requests and
// each wait covers exactly the batch it needs.  Same per-row results as
// gap_sweep_kernel (and, with R = 2, the same summation order).
//
// ROT (wide rows): each row group starts its column sweep at a hashed
// vector offset and wraps around, so the waves in flight read different
// parts of r at any moment instead of all requesting the same L2 lines; the
// argmin then keeps the lowest index among equal values explicitly.
constexpr int GAP_MW = 8;  // mask words per lane and row read ahead

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int COST, int R, int GU, bool FW, bool ROT>
__global__ __launch_bounds__(GAP_NT) __attribute__((amdgpu_waves_per_eu(2))) void gap_stream_kernel(ProblemView P, double *__restrict__ T,
                                                            double *__restrict__ rg,
                                                            uint32_t *__restrict__ M, Ownership own,
                                                            double *__restrict__ row_G,
                                                            int32_t *__restrict__ row_j,
                                                            double *__restrict__ row_g,
                                                            double *__restrict__ partials,
                                                            double *__restrict__ out, FwSweep fw)
{
    if (P.stop && *P.stop) return;  // the solve has stopped
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr int VEC = 16 / (int)sizeof(CT);  // columns per 16-byte vector
    constexpr int RV = VEC / 2;                // 16-byte vectors of r per cost vector
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int m = P.m, n = P.n;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;
    const int slots = own.words * own.nt;
    const int nq = (n + 64 * VEC - 1) / (64 * VEC);
    const __amdgpu_buffer_rsrc_t rs_r = buf_rsrc(rg, (unsigned)n * 8u);

    bool pending = false;
    double gprev = 0.0, scale = 0.0;
    if constexpr (FW) {
        if (fw.state[0]) return;  // the run has reached its gap: every workgroup leaves
        pending = fw.state[1] != 0;
        gprev = out[5];
        scale = *fw.scale;
    }
    double aG = 0.0, lin = 0.0, gs = 0.0;
    const int stride = gridDim.x * GAP_NW * R;
    for (int i0 = (blockIdx.x * GAP_NW + wid) * R; i0 < m; i0 += stride) {
        int ir[R];
        __amdgpu_buffer_rsrc_t rs_c[R];
        uint32_t mw[R][GAP_MW];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            ir[k] = (i0 + k < m) ? i0 + k : m - 1;
            rs_c[k] = buf_rsrc(C + (size_t)ir[k] * (size_t)n, (unsigned)(n * sizeof(CT)));
        }
        u32x4 ca[R][GU], cb[R][GU];
        u32x4 ra[GU][RV], rb[GU][RV];
        // vector group qq of the sweep order -> its place in the row
        int rot = 0;
        if constexpr (ROT) rot = (int)((((unsigned)(i0 / R) * 2654435761u) >> 8) % (unsigned)nq);
        auto qmap = [&](int qq) {
            if constexpr (!ROT) return qq;
            return qq < nq ? (qq + rot >= nq ? qq + rot - nq : qq + rot) : nq;
        };
        auto issue = [&](u32x4 (&c)[R][GU], u32x4 (&rr)[GU][RV], int q0) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int jb = (qmap(q0 + u) * 64 + lane) * VEC;
                const unsigned oc = jb < n ? (unsigned)jb * (unsigned)sizeof(CT) : kOOB;
                const unsigned orr = jb < n ? (unsigned)jb * 8u : kOOB;
#pragma unroll
                for (int k = 0; k < R; ++k) c[k][u] = __builtin_amdgcn_raw_buffer_load_b128(rs_c[k], (int)oc, 0, 0);
#pragma unroll
                for (int h = 0; h < RV; ++h)
                    rr[u][h] = __builtin_amdgcn_raw_buffer_load_b128(rs_r, (int)(orr + 16u * h), 0, 0);
            }
        };
        double best[R];
        int bj[R];
#pragma unroll
        for (int k = 0; k < R; ++k) { best[k] = INFINITY; bj[k] = 0x7fffffff; }
        auto consume = [&](const u32x4 (&c)[R][GU], const u32x4 (&rr)[GU][RV], int q0) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int jb = (qmap(q0 + u) * 64 + lane) * VEC;
                double rv[VEC];
#pragma unroll
                for (int h = 0; h < RV; ++h) {
                    rv[2 * h] = __builtin_bit_cast(double, (unsigned long long)rr[u][h].x | ((unsigned long long)rr[u][h].y << 32));
                    rv[2 * h + 1] = __builtin_bit_cast(double, (unsigned long long)rr[u][h].z | ((unsigned long long)rr[u][h].w << 32));
                }
#pragma unroll
                for (int k = 0; k < R; ++k) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        double cval;
                        if constexpr (sizeof(CT) == 4) {
                            const unsigned bits = e == 0 ? c[k][u].x : (e == 1 ? c[k][u].y : (e == 2 ? c[k][u].z : c[k][u].w));
                            cval = (double)__builtin_bit_cast(float, bits);
                        } else {
                            const unsigned lo = e == 0 ? c[k][u].x : c[k][u].z, hi = e == 0 ? c[k][u].y : c[k][u].w;
                            cval = __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
                        }
                        const double v = (jb < n) ? cval + w * rv[e] : INFINITY;
                        if (ROT ? (v < best[k] || (v == best[k] && jb + e < bj[k])) : (v < best[k])) {
                            best[k] = v;
                            bj[k] = jb + e;
                        }
                    }
                }
            }
        };
        if constexpr (!FW) issue(ca, ra, 0);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            // rows past the end read an empty range: no support, no cost
            const __amdgpu_buffer_rsrc_t rs_m =
                buf_rsrc(M + (size_t)ir[k] * slots, (i0 + k < m) ? (unsigned)slots * 4u : 0u);
#pragma unroll
            for (int q = 0; q < GAP_MW; ++q)
                mw[k][q] = __builtin_amdgcn_raw_buffer_load_b32(rs_m, (int)((lane + 64 * q) * 4), 0, 0);
        }

        // support entries of the rows from the mask words (first GAP_KS per
        // lane and row gathered now, further ones after the scan); sq / sb
        // keep each entry's mask word and bit
        int sj[R][GAP_KS], sq[R][GAP_KS], sb[R][GAP_KS];
        double st[R][GAP_KS], sc[R][GAP_KS], sr[R][GAP_KS];
        bool more[R];
        int nfound[R];
        auto extract = [&](int k) {
            more[k] = false;
            int found = 0;
#pragma unroll
            for (int e = 0; e < GAP_KS; ++e) { sj[k][e] = -1; sq[k][e] = 0; sb[k][e] = 0; }
            for (int q = 0; q < GAP_MW; ++q) {
                uint32_t mk = mw[k][q];
                const int sl = lane + 64 * q;
                const int wd = sl / own.nt, ts = sl - wd * own.nt;
                while (mk) {
                    const int b = __ffs(mk) - 1;
                    mk &= mk - 1u;
                    const int u = wd * 32 + b;
                    const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                    if (found < GAP_KS) {
#pragma unroll
                        for (int e = 0; e < GAP_KS; ++e) {
                            sj[k][e] = (e == found) ? j : sj[k][e];
                            sq[k][e] = (e == found) ? q : sq[k][e];
                            sb[k][e] = (e == found) ? b : sb[k][e];
                        }
                        ++found;
                    } else {
                        more[k] = true;
                    }
                }
            }
            nfound[k] = found;
            more[k] |= (slots > 64 * GAP_MW) && (i0 + k < m);
        };
        auto gather = [&](int k) {
#pragma unroll
            for (int e = 0; e < GAP_KS; ++e) {
                const int j = sj[k][e] >= 0 ? sj[k][e] : 0;
                st[k][e] = T[(size_t)ir[k] * (size_t)n + j];
                sr[k][e] = rg[j];
                sc[k][e] = (double)C[(size_t)ir[k] * (size_t)n + j];
            }
        };
#pragma unroll
        for (int k = 0; k < R; ++k) extract(k);
        if constexpr (FW) {
            // the previous iteration's step on these rows (Alg. A.1:
            // t_ij <- (1 - gamma) t_ij + gamma a_i [j == js], js the row's
            // previous vertex), taken on the entries gathered here when each
            // lane's part of the support, the vertex included, fits them;
            // otherwise the row is updated in full first and read again
            if (pending) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int i = i0 + k;
                    if (i >= m) break;  // uniform over the wave
                    const int js = row_j[i];
                    const int jg = js / own.vec;
                    const int u_star = (jg / own.nt) * own.vec + (js % own.vec);
                    const int s_star = (u_star >> 5) * own.nt + jg % own.nt;
                    const int q_star = s_star >> 6, b_star = u_star & 31;
                    const bool mine = (s_star & 63) == lane;
                    // js joins the lane's entries unless its bit is set already
                    const bool add = mine && q_star < GAP_MW && !((mw[k][q_star < GAP_MW ? q_star : 0] >> b_star) & 1u);
                    const bool over = more[k] || (add && nfound[k] >= GAP_KS) || (mine && q_star >= GAP_MW);
                    if (__any(over)) {
                        fw_apply_row(i, n, gprev, P.a[i], js, own, T, M, lane, 64);
                        drain_memory();
                        const __amdgpu_buffer_rsrc_t rs_m = buf_rsrc(M + (size_t)i * slots, (unsigned)slots * 4u);
#pragma unroll
                        for (int q = 0; q < GAP_MW; ++q)
                            mw[k][q] = __builtin_amdgcn_raw_buffer_load_b32(rs_m, (int)((lane + 64 * q) * 4), 0, 0);
                        extract(k);
                        gather(k);
                        continue;
                    }
                    if (add) {
#pragma unroll
                        for (int e = 0; e < GAP_KS; ++e) {
                            const bool here = e == nfound[k];
                            sj[k][e] = here ? js : sj[k][e];
                            sq[k][e] = here ? q_star : sq[k][e];
                            sb[k][e] = here ? b_star : sb[k][e];
                        }
                        ++nfound[k];
                    }
                    gather(k);
                    const double gadd = gprev * P.a[i];
                    uint32_t nm[GAP_MW];
#pragma unroll
                    for (int q = 0; q < GAP_MW; ++q) nm[q] = mw[k][q];
#pragma unroll
                    for (int e = 0; e < GAP_KS; ++e) {
                        const int j = sj[k][e];
                        if (j < 0) continue;
                        const bool fresh = add && j == js;  // not in the support before
                        const double t = fresh ? 0.0 : st[k][e];
                        const double tn = (1.0 - gprev) * t + ((j == js) ? gadd : 0.0);
                        if (tn != t || fresh) T[(size_t)i * (size_t)n + j] = tn;
                        st[k][e] = tn;
                        const uint32_t bit = 1u << sb[k][e];
#pragma unroll
                        for (int q = 0; q < GAP_MW; ++q)
                            if (q == sq[k][e]) nm[q] = (tn != 0.0) ? (nm[q] | bit) : (nm[q] & ~bit);
                    }
#pragma unroll
                    for (int q = 0; q < GAP_MW; ++q)
                        if (nm[q] != mw[k][q]) M[(size_t)i * slots + lane + 64 * q] = nm[q];
                }
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k) gather(k);
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) gather(k);
        }

        if constexpr (FW) issue(ca, ra, 0);
        for (int q0 = 0; q0 < nq; q0 += 2 * GU) {
            issue(cb, rb, q0 + GU);
            consume(ca, ra, q0);
            issue(ca, ra, q0 + 2 * GU);
            consume(cb, rb, q0 + GU);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (i0 + k >= m) break;  // uniform over the wave
            const int i = i0 + k;
            double G = best[k];
            int J = bj[k];
            wave_argmin(G, J);
            double x[2] = {0.0, 0.0};
#pragma unroll
            for (int e = 0; e < GAP_KS; ++e) {
                if (sj[k][e] >= 0) {
                    x[0] += st[k][e] * (sc[k][e] + w * sr[k][e] - G);
                    x[1] += st[k][e] * sc[k][e];
                }
            }
            if (__any(more[k])) {
                // every support entry of this lane after the ones gathered
                // above (its first nfound, in slot order)
                int seen = 0;
                for (int sl = lane; sl < slots; sl += 64) {
                    const int wd = sl / own.nt, ts = sl - wd * own.nt;
                    uint32_t mk = M[(size_t)i * slots + sl];
                    while (mk) {
                        const int b = __ffs(mk) - 1;
                        mk &= mk - 1u;
                        if (seen++ < nfound[k]) continue;
                        const int u = wd * 32 + b;
                        const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                        const double t = T[(size_t)i * (size_t)n + j];
                        const double c = (double)C[(size_t)i * (size_t)n + j];
                        x[0] += t * (c + w * rg[j] - G);
                        x[1] += t * c;
                    }
                }
            }
            wave_sum<2>(x);
            if (lane == 0) {
                row_G[i] = G;
                row_j[i] = J;
                row_g[i] = x[0];
                // full FW: a_i joins its vertex column's sum (the atomics
                // have completed when the kernel ends)
                if constexpr (FW)
                    __hip_atomic_fetch_add(fw.s_fixed + J, (unsigned long long)__double2ull_rn(P.a[i] * scale),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            aG += P.a[i] * G;
            lin += x[1];
            gs += x[0];
        }
    }
    gap_partials(P, rg, aG, lin, gs, partials);
}

// ---------------------------------------------------------------------------
// Initial plan t_i = a_i e_0, residual, support masks, validation.
// ---------------------------------------------------------------------------
__global__ void init_plan_kernel(int32_t m, int32_t n, const double *__restrict__ a,
                                 double *__restrict__ T)
{
    const size_t total = (size_t)m * (size_t)n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t i = e / (size_t)n, j = e - i * (size_t)n;
        T[e] = (j == 0) ? a[i] : 0.0;
    }
}

// Target points padded to 16 bytes (one vector load per point), followed by
// sentinel points 3e18 away from every coordinate up to entry y4n - 1: a
// streamed screen reads them for columns past n - 1 instead of selecting
// per column.
__global__ void pad_points_kernel(int32_t n, int32_t y4n, const float *__restrict__ Y, float4 *__restrict__ Y4)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < y4n; j += gridDim.x * blockDim.x)
        Y4[j] = (j < n) ? make_float4(Y[3 * j], Y[3 * j + 1], Y[3 * j + 2], 0.f) : make_float4(3e18f, 3e18f, 3e18f, 0.f);
}

// r_j = sum_i T_ij - b_j, rows added in order.
__global__ void residual_kernel(int32_t m, int32_t n, const double *__restrict__ T,
                                const double *__restrict__ b, double *__restrict__ r)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += T[(size_t)i * (size_t)n + j];
    r[j] = s - b[j];
}

// Support masks from a dense plan, in the layout of Ownership.
__global__ void mask_build_kernel(int32_t m, int32_t n, Ownership own, const double *__restrict__ T,
                                  uint32_t *__restrict__ M)
{
    const int tid = threadIdx.x;  // blockDim.x == own.nt
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const size_t base = (size_t)i * (size_t)n;
        for (int wd = 0; wd < own.words; ++wd) {
            uint32_t word = 0u;
            for (int b = 0; b < 32; ++b) {
                const int u = wd * 32 + b;
                const int j = ((u / own.vec) * own.nt + tid) * own.vec + (u % own.vec);
                if (u < own.cpt && j < n && T[base + j] != 0.0) word |= (1u << b);
            }
            M[((size_t)i * own.words + wd) * own.nt + tid] = word;
        }
    }
}

template <typename V>
__device__ __forceinline__ bool bad_value(V x) { return !isfinite((double)x); }

__global__ void validate_kernel(ProblemView P, int32_t *__restrict__ flag)
{
    const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    const size_t mn = (size_t)P.m * (size_t)P.n;
    if (P.cost == SROT_COST_F32) {
        const float *C = (const float *)P.C;
        for (size_t e = tid; e < mn; e += stride) bad |= bad_value(C[e]);
    } else if (P.cost == SROT_COST_F64) {
        const double *C = (const double *)P.C;
        for (size_t e = tid; e < mn; e += stride) bad |= bad_value(C[e]);
    }
    if (P.X) for (size_t e = tid; e < (size_t)P.m * 3; e += stride) bad |= bad_value(P.X[e]);
    if (P.Y) for (size_t e = tid; e < (size_t)P.n * 3; e += stride) bad |= bad_value(P.Y[e]);
    for (size_t e = tid; e < (size_t)P.m; e += stride) bad |= bad_value(P.a[e]) || P.a[e] < 0.0;
    for (size_t e = tid; e < (size_t)P.n; e += stride) bad |= bad_value(P.b[e]) || P.b[e] < 0.0;
    if (bad) atomicOr(flag, 1);
}

__global__ void check_indices_kernel(const int32_t *__restrict__ idx, int64_t count, int32_t m,
                                     int32_t *__restrict__ flag)
{
    bool bad = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        bad |= (idx[e] < 0) || (idx[e] >= m);
    if (bad) atomicOr(flag, 2);
}

// uniform block index floor(x * m / 2^64)
__global__ void sample_uniform_kernel(uint64_t seed, int64_t k0, int64_t count, int32_t m,
                                      int32_t *__restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = philox_output(seed, (uint64_t)(k0 + e));
        out[e] = (int32_t)__umul64hi(x, (uint64_t)m);
    }
}

// Pass p visits rows in the order of a stable ascending sort of the keys
// x_{p m + t}: row t goes to position rank(t) = #{t' : key t' < key t, or equal
// with t' < t}.  One workgroup per pass, keys staged through LDS tiles.
__global__ __launch_bounds__(256) void sample_permute_kernel(uint64_t seed, int64_t p0, int32_t m,
                                                             int32_t *__restrict__ out)
{
    // grid: (ceil(m / 256) key tiles, passes); each thread ranks one key of
    // its pass against all m keys of that pass (stable: ties by position)
    __shared__ uint64_t tile[256];
    const int64_t p = p0 + blockIdx.y;
    int32_t *o = out + (int64_t)blockIdx.y * m;
    const int32_t t = (int32_t)blockIdx.x * 256 + (int32_t)threadIdx.x;
    const uint64_t kt = (t < m) ? philox_output(seed, (uint64_t)(p * m + t)) : 0ull;
    int32_t rank = 0;
    for (int32_t ub = 0; ub < m; ub += 256) {
        const int32_t u = ub + threadIdx.x;
        tile[threadIdx.x] = (u < m) ? philox_output(seed, (uint64_t)(p * m + u)) : 0ull;
        __syncthreads();
        const int32_t lim = min(256, m - ub);
        for (int32_t q = 0; q < lim; ++q) {
            const uint64_t ku = tile[q];
            rank += (ku < kt) || (ku == kt && ub + q < t);
        }
        __syncthreads();
    }
    if (t < m) o[rank] = t;
}

// ---------------------------------------------------------------------------
// Variant choice and launch wrappers
// ---------------------------------------------------------------------------
static int grid_for(size_t work, int nt, int cap)
{
    size_t g = (work + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

#define SROT_VARIANTS_V1(X) \
    X(64, 2, 1) X(64, 4, 1) X(128, 4, 1) X(256, 4, 1) X(256, 8, 1) X(256, 16, 1) X(512, 8, 1)
#define SROT_VARIANTS_V2(X) \
    X(64, 2, 2) X(64, 4, 2) X(128, 4, 2) X(256, 4, 2) X(256, 8, 2) X(256, 16, 2) X(512, 8, 2)
#define SROT_VARIANTS_V4(X) \
    X(64, 4, 4) X(128, 4, 4) X(256, 4, 4) X(256, 8, 4) X(256, 16, 4) X(512, 8, 4)

static bool variant_exists(int nt, int cpt, int vec)
{
    bool ok = false;
#define SROT_HAS(NT_, CPT_, VEC_) ok |= (nt == NT_ && cpt == CPT_ && vec == VEC_);
    SROT_VARIANTS_V1(SROT_HAS)
    SROT_VARIANTS_V2(SROT_HAS)
    SROT_VARIANTS_V4(SROT_HAS)
#undef SROT_HAS
    return ok;
}

// Default: the fewest threads with at most 16 columns each (rows up to 4096
// columns keep r in registers), 16-byte cost loads when the row length and
// alignment allow; wider rows take the global-residual kernel.
// SROT_CHAIN_VARIANT=<nt>x<cpt>[x<vec>] overrides the choice when valid.
Ownership choose_ownership(int64_t n, int cost, bool aligned16)
{
    int pref = cost == SROT_COST_F32 ? 4 : (cost == SROT_COST_F64 ? 2 : 1);
    if (n % pref != 0 || !aligned16) pref = 1;
    int nt = 0, cpt = 0, vec = 1;
    const char *env = getenv("SROT_CHAIN_VARIANT");
    if (env) {
        int a = 0, b = 0, c = 1;
        const int got = sscanf(env, "%dx%dx%d", &a, &b, &c);
        if (got >= 2) {
            if (got == 2) c = (b % pref == 0) ? pref : 1;
            if (n <= (int64_t)a * b && (c == 1 || c == pref) && variant_exists(a, b, c)) {
                nt = a; cpt = b; vec = c;
            }
        }
    }
    if (nt == 0) {
        if (n <= 128) { nt = 64; cpt = 2; }
        else if (n <= 256) { nt = 64; cpt = 4; }
        else if (n <= 512) { nt = 128; cpt = 4; }
        else if (n <= 1024) { nt = 256; cpt = 4; }
        else if (n <= 2048) { nt = 256; cpt = 8; }
        else if (n <= 4096) { nt = 256; cpt = 16; }
        if (nt > 0) vec = (cpt % pref == 0 && variant_exists(nt, cpt, pref)) ? pref : 1;
    }
    Ownership o;
    if (nt > 0) {
        o.nt = nt; o.cpt = cpt; o.vec = vec; o.words = 1; o.reg = 1;
    } else {
        o.nt = GLB_NT;
        o.cpt = (int32_t)((n + GLB_NT - 1) / GLB_NT);
        o.vec = 1;
        o.words = (o.cpt + 31) / 32;
        o.reg = 0;
    }
    return o;
}

hipError_t launch_validate(const ProblemView &P, const DeviceState &S, hipStream_t stream)
{
    const size_t work = (size_t)P.m * (size_t)P.n + (size_t)P.m + (size_t)P.n;
    hipLaunchKernelGGL(validate_kernel, dim3(grid_for(work, 256, 4096)), dim3(256), 0, stream, P,
                       S.flags);
    return hipGetLastError();
}

hipError_t launch_check_indices(const int32_t *idx, int64_t count, int32_t m, int32_t *flag,
                                hipStream_t stream)
{
    hipLaunchKernelGGL(check_indices_kernel, dim3(grid_for((size_t)count, 256, 1024)), dim3(256), 0,
                       stream, idx, count, m, flag);
    return hipGetLastError();
}

hipError_t launch_init_plan(const ProblemView &P, const DeviceState &S, hipStream_t stream)
{
    const size_t total = (size_t)P.m * (size_t)P.n;
    hipLaunchKernelGGL(init_plan_kernel, dim3(grid_for(total, 256, 16384)), dim3(256), 0, stream,
                       P.m, P.n, P.a, S.T);
    return hipGetLastError();
}

hipError_t launch_residual(const ProblemView &P, const DeviceState &S, hipStream_t stream)
{
    hipLaunchKernelGGL(residual_kernel, dim3((P.n + 255) / 256), dim3(256), 0, stream, P.m, P.n,
                       S.T, P.b, S.r);
    return hipGetLastError();
}

hipError_t launch_pad_points(const ProblemView &P, hipStream_t stream)
{
    if (!P.Y || !P.Y4) return hipSuccess;
    hipLaunchKernelGGL(pad_points_kernel, dim3(grid_for((size_t)P.y4n, 256, 1024)), dim3(256), 0, stream,
                       P.n, P.y4n, P.Y, const_cast<float4 *>(P.Y4));
    return hipGetLastError();
}

hipError_t launch_mask_build(const ProblemView &P, const DeviceState &S, hipStream_t stream)
{
    const int grid = P.m < 4096 ? P.m : 4096;
    hipLaunchKernelGGL(mask_build_kernel, dim3(grid), dim3(S.own.nt), 0, stream, P.m, P.n, S.own,
                       S.T, S.mask);
    return hipGetLastError();
}

hipError_t launch_sample_uniform(uint64_t seed, int64_t k0, int64_t count, int32_t m,
                                 int32_t *out, hipStream_t stream)
{
    hipLaunchKernelGGL(sample_uniform_kernel, dim3(grid_for((size_t)count, 256, 4096)), dim3(256),
                       0, stream, seed, k0, count, m, out);
    return hipGetLastError();
}

hipError_t launch_sample_permute(uint64_t seed, int64_t p0, int64_t npasses, int32_t m,
                                 int32_t *out, hipStream_t stream)
{
    // passes along the grid's second dimension, at most 65535 per launch
    for (int64_t c = 0; c < npasses; c += 65535) {
        const int64_t np = std::min<int64_t>(65535, npasses - c);
        hipLaunchKernelGGL(sample_permute_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)np), dim3(256), 0,
                           stream, seed, p0 + c, m, out + c * (int64_t)m);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int COST>
static hipError_t launch_chain_cost(const ProblemView &P, const DeviceState &S, const int32_t *idx,
                                    int64_t k0, int64_t nsteps, int rule, int32_t *tj, double *tg,
                                    hipStream_t st)
{
    const Ownership &o = S.own;
    if constexpr (COST == SROT_COST_F32) {
        if (S.screen_err > 0.0 && screened_chain_supported(P, S))
            return launch_chain_screened(P, S, idx, k0, nsteps, rule, tj, tg, st);
    }
    if (o.reg) {
#define SROT_CHAIN(NT_, CPT_, VEC_)                                                                \
        if (o.nt == NT_ && o.cpt == CPT_ && o.vec == VEC_) {                                       \
            if (tj || tg)                                                                          \
                hipLaunchKernelGGL((chain_kernel<NT_, CPT_, VEC_, COST, true>), dim3(1), dim3(NT_), 0, \
                                   st, P, S.T, S.r, S.mask, idx, k0, nsteps, rule, tj, tg, S.slow_steps); \
            else                                                                                   \
                hipLaunchKernelGGL((chain_kernel<NT_, CPT_, VEC_, COST, false>), dim3(1), dim3(NT_),  \
                                   0, st, P, S.T, S.r, S.mask, idx, k0, nsteps, rule, tj, tg,       \
                                   S.slow_steps);                                                  \
            return hipGetLastError();                                                              \
        }
        SROT_VARIANTS_V1(SROT_CHAIN)
        if constexpr (COST == SROT_COST_F32) { SROT_VARIANTS_V4(SROT_CHAIN) }
        if constexpr (COST == SROT_COST_F64) { SROT_VARIANTS_V2(SROT_CHAIN) }
#undef SROT_CHAIN
        return hipErrorInvalidConfiguration;
    }
    if (S.team) return launch_chain_team(P, S, idx, k0, nsteps, rule, tj, tg, st);
    if constexpr (COST == SROT_COST_SQEUCLID) {
        if (P.n <= WIDE_MAX_N && S.screen_delta2 > 0.0) {
            const size_t lds = sizeof(float) * (size_t)WIDE_NT * (o.cpt <= 16 ? 16 : (o.cpt <= 32 ? 32 : 64));
#define SROT_WIDE(CPTK_, YMODE_)                                                                    \
            if (o.cpt <= CPTK_) {                                                                  \
                const void *fn = (tj || tg) ? (const void *)&chain_wide_kernel<CPTK_, YMODE_, true>   \
                                            : (const void *)&chain_wide_kernel<CPTK_, YMODE_, false>; \
                hipError_t e_ = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                                                    (int)lds);                                       \
                if (e_ != hipSuccess) return e_;                                                   \
                if (tj || tg)                                                                      \
                    hipLaunchKernelGGL((chain_wide_kernel<CPTK_, YMODE_, true>), dim3(1), dim3(WIDE_NT), \
                                       lds, st, P, S.T, S.r, S.mask, o.words, idx, k0, nsteps, rule, tj, \
                                       tg, S.screen_delta2, S.slow_steps);                         \
                else                                                                               \
                    hipLaunchKernelGGL((chain_wide_kernel<CPTK_, YMODE_, false>), dim3(1), dim3(WIDE_NT), \
                                       lds, st, P, S.T, S.r, S.mask, o.words, idx, k0, nsteps, rule, tj, \
                                       tg, S.screen_delta2, S.slow_steps);                         \
                return hipGetLastError();                                                          \
            }
            SROT_WIDE(16, 1)
            SROT_WIDE(32, 1)
            SROT_WIDE(64, 0)
#undef SROT_WIDE
        }
    }
    hipLaunchKernelGGL((chain_glb_kernel<COST>), dim3(1), dim3(GLB_NT), 0, st, P, S.T, S.r, S.mask,
                       o.words, idx, k0, nsteps, rule, tj, tg, S.slow_steps);
    return hipGetLastError();
}

hipError_t launch_screen_bounds(const ProblemView &P, double *out2, hipStream_t stream)
{
    hipLaunchKernelGGL(screen_bounds_kernel, dim3(1), dim3(256), 0, stream, P, out2);
    return hipGetLastError();
}

hipError_t launch_chain(const ProblemView &P, const DeviceState &S, const int32_t *idx, int64_t k0,
                        int64_t nsteps, int rule, int32_t *trace_j, double *trace_gamma,
                        hipStream_t stream)
{
    if (nsteps <= 0) return hipSuccess;
    switch (P.cost) {
    case SROT_COST_F32:
        return launch_chain_cost<SROT_COST_F32>(P, S, idx, k0, nsteps, rule, trace_j, trace_gamma, stream);
    case SROT_COST_F64:
        return launch_chain_cost<SROT_COST_F64>(P, S, idx, k0, nsteps, rule, trace_j, trace_gamma, stream);
    default:
        return launch_chain_cost<SROT_COST_SQEUCLID>(P, S, idx, k0, nsteps, rule, trace_j, trace_gamma, stream);
    }
}

// Workgroups of a gap sweep: two rows per wave, four waves per workgroup.
int32_t gap_blocks_for(int64_t m)
{
    int64_t b = (m + 2 * GAP_NW - 1) / (2 * GAP_NW);
    if (b < 1) b = 1;
    if (b > GAP_MAX_BLOCKS) b = GAP_MAX_BLOCKS;
    return (int32_t)b;
}

// Row-strided sweep (fused cost, or rows not split into 16-byte vectors):
// at most 1024 workgroups, where it measured best; each r_j (and target
// point) read serves R rows: 2, or 4 for the fused cost, whose FP32 screen
// leaves the loads of r and the points as the larger part of the work.
template <int COST, int VEC>
static hipError_t launch_gap_rows(const ProblemView &P, const DeviceState &S, const FwSweep *fw, hipStream_t st,
                                  int *nb_out)
{
    constexpr int R = (COST == SROT_COST_SQEUCLID) ? 4 : 2;
    const int64_t waves = (P.m + R - 1) / R;
    const int nb = (int)std::min<int64_t>(std::min<int64_t>((waves + GAP_NW - 1) / GAP_NW, 1024), S.gap_blocks);
    *nb_out = nb;
    if (fw)
        hipLaunchKernelGGL((gap_sweep_kernel<COST, VEC, R, true>), dim3(nb), dim3(GAP_NT), 0, st, P, S.T, S.r, S.mask,
                           S.own, S.row_G, S.row_j, S.row_g, S.partials, S.scalars, *fw, S.screen_delta2);
    else
        hipLaunchKernelGGL((gap_sweep_kernel<COST, VEC, R, false>), dim3(nb), dim3(GAP_NT), 0, st, P, S.T, S.r,
                           S.mask, S.own, S.row_G, S.row_j, S.row_g, S.partials, S.scalars, FwSweep{},
                           S.screen_delta2);
    return hipGetLastError();
}

// Stored cost in 16-byte vectors: two rows per wave, double-buffered
// batches of two vectors (FP32) or four (FP64) per lane and row; rows of
// 8192 columns or more: rotated starts and, for the plain sweep, four rows
// per wave, half the batch, at most 512 workgroups (measured best on
// 16384 x 16384; the full-FW form keeps two rows per wave, which its
// registers allow at two waves per SIMD).
template <int COST, int R, int GU, bool ROT>
static hipError_t launch_gap_stream_rg(const ProblemView &P, const DeviceState &S, const FwSweep *fw, hipStream_t st,
                                       int cap, int *nb_out)
{
    const int64_t waves = (P.m + R - 1) / R;
    const int nb = (int)std::min<int64_t>(std::min<int64_t>((waves + GAP_NW - 1) / GAP_NW, cap), S.gap_blocks);
    *nb_out = nb;
    if (fw)
        hipLaunchKernelGGL((gap_stream_kernel<COST, R, GU, true, ROT>), dim3(nb), dim3(GAP_NT), 0, st, P, S.T, S.r,
                           S.mask, S.own, S.row_G, S.row_j, S.row_g, S.partials, S.scalars, *fw);
    else
        hipLaunchKernelGGL((gap_stream_kernel<COST, R, GU, false, ROT>), dim3(nb), dim3(GAP_NT), 0, st, P, S.T, S.r,
                           S.mask, S.own, S.row_G, S.row_j, S.row_g, S.partials, S.scalars, FwSweep{});
    return hipGetLastError();
}

template <int COST>
static hipError_t launch_gap_stream(const ProblemView &P, const DeviceState &S, const FwSweep *fw, hipStream_t st,
                                    int *nb_out)
{
    constexpr int GU = (COST == SROT_COST_F32) ? 2 : 4;
    if (P.n >= 8192) {
        if (fw) return launch_gap_stream_rg<COST, 4, GU / 2, true>(P, S, fw, st, 512, nb_out);
        return launch_gap_stream_rg<COST, 4, GU / 2, true>(P, S, fw, st, 512, nb_out);
    }
    return launch_gap_stream_rg<COST, 2, GU, false>(P, S, fw, st, GAP_MAX_BLOCKS, nb_out);
}

static hipError_t launch_gap_any(const ProblemView &P, const DeviceState &S, const FwSweep *fw, hipStream_t stream,
                                 int *nb)
{
    const uintptr_t cbase = (uintptr_t)P.C;
    // buffer ranges of one cost row and of r are 32-bit byte counts
    const bool ranged = (int64_t)P.n * 8 < (int64_t)0x7fffffff;
    switch (P.cost) {
    case SROT_COST_F32:
        if (P.n % 4 == 0 && cbase % 16 == 0 && ranged) return launch_gap_stream<SROT_COST_F32>(P, S, fw, stream, nb);
        return launch_gap_rows<SROT_COST_F32, 1>(P, S, fw, stream, nb);
    case SROT_COST_F64:
        if (P.n % 2 == 0 && cbase % 16 == 0 && ranged) return launch_gap_stream<SROT_COST_F64>(P, S, fw, stream, nb);
        return launch_gap_rows<SROT_COST_F64, 1>(P, S, fw, stream, nb);
    default:
        return launch_gap_rows<SROT_COST_SQEUCLID, 1>(P, S, fw, stream, nb);
    }
}

hipError_t launch_gap(const ProblemView &P, const DeviceState &S, hipStream_t stream, double *out_dev)
{
    int nb = 0;
    hipError_t e = launch_gap_any(P, S, nullptr, stream, &nb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gap_final_kernel, dim3(1), dim3(GAP_FINAL_NT), 0, stream, P, (const double *)S.partials, nb,
                       S.scalars, out_dev, (int32_t *)nullptr, 0.0, 0);
    return hipGetLastError();
}

hipError_t launch_gap_stop(const ProblemView &P, const DeviceState &S, hipStream_t stream, int32_t *stop_w, double eps,
                           int32_t pass)
{
    int nb = 0;
    hipError_t e = launch_gap_any(P, S, nullptr, stream, &nb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gap_final_kernel, dim3(1), dim3(GAP_FINAL_NT), 0, stream, P, (const double *)S.partials, nb,
                       S.scalars, S.meas, stop_w, eps, pass);
    return hipGetLastError();
}

hipError_t launch_gap_fw(const ProblemView &P, const DeviceState &S, const FwSweep &fw, hipStream_t stream, int *nb)
{
    return launch_gap_any(P, S, &fw, stream, nb);
}

}  // namespace srot
