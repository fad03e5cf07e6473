// HIP kernels for block-coordinate Frank-Wolfe on quadratic semi-relaxed OT
// (Fukunaga & Kasai, arXiv:2103.05857), written for gfx950 (CDNA4, wave64).
//
// Orientation: T is m x n, rows are the blocks (T 1 = a exact), the relaxed
// marginal is the column sum with residual r = T^T 1 - b, and w is the
// penalty weight (the paper's 1/lambda).
//
// Kernels
//   chain_reg_kernel  one workgroup runs a sequence of BCFW block steps
//                     (Alg. 1).  Thread `tid` owns columns j = q*NT + tid, so
//                     r_j lives in that thread's registers for the whole launch
//                     and every per-column update is thread-local; only the
//                     LMO argmin and the line-search sums cross threads (one
//                     wave64 butterfly + one LDS exchange, one barrier/step).
//                     The next row of C and T is prefetched during the
//                     current step (the row sequence is known in advance).
//   chain_glb_kernel  same step for n too large for registers: r stays in
//                     global memory (L2) with the same fixed column ownership.
//   gap_kernel        per-pass duality-gap sweep (Thm 2): one wave per row,
//                     streams the row of C and T once, HBM bound.
//   gap_final_kernel  deterministic fixed-order reduction of the sweep.
//   sample kernels    counter-based Philox4x64-10 block indices.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <type_traits>

#include "../../include/srot.h"
#include "srot_internal.h"

namespace srot {

// ---------------------------------------------------------------------------
// LMO + line-search partial over a set of columns of one block.
//
// For the block gradient v_j = c_ij + w r_j of row i and its plan entries t_j:
//   v, j   smallest v and its lowest index (the LMO vertex,
//          eq. SemiRelaxedSubproblemImplement, ties to the lowest index)
//   t      t_j at that index
//   Q      sum of t_j^2 over the other columns of the set
//   P      sum of t_j (v_j - v)   (>= 0 term by term)
//   Ts     sum of t_j
// With s_i = a_i e_j*, the exact line search (eq. SemiRelaxedBCFWStep) needs
//   <t_i - s_i, grad_i f> = P + (Ts - a_i) v  ~  P   (row sums equal a_i)
//   ||t_i - s_i||^2       = Q + (t - a_i)^2
// Both are accumulated without cancellation: when the running minimum moves
// down, earlier terms grow by (old v - new v) * Ts, and the displaced
// winner's t^2 joins Q.
// ---------------------------------------------------------------------------
struct ArgPart {
    double v, t, Q, P, Ts;
    int j;
};

__device__ __forceinline__ void part_init(ArgPart &p)
{
    p.v = INFINITY; p.t = 0.0; p.Q = 0.0; p.P = 0.0; p.Ts = 0.0; p.j = 0x7fffffff;
}

// Columns must be pushed in increasing j within one partial.
__device__ __forceinline__ void part_push(ArgPart &p, double v, double t, int j)
{
    if (v < p.v) {
        if (p.Ts != 0.0) p.P += (p.v - v) * p.Ts;
        p.Q += p.t * p.t;
        p.v = v; p.t = t; p.j = j;
    } else {
        p.Q += t * t;
        p.P += t * (v - p.v);
    }
    p.Ts += t;
}

// Symmetric in (A, B) bit for bit: every sum is formed from commutative pairs.
__device__ __forceinline__ ArgPart part_merge(const ArgPart &A, const ArgPart &B)
{
    const bool bw = (B.v < A.v) || (B.v == A.v && B.j < A.j);
    const ArgPart &W = bw ? B : A;
    const ArgPart &L = bw ? A : B;
    ArgPart o;
    o.v = W.v; o.t = W.t; o.j = W.j;
    o.Q = (A.Q + B.Q) + L.t * L.t;
    const double pa = (A.Ts != 0.0) ? (A.v - W.v) * A.Ts : 0.0;
    const double pb = (B.Ts != 0.0) ? (B.v - W.v) * B.Ts : 0.0;
    o.P = (A.P + B.P) + (pa + pb);
    o.Ts = A.Ts + B.Ts;
    return o;
}

__device__ __forceinline__ ArgPart part_shfl_xor(const ArgPart &p, int off)
{
    ArgPart o;
    o.v = __shfl_xor(p.v, off);
    o.t = __shfl_xor(p.t, off);
    o.Q = __shfl_xor(p.Q, off);
    o.P = __shfl_xor(p.P, off);
    o.Ts = __shfl_xor(p.Ts, off);
    o.j = __shfl_xor(p.j, off);
    return o;
}

__device__ __forceinline__ ArgPart wave_reduce(ArgPart p)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) p = part_merge(p, part_shfl_xor(p, off));
    return p;
}

// Block-wide reduction; every thread returns the same result (waves merged in
// a fixed order).  `sh` must not be reused until one more barrier has passed
// (callers alternate two slots).
template <int NW>
__device__ __forceinline__ ArgPart block_reduce(ArgPart p, ArgPart *sh)
{
    p = wave_reduce(p);
    if (NW == 1) return p;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = p;
    __syncthreads();
    ArgPart res = sh[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) res = part_merge(res, sh[k]);
    return res;
}

// Step size of Alg. 1: decay 2m/(k+2m), or the exact line search
// (eq. SemiRelaxedBCFWStep) restricted to [0, 1]; with a vanishing
// denominator the objective is linear along the segment.
__device__ __forceinline__ double step_size(int rule, int64_t k, int32_t m, double w,
                                            const ArgPart &res, double ai)
{
    if (rule == SROT_DEC) return (2.0 * (double)m) / ((double)k + 2.0 * (double)m);
    const double num = res.P;
    const double dt = res.t - ai;
    const double den = w * (res.Q + dt * dt);
    if (!(num > 0.0)) return 0.0;
    if (den == 0.0 || num >= den) return 1.0;
    return num / den;
}

__device__ __forceinline__ double sqdist(float x0, float x1, float x2, float y0, float y1, float y2)
{
    const double d0 = (double)x0 - (double)y0;
    const double d1 = (double)x1 - (double)y1;
    const double d2 = (double)x2 - (double)y2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

// ---------------------------------------------------------------------------
// Block-step chain, r in registers.  Requires n <= NT * CPT.
// ---------------------------------------------------------------------------
template <int NT, int CPT, int COST>
__global__ __launch_bounds__(NT) void chain_reg_kernel(ProblemView P, double *__restrict__ T,
                                                       double *__restrict__ rg,
                                                       const int32_t *__restrict__ idx, int64_t k0,
                                                       int64_t nsteps, int rule,
                                                       int32_t *__restrict__ trace_j,
                                                       double *__restrict__ trace_gamma)
{
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr int NW = NT / 64;
    __shared__ ArgPart sh[2][NW];
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;

    double r[CPT];
    float y0[CPT], y1[CPT], y2[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = q * NT + tid;
        r[q] = (j < n) ? rg[j] : 0.0;
        if constexpr (COST == SROT_COST_SQEUCLID) {
            y0[q] = (j < n) ? P.Y[3 * j + 0] : 0.f;
            y1[q] = (j < n) ? P.Y[3 * j + 1] : 0.f;
            y2[q] = (j < n) ? P.Y[3 * j + 2] : 0.f;
        }
    }

    CT c_cur[CPT], c_nxt[CPT];
    double t_cur[CPT], t_nxt[CPT];
    float x_cur[3] = {0.f, 0.f, 0.f}, x_nxt[3] = {0.f, 0.f, 0.f};

    auto load_row = [&](int i, CT (&c)[CPT], double (&t)[CPT], float (&x)[3]) {
        const size_t base = (size_t)i * (size_t)n;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int j = q * NT + tid;
            if (j < n) {
                if constexpr (COST != SROT_COST_SQEUCLID) c[q] = C[base + j];
                t[q] = T[base + j];
            } else {
                if constexpr (COST != SROT_COST_SQEUCLID) c[q] = (CT)0;
                t[q] = 0.0;
            }
        }
        if constexpr (COST == SROT_COST_SQEUCLID) {
            x[0] = P.X[3 * i + 0]; x[1] = P.X[3 * i + 1]; x[2] = P.X[3 * i + 2];
        }
    };

    int i_cur = idx[0];
    load_row(i_cur, c_cur, t_cur, x_cur);

    for (int64_t s = 0; s < nsteps; ++s) {
        int i_nxt = i_cur;
        if (s + 1 < nsteps) {
            i_nxt = idx[s + 1];
            load_row(i_nxt, c_nxt, t_nxt, x_nxt);
        }
        const double ai = P.a[i_cur];

        // block gradient c_i + w r (eq. RelaxedGradient) and the partial LMO
        ArgPart p;
        part_init(p);
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int j = q * NT + tid;
            if (j < n) {
                double c;
                if constexpr (COST == SROT_COST_SQEUCLID)
                    c = sqdist(x_cur[0], x_cur[1], x_cur[2], y0[q], y1[q], y2[q]);
                else
                    c = (double)c_cur[q];
                part_push(p, c + w * r[q], t_cur[q], j);
            }
        }
        const ArgPart res = block_reduce<NW>(p, sh[s & 1]);
        const double gamma = step_size(rule, k0 + s, m, w, res, ai);

        // t_i <- (1 - gamma) t_i + gamma a_i e_j*;  r <- r + (t_i new - t_i old)
        const size_t base = (size_t)i_cur * (size_t)n;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int j = q * NT + tid;
            if (j < n) {
                const double sv = (j == res.j) ? ai : 0.0;
                const double tn = (1.0 - gamma) * t_cur[q] + gamma * sv;
                r[q] += tn - t_cur[q];
                if (tn != t_cur[q]) T[base + j] = tn;
                t_cur[q] = tn;
            }
        }
        if (tid == 0) {
            if (trace_j) trace_j[s] = res.j;
            if (trace_gamma) trace_gamma[s] = gamma;
        }
        // the prefetched copy of a row updated in this step is stale
        if (s + 1 < nsteps) {
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                if (i_nxt == i_cur) t_nxt[q] = t_cur[q];
                t_cur[q] = t_nxt[q];
                if constexpr (COST != SROT_COST_SQEUCLID) c_cur[q] = c_nxt[q];
            }
            x_cur[0] = x_nxt[0]; x_cur[1] = x_nxt[1]; x_cur[2] = x_nxt[2];
            i_cur = i_nxt;
        }
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int j = q * NT + tid;
        if (j < n) rg[j] = r[q];
    }
}

// ---------------------------------------------------------------------------
// Block-step chain for any n: r in global memory, column j owned by thread
// j mod GLB_NT for reads and writes, so no cross-thread hazard on r or T.
// ---------------------------------------------------------------------------
constexpr int GLB_NT = 512;

template <int COST>
__global__ __launch_bounds__(GLB_NT) void chain_glb_kernel(ProblemView P, double *__restrict__ T,
                                                         double *__restrict__ rg,
                                                         const int32_t *__restrict__ idx,
                                                         int64_t k0, int64_t nsteps, int rule,
                                                         int32_t *__restrict__ trace_j,
                                                         double *__restrict__ trace_gamma)
{
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr int NT = GLB_NT, NW = NT / 64;
    __shared__ ArgPart sh[2][NW];
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;

    for (int64_t s = 0; s < nsteps; ++s) {
        const int i = idx[s];
        const double ai = P.a[i];
        const size_t base = (size_t)i * (size_t)n;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if constexpr (COST == SROT_COST_SQEUCLID) {
            x0 = P.X[3 * i]; x1 = P.X[3 * i + 1]; x2 = P.X[3 * i + 2];
        }
        ArgPart p;
        part_init(p);
        for (int j = tid; j < n; j += NT) {
            double c;
            if constexpr (COST == SROT_COST_SQEUCLID)
                c = sqdist(x0, x1, x2, P.Y[3 * j], P.Y[3 * j + 1], P.Y[3 * j + 2]);
            else
                c = (double)C[base + j];
            part_push(p, c + w * rg[j], T[base + j], j);
        }
        const ArgPart res = block_reduce<NW>(p, sh[s & 1]);
        const double gamma = step_size(rule, k0 + s, m, w, res, ai);
        for (int j = tid; j < n; j += NT) {
            const double t = T[base + j];
            const double sv = (j == res.j) ? ai : 0.0;
            const double tn = (1.0 - gamma) * t + gamma * sv;
            if (tn != t) {
                T[base + j] = tn;
                rg[j] += tn - t;
            }
        }
        if (tid == 0) {
            if (trace_j) trace_j[s] = res.j;
            if (trace_gamma) trace_gamma[s] = gamma;
        }
    }
}

// ---------------------------------------------------------------------------
// Gap sweep (Thm 2, eq. AppenEq:Gi, dual of App. D).  One wave per row:
//   G_i = min_j v_ij (lowest argmin j*_i),  g_i = sum_j t_ij (v_ij - G_i),
//   lin_i = sum_j t_ij c_ij.
// Per block: sums of a_i G_i, lin_i and g_i, in row order per wave and wave
// order per block; gap_final_kernel adds the blocks in order.
// ---------------------------------------------------------------------------
struct GapPart {
    double v, P, Ts, lin;
    int j;
};

__device__ __forceinline__ void gpart_push(GapPart &p, double v, double t, double c, int j)
{
    if (v < p.v) {
        if (p.Ts != 0.0) p.P += (p.v - v) * p.Ts;
        p.v = v; p.j = j;
    } else {
        p.P += t * (v - p.v);
    }
    p.Ts += t;
    p.lin += t * c;
}

__device__ __forceinline__ GapPart gpart_merge(const GapPart &A, const GapPart &B)
{
    const bool bw = (B.v < A.v) || (B.v == A.v && B.j < A.j);
    const GapPart &W = bw ? B : A;
    GapPart o;
    o.v = W.v; o.j = W.j;
    const double pa = (A.Ts != 0.0) ? (A.v - W.v) * A.Ts : 0.0;
    const double pb = (B.Ts != 0.0) ? (B.v - W.v) * B.Ts : 0.0;
    o.P = (A.P + B.P) + (pa + pb);
    o.Ts = A.Ts + B.Ts;
    o.lin = A.lin + B.lin;
    return o;
}

constexpr int GAP_NT = 256;

template <int COST>
__global__ __launch_bounds__(GAP_NT) void gap_kernel(ProblemView P, const double *__restrict__ T,
                                                     const double *__restrict__ rg,
                                                     double *__restrict__ row_G,
                                                     int32_t *__restrict__ row_j,
                                                     double *__restrict__ row_g,
                                                     double *__restrict__ partials)
{
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr int NW = GAP_NT / 64;
    __shared__ double sh[NW][3];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;
    const int gw = blockIdx.x * NW + wid;
    const int nw_total = gridDim.x * NW;

    double acc_aG = 0.0, acc_lin = 0.0, acc_g = 0.0;
    for (int i = gw; i < m; i += nw_total) {
        const size_t base = (size_t)i * (size_t)n;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if constexpr (COST == SROT_COST_SQEUCLID) {
            x0 = P.X[3 * i]; x1 = P.X[3 * i + 1]; x2 = P.X[3 * i + 2];
        }
        GapPart p;
        p.v = INFINITY; p.P = 0.0; p.Ts = 0.0; p.lin = 0.0; p.j = 0x7fffffff;
        for (int j = lane; j < n; j += 64) {
            double c;
            if constexpr (COST == SROT_COST_SQEUCLID)
                c = sqdist(x0, x1, x2, P.Y[3 * j], P.Y[3 * j + 1], P.Y[3 * j + 2]);
            else
                c = (double)C[base + j];
            gpart_push(p, c + w * rg[j], T[base + j], c, j);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            GapPart o;
            o.v = __shfl_xor(p.v, off);
            o.P = __shfl_xor(p.P, off);
            o.Ts = __shfl_xor(p.Ts, off);
            o.lin = __shfl_xor(p.lin, off);
            o.j = __shfl_xor(p.j, off);
            p = gpart_merge(p, o);
        }
        if (lane == 0) {
            row_G[i] = p.v;
            row_j[i] = p.j;
            row_g[i] = p.P;
            acc_aG += P.a[i] * p.v;
            acc_lin += p.lin;
            acc_g += p.P;
        }
    }
    if (lane == 0) {
        sh[wid][0] = acc_aG; sh[wid][1] = acc_lin; sh[wid][2] = acc_g;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < NW; ++k) { s0 += sh[k][0]; s1 += sh[k][1]; s2 += sh[k][2]; }
        partials[4 * blockIdx.x + 0] = s0;
        partials[4 * blockIdx.x + 1] = s1;
        partials[4 * blockIdx.x + 2] = s2;
    }
}

// Fixed-order tree reduction of a per-thread value over a 256-thread block.
__device__ double block_sum_256(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

// g = sum g_i;  f = <T,C> + (w/2)||r||^2;
// D = sum a_i G_i - w <b, r> - (w/2)||r||^2   (App. D dual with
//     sum_i <t_i, grad_i f> = <T,C> + w <r + b, r>).
__global__ __launch_bounds__(256) void gap_final_kernel(ProblemView P, const double *__restrict__ rg,
                                                        const double *__restrict__ partials,
                                                        int nparts, double *__restrict__ out)
{
    __shared__ double sh[256];
    double aG = 0.0, lin = 0.0, g = 0.0, rr = 0.0, br = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) {
        aG += partials[4 * k + 0];
        lin += partials[4 * k + 1];
        g += partials[4 * k + 2];
    }
    for (int j = threadIdx.x; j < P.n; j += 256) {
        rr += rg[j] * rg[j];
        br += P.b[j] * rg[j];
    }
    aG = block_sum_256(aG, sh);
    lin = block_sum_256(lin, sh);
    g = block_sum_256(g, sh);
    rr = block_sum_256(rr, sh);
    br = block_sum_256(br, sh);
    if (threadIdx.x == 0) {
        out[0] = g;
        out[1] = lin + 0.5 * P.w * rr;
        out[2] = aG - P.w * br - 0.5 * P.w * rr;
        out[3] = lin;
        out[4] = rr;
    }
}

// ---------------------------------------------------------------------------
// Initial plan t_i = a_i e_0, residual, validation.
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

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// multiply / xor-swap round with Weyl key schedule.  Output k of the stream
// with key (seed, 0) is lane k mod 4 of the block at counter 1 + floor(k/4)
// (the counter convention of numpy's Philox bit generator).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
#pragma unroll
    for (int rd = 0; rd < 10; ++rd) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

__device__ __forceinline__ uint64_t philox_output(uint64_t seed, uint64_t k)
{
    uint64_t c[4] = {(k >> 2) + 1ull, 0ull, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
    return c[k & 3];
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
    __shared__ uint64_t tile[256];
    const int64_t p = p0 + blockIdx.x;
    int32_t *o = out + (int64_t)blockIdx.x * m;
    for (int32_t tb = 0; tb < m; tb += 256) {
        const int32_t t = tb + threadIdx.x;
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
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
static int grid_for(size_t work, int nt, int cap)
{
    size_t g = (work + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
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
    hipLaunchKernelGGL(sample_permute_kernel, dim3((unsigned)npasses), dim3(256), 0, stream, seed,
                       p0, m, out);
    return hipGetLastError();
}

// Register-resident variants (NT threads x CPT columns per thread).
struct ChainVariant {
    int nt, cpt;
};
static const ChainVariant kChainVariants[] = {
    {64, 1}, {64, 2}, {64, 4}, {128, 4}, {256, 4}, {256, 8}, {256, 16}, {512, 8},
};

// Default choice: the fewest threads with at most 16 columns each, except
// that small rows keep one wave.  SROT_CHAIN_VARIANT=<nt>x<cpt> overrides it
// (used by the tuner); n above 4096 takes the global-residual kernel.
static ChainVariant pick_chain_variant(int n)
{
    const char *env = getenv("SROT_CHAIN_VARIANT");
    if (env) {
        int nt = 0, cpt = 0;
        if (sscanf(env, "%dx%d", &nt, &cpt) == 2) {
            for (const ChainVariant &v : kChainVariants)
                if (v.nt == nt && v.cpt == cpt && n <= nt * cpt) return v;
        }
    }
    if (n <= 64) return {64, 1};
    if (n <= 128) return {64, 2};
    if (n <= 256) return {64, 4};
    if (n <= 512) return {128, 4};
    if (n <= 1024) return {256, 4};
    if (n <= 2048) return {256, 8};
    if (n <= 4096) return {256, 16};
    return {0, 0};
}

template <int COST>
static hipError_t launch_chain_cost(const ProblemView &P, const DeviceState &S, const int32_t *idx,
                                    int64_t k0, int64_t nsteps, int rule, int32_t *tj, double *tg,
                                    hipStream_t st)
{
    const ChainVariant v = pick_chain_variant(P.n);
#define SROT_CHAIN(NT_, CPT_)                                                                      \
    if (v.nt == NT_ && v.cpt == CPT_) {                                                            \
        hipLaunchKernelGGL((chain_reg_kernel<NT_, CPT_, COST>), dim3(1), dim3(NT_), 0, st, P, S.T,   \
                           S.r, idx, k0, nsteps, rule, tj, tg);                                    \
        return hipGetLastError();                                                                  \
    }
    SROT_CHAIN(64, 1)
    SROT_CHAIN(64, 2)
    SROT_CHAIN(64, 4)
    SROT_CHAIN(128, 4)
    SROT_CHAIN(256, 4)
    SROT_CHAIN(256, 8)
    SROT_CHAIN(256, 16)
    SROT_CHAIN(512, 8)
#undef SROT_CHAIN
    hipLaunchKernelGGL((chain_glb_kernel<COST>), dim3(1), dim3(GLB_NT), 0, st, P, S.T, S.r, idx, k0,
                       nsteps, rule, tj, tg);
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

int32_t gap_blocks_for(int64_t m)
{
    // one wave per row, 4 waves per block; at most 2048 blocks (8 per CU)
    int64_t b = (m + 3) / 4;
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int32_t)b;
}

hipError_t launch_gap(const ProblemView &P, const DeviceState &S, hipStream_t stream)
{
    const int nb = S.gap_blocks;
    switch (P.cost) {
    case SROT_COST_F32:
        hipLaunchKernelGGL(gap_kernel<SROT_COST_F32>, dim3(nb), dim3(GAP_NT), 0, stream, P, S.T, S.r,
                           S.row_G, S.row_j, S.row_g, S.partials);
        break;
    case SROT_COST_F64:
        hipLaunchKernelGGL(gap_kernel<SROT_COST_F64>, dim3(nb), dim3(GAP_NT), 0, stream, P, S.T, S.r,
                           S.row_G, S.row_j, S.row_g, S.partials);
        break;
    default:
        hipLaunchKernelGGL(gap_kernel<SROT_COST_SQEUCLID>, dim3(nb), dim3(GAP_NT), 0, stream, P, S.T,
                           S.r, S.row_G, S.row_j, S.row_g, S.partials);
        break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gap_final_kernel, dim3(1), dim3(256), 0, stream, P, S.r, S.partials, nb,
                       S.scalars);
    return hipGetLastError();
}

}  // namespace srot
