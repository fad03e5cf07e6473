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
//   gap_kernel        per-pass duality-gap sweep (Thm 2), one workgroup per
//                     row at a time, streaming the cost row once: HBM bound.
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
                                                   int64_t *__restrict__ resume)
{
    const int64_t done = chain_fast<NT, CPT, VEC, COST, TRACE>(P, T, rg, M, idx, k0, nsteps, rule,
                                                               trace_j, trace_gamma);
    if (threadIdx.x == 0) *resume = done;
}

template <int NT, int CPT, int VEC, int COST>
__global__ __launch_bounds__(NT) void chain_tail_kernel(ProblemView P, double *__restrict__ T,
                                                        double *__restrict__ rg,
                                                        uint32_t *__restrict__ M,
                                                        const int32_t *__restrict__ idx, int64_t k0,
                                                        int64_t nsteps, int rule,
                                                        int32_t *__restrict__ trace_j,
                                                        double *__restrict__ trace_gamma,
                                                        const int64_t *__restrict__ resume)
{
    chain_tail<NT, CPT, VEC, COST>(P, T, rg, M, idx, k0, *resume, nsteps, rule, trace_j, trace_gamma);
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
                                                           double *__restrict__ trace_gamma)
{
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NT = GLB_NT, NW = NT / 64;
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
// Gap sweep (Thm 2, eq. AppenEq:Gi, dual of App. D).  One workgroup handles
// one row at a time with the handle's column ownership:
//   G_i = min_j v_ij (lowest argmin j*_i),  g_i = sum_j t_ij (v_ij - G_i),
//   lin_i = sum_j t_ij c_ij   (sums over the support only).
// Thread 0 accumulates a_i G_i, lin_i and g_i over its rows in row order;
// gap_final_kernel adds the workgroups in order.
// CPT > 0: r held in registers (n <= NT * CPT); CPT == 0: r read from memory
// (VEC must be 1 then).
// ---------------------------------------------------------------------------
template <int NT, int CPT, int VEC, int COST>
__global__ __launch_bounds__(NT) void gap_kernel(ProblemView P, const double *__restrict__ T,
                                                 const double *__restrict__ rg,
                                                 const uint32_t *__restrict__ M, int words,
                                                 double *__restrict__ row_G,
                                                 int32_t *__restrict__ row_j,
                                                 double *__restrict__ row_g,
                                                 double *__restrict__ partials)
{
    using CT = typename std::conditional<COST == SROT_COST_F32, float, double>::type;
    constexpr bool FUSED = (COST == SROT_COST_SQEUCLID);
    constexpr int NW = NT / 64;
    constexpr int RC = CPT > 0 ? CPT : 1;
    __shared__ double s_v[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_sum[2][NW][2];
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    const double w = P.w;
    const CT *__restrict__ C = (const CT *)P.C;

    double r[RC];
    if constexpr (CPT > 0) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int j = owned_col<NT, VEC>(u, tid);
            r[u] = (j < n) ? rg[j] : 0.0;
        }
    }
    auto cost = [&](int i, int j, float x0, float x1, float x2) -> double {
        if constexpr (FUSED) return sqdist(x0, x1, x2, P.Y[3 * j], P.Y[3 * j + 1], P.Y[3 * j + 2]);
        else return (double)C[(size_t)i * (size_t)n + j];
    };

    double acc_aG = 0.0, acc_lin = 0.0, acc_g = 0.0;
    int par = 0;
    for (int i = blockIdx.x; i < m; i += gridDim.x, par ^= 1) {
        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
        if constexpr (FUSED) { x0 = P.X[3 * i]; x1 = P.X[3 * i + 1]; x2 = P.X[3 * i + 2]; }
        double best = INFINITY;
        int bj = 0x7fffffff;
        if constexpr (CPT > 0) {
            CT cv[RC];
            if constexpr (!FUSED) load_cost_row<NT, CPT, VEC, CT>(C + (size_t)i * (size_t)n, n, tid, cv);
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int j = owned_col<NT, VEC>(u, tid);
                double c;
                if constexpr (FUSED) c = (j < n) ? cost(i, j, x0, x1, x2) : 0.0;
                else c = (double)cv[u];
                const double v = (j < n) ? c + w * r[u] : INFINITY;
                if (v < best) { best = v; bj = j; }
            }
        } else {
            for (int j = tid; j < n; j += NT) {
                const double v = cost(i, j, x0, x1, x2) + w * rg[j];
                if (v < best) { best = v; bj = j; }
            }
        }
        block_argmin<NW>(best, bj, s_v[par], s_j[par]);
        const double G = best;

        double acc[2] = {0.0, 0.0};  // g_i, lin_i
        const uint32_t *Mi = M + (size_t)i * words * NT + tid;
        const size_t base = (size_t)i * (size_t)n;
        for (int wd = 0; wd < words; ++wd) {
            uint32_t mk = Mi[(size_t)wd * NT];
            while (mk) {
                const int b = __ffs(mk) - 1;
                mk &= mk - 1u;
                const int u = wd * 32 + b;
                int j;
                double rj;
                if constexpr (CPT > 0) {
                    j = owned_col<NT, VEC>(u, tid);
                    rj = 0.0;
#pragma unroll
                    for (int q = 0; q < CPT; ++q) rj = (q == u) ? r[q] : rj;
                } else {
                    j = u * NT + tid;
                    rj = rg[j];
                }
                const double t = T[base + j];
                const double c = cost(i, j, x0, x1, x2);
                acc[0] += t * (c + w * rj - G);
                acc[1] += t * c;
            }
        }
        block_sum<NW, 2>(acc, s_sum[par]);
        if (tid == 0) {
            row_G[i] = G;
            row_j[i] = bj;
            row_g[i] = acc[0];
            acc_aG += P.a[i] * G;
            acc_lin += acc[1];
            acc_g += acc[0];
        }
    }
    if (tid == 0) {
        partials[4 * blockIdx.x + 0] = acc_aG;
        partials[4 * blockIdx.x + 1] = acc_lin;
        partials[4 * blockIdx.x + 2] = acc_g;
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

// Target points padded to 16 bytes (one vector load per point).
__global__ void pad_points_kernel(int32_t n, const float *__restrict__ Y, float4 *__restrict__ Y4)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        Y4[j] = make_float4(Y[3 * j], Y[3 * j + 1], Y[3 * j + 2], 0.f);
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
    hipLaunchKernelGGL(pad_points_kernel, dim3(grid_for((size_t)P.n, 256, 1024)), dim3(256), 0, stream,
                       P.n, P.Y, const_cast<float4 *>(P.Y4));
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
    hipLaunchKernelGGL(sample_permute_kernel, dim3((unsigned)npasses), dim3(256), 0, stream, seed,
                       p0, m, out);
    return hipGetLastError();
}

template <int COST>
static hipError_t launch_chain_cost(const ProblemView &P, const DeviceState &S, const int32_t *idx,
                                    int64_t k0, int64_t nsteps, int rule, int32_t *tj, double *tg,
                                    hipStream_t st)
{
    const Ownership &o = S.own;
    if (o.reg) {
#define SROT_CHAIN(NT_, CPT_, VEC_)                                                                \
        if (o.nt == NT_ && o.cpt == CPT_ && o.vec == VEC_) {                                       \
            if (tj || tg)                                                                          \
                hipLaunchKernelGGL((chain_kernel<NT_, CPT_, VEC_, COST, true>), dim3(1), dim3(NT_), 0, \
                                   st, P, S.T, S.r, S.mask, idx, k0, nsteps, rule, tj, tg, S.resume); \
            else                                                                                   \
                hipLaunchKernelGGL((chain_kernel<NT_, CPT_, VEC_, COST, false>), dim3(1), dim3(NT_),  \
                                   0, st, P, S.T, S.r, S.mask, idx, k0, nsteps, rule, tj, tg,       \
                                   S.resume);                                                      \
            hipError_t e_ = hipGetLastError();                                                     \
            if (e_ != hipSuccess) return e_;                                                       \
            hipLaunchKernelGGL((chain_tail_kernel<NT_, CPT_, VEC_, COST>), dim3(1), dim3(NT_), 0,    \
                               st, P, S.T, S.r, S.mask, idx, k0, nsteps, rule, tj, tg, S.resume);  \
            return hipGetLastError();                                                              \
        }
        SROT_VARIANTS_V1(SROT_CHAIN)
        if constexpr (COST == SROT_COST_F32) { SROT_VARIANTS_V4(SROT_CHAIN) }
        if constexpr (COST == SROT_COST_F64) { SROT_VARIANTS_V2(SROT_CHAIN) }
#undef SROT_CHAIN
        return hipErrorInvalidConfiguration;
    }
    hipLaunchKernelGGL((chain_glb_kernel<COST>), dim3(1), dim3(GLB_NT), 0, st, P, S.T, S.r, S.mask,
                       o.words, idx, k0, nsteps, rule, tj, tg);
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
    int64_t b = m;
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int32_t)b;
}

template <int COST>
static hipError_t launch_gap_cost(const ProblemView &P, const DeviceState &S, hipStream_t st)
{
    const Ownership &o = S.own;
    const int nb = S.gap_blocks;
    if (o.reg) {
#define SROT_GAP(NT_, CPT_, VEC_)                                                                  \
        if (o.nt == NT_ && o.cpt == CPT_ && o.vec == VEC_) {                                       \
            hipLaunchKernelGGL((gap_kernel<NT_, CPT_, VEC_, COST>), dim3(nb), dim3(NT_), 0, st, P,   \
                               S.T, S.r, S.mask, o.words, S.row_G, S.row_j, S.row_g, S.partials);  \
            return hipGetLastError();                                                              \
        }
        SROT_VARIANTS_V1(SROT_GAP)
        if constexpr (COST == SROT_COST_F32) { SROT_VARIANTS_V4(SROT_GAP) }
        if constexpr (COST == SROT_COST_F64) { SROT_VARIANTS_V2(SROT_GAP) }
#undef SROT_GAP
        return hipErrorInvalidConfiguration;
    }
    hipLaunchKernelGGL((gap_kernel<GLB_NT, 0, 1, COST>), dim3(nb), dim3(GLB_NT), 0, st, P, S.T, S.r,
                       S.mask, o.words, S.row_G, S.row_j, S.row_g, S.partials);
    return hipGetLastError();
}

hipError_t launch_gap(const ProblemView &P, const DeviceState &S, hipStream_t stream)
{
    hipError_t e;
    switch (P.cost) {
    case SROT_COST_F32: e = launch_gap_cost<SROT_COST_F32>(P, S, stream); break;
    case SROT_COST_F64: e = launch_gap_cost<SROT_COST_F64>(P, S, stream); break;
    default: e = launch_gap_cost<SROT_COST_SQEUCLID>(P, S, stream); break;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gap_final_kernel, dim3(1), dim3(256), 0, stream, P, S.r, S.partials,
                       S.gap_blocks, S.scalars);
    return hipGetLastError();
}

}  // namespace srot
