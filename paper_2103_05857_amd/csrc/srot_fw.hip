// Full Frank-Wolfe iteration (Alg. A.1, step eq. AppenEq:SemiRelaxedFWStep)
// on the handle's plan, for gfx950.  One iteration:
//   1. the gap sweep (srot_kernels.hip) gives every row's LMO vertex j*_i
//      and the gap g = <T - S, grad f> with S = (a_i e_{j*_i})_i;
//   2. fw_colsum_kernel / fw_finish_kernel: s = S^T 1 (s_j = sum of a_i over
//      the rows whose vertex is j, rows added in order), d = T^T 1 - s =
//      r + b - s, and the step size: decay 2/(k+2) or the exact line search
//      gamma = clip(g / (w ||d||^2), 0, 1) -- f is quadratic along T -> S
//      with curvature w ||(T - S)^T 1||^2;
//   3. fw_update_rows_kernel: t_i <- (1 - gamma) t_i + gamma a_i e_{j*_i} on
//      the support (bitmasks) and at j*_i; fw_update_r_kernel:
//      r <- (1 - gamma)(r + b) + gamma s - b.
// Every sum has a fixed order, so iterations are bit-reproducible, and the
// host is not involved between iterations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/srot.h"
#include "srot_device.h"
#include "srot_internal.h"

namespace srot {

namespace {

constexpr int FW_NT = 256;

// part[sl * n + j] = sum of a_i over rows i of slice sl with j*_i = j.
__global__ __launch_bounds__(FW_NT) void fw_colsum_kernel(int32_t m, int32_t n, const double *__restrict__ a,
                                                          const int32_t *__restrict__ row_j,
                                                          int rows_per_slice, double *__restrict__ part)
{
    __shared__ int4 sj[FW_NT / 4];
    __shared__ double2 sa[FW_NT / 2];
    const int j = blockIdx.x * FW_NT + threadIdx.x;
    const int sl = blockIdx.y;
    const int i0 = sl * rows_per_slice, i1 = min(m, i0 + rows_per_slice);
    double acc = 0.0;
    for (int c0 = i0; c0 < i1; c0 += FW_NT) {
        const int i = c0 + threadIdx.x;
        reinterpret_cast<int32_t *>(sj)[threadIdx.x] = i < i1 ? row_j[i] : -1;
        reinterpret_cast<double *>(sa)[threadIdx.x] = i < i1 ? a[i] : 0.0;
        __syncthreads();
        // rows in order, four at a time from 16-byte LDS reads (rows past
        // the slice hold column -1 and add nothing)
#pragma unroll 4
        for (int k = 0; k < FW_NT / 4; ++k) {
            const int4 q = sj[k];
            const double2 x = sa[2 * k], y = sa[2 * k + 1];
            acc += (q.x == j) ? x.x : 0.0;
            acc += (q.y == j) ? x.y : 0.0;
            acc += (q.z == j) ? y.x : 0.0;
            acc += (q.w == j) ? y.y : 0.0;
        }
        __syncthreads();
    }
    if (j < n) part[(size_t)sl * n + j] = acc;
}

// s_j (slices added in order), d_j = r_j + b_j - s_j, ||d||^2 by a fixed tree
// over the workgroups (the last one to finish), then the step size.
// scal[0] holds g from the sweep; scal[5] receives gamma, scal[6] ||d||^2.
__global__ __launch_bounds__(FW_NT) void fw_finish_kernel(int32_t n, const double *__restrict__ r,
                                                          const double *__restrict__ b,
                                                          const double *__restrict__ part, int slices,
                                                          double *__restrict__ s_out,
                                                          double *__restrict__ blk,
                                                          int32_t *__restrict__ ticket,
                                                          double *__restrict__ scal, double w, int rule,
                                                          int64_t k, double *__restrict__ trace_gamma)
{
    __shared__ double sh[FW_NT];
    __shared__ int s_last;
    const int j = blockIdx.x * FW_NT + threadIdx.x;
    double dd = 0.0;
    if (j < n) {
        // slices in order; eight requested at a time
        double s = 0.0;
        for (int sl0 = 0; sl0 < slices; sl0 += 8) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (sl0 + q < slices) ? part[(size_t)(sl0 + q) * n + j] : 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) s += v[q];
        }
        s_out[j] = s;
        const double d = (r[j] + b[j]) - s;
        dd = d * d;
    }
    sh[threadIdx.x] = dd;
    __syncthreads();
    for (int h = FW_NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // the block sum travels through a device-scope atomic; the ticket
        // increment depends on its returned value, so it lands first
        unsigned long long seen = __hip_atomic_exchange(reinterpret_cast<unsigned long long *>(blk) + blockIdx.x,
                                                        (unsigned long long)__double_as_longlong(sh[0]),
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int zero;
        asm volatile("v_mov_b32 %0, 0" : "=v"(zero) : "v"((unsigned)(seen ^ (seen >> 32))));
        s_last = (__hip_atomic_fetch_add(ticket, 1 + zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                  (int)gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    double v = 0.0;
    for (int q = threadIdx.x; q < (int)gridDim.x; q += FW_NT)
        v += __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<unsigned long long *>(blk) + q,
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = FW_NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double num = scal[0], den = w * sh[0];
        double gamma;
        if (rule == SROT_DEC) gamma = 2.0 / ((double)k + 2.0);
        else if (!(num > 0.0)) gamma = 0.0;
        else if (den == 0.0 || num >= den) gamma = 1.0;
        else gamma = num / den;
        scal[5] = gamma;
        scal[6] = sh[0];
        if (trace_gamma) trace_gamma[0] = gamma;
        __hip_atomic_store(ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// t_i <- (1 - gamma) t_i + gamma a_i e_{j*_i} on the support and at j*_i.
__global__ __launch_bounds__(FW_NT) void fw_update_rows_kernel(int32_t m, int32_t n, const double *__restrict__ a,
                                                               const int32_t *__restrict__ row_j,
                                                               const double *__restrict__ scal,
                                                               Ownership own, double *__restrict__ T,
                                                               uint32_t *__restrict__ M)
{
    const double gamma = scal[5];
    const int slots = own.words * own.nt;
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const size_t base = (size_t)i * (size_t)n;
        const int js = row_j[i];
        const double gadd = gamma * a[i];
        // owner of the vertex column in the mask layout
        const int jg = js / own.vec;
        const int ts_star = jg % own.nt;
        const int u_star = (jg / own.nt) * own.vec + (js % own.vec);
        for (int s = threadIdx.x; s < slots; s += FW_NT) {
            const int wd = s / own.nt, ts = s - wd * own.nt;
            const uint32_t mk = M[(size_t)i * slots + s];
            uint32_t todo = mk, nm = mk;
            const bool star_here = ts == ts_star && (u_star >> 5) == wd;
            if (star_here) todo |= 1u << (u_star & 31);
            while (todo) {
                const int bt = __ffs(todo) - 1;
                todo &= todo - 1u;
                const int u = wd * 32 + bt;
                const int j = ((u / own.vec) * own.nt + ts) * own.vec + (u % own.vec);
                const bool on = (mk >> bt) & 1u;
                const double t = on ? T[base + j] : 0.0;
                const double tn = (1.0 - gamma) * t + ((j == js) ? gadd : 0.0);
                if (tn != t || !on) T[base + j] = tn;
                nm = (tn != 0.0) ? (nm | (1u << bt)) : (nm & ~(1u << bt));
            }
            if (nm != mk) M[(size_t)i * slots + s] = nm;
        }
    }
}

// r <- (1 - gamma)(r + b) + gamma s - b
__global__ void fw_update_r_kernel(int32_t n, const double *__restrict__ b, const double *__restrict__ s,
                                   const double *__restrict__ scal, double *__restrict__ r)
{
    const double gamma = scal[5];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
        r[j] = (1.0 - gamma) * (r[j] + b[j]) + gamma * s[j] - b[j];
}

}  // namespace

// Row slices of the vertex column sums: at most 95, so the partials and s
// fit in the adjoint's partial buffer (>= 96 n doubles when m >= 32, and 3 m
// n doubles otherwise, with one slice).
static int fw_rows_per_slice(int64_t m)
{
    return (int)std::max<int64_t>(FW_NT, (m + 94) / 95);
}

hipError_t launch_fw_update(const ProblemView &P, const DeviceState &S, int64_t k, int rule,
                            double *trace_gamma, hipStream_t st)
{
    hipError_t e;
    const int rps = fw_rows_per_slice(P.m);
    const int slices = (int)((P.m + rps - 1) / rps);
    const int cb = (P.n + FW_NT - 1) / FW_NT;
    double *part = S.adj_part;
    double *s_vec = S.adj_part + (size_t)slices * (size_t)P.n;
    hipLaunchKernelGGL(fw_colsum_kernel, dim3(cb, slices), dim3(FW_NT), 0, st, P.m, P.n, P.a,
                       (const int32_t *)S.row_j, rps, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // per-workgroup sums of ||d||^2 reuse the gap sweep's partial buffer,
    // sized for both (fw_finish_blocks)
    hipLaunchKernelGGL(fw_finish_kernel, dim3(cb), dim3(FW_NT), 0, st, P.n, (const double *)S.r, P.b,
                       (const double *)part, slices, s_vec, S.partials, S.flags + 5, S.scalars, P.w, rule,
                       k, trace_gamma);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int rb = (int)std::min<int64_t>(P.m, 4096);
    hipLaunchKernelGGL(fw_update_rows_kernel, dim3(rb), dim3(FW_NT), 0, st, P.m, P.n, P.a,
                       (const int32_t *)S.row_j, (const double *)S.scalars, S.own, S.T, S.mask);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(fw_update_r_kernel, dim3(std::min(cb, 1024)), dim3(FW_NT), 0, st, P.n, P.b,
                       (const double *)s_vec, (const double *)S.scalars, S.r);
    return hipGetLastError();
}

hipError_t launch_fw_step(const ProblemView &P, const DeviceState &S, int64_t k, int rule,
                          double *trace_gamma, hipStream_t st)
{
    hipError_t e = launch_gap(P, S, st);
    if (e != hipSuccess) return e;
    return launch_fw_update(P, S, k, rule, trace_gamma, st);
}

int32_t fw_finish_blocks(int64_t n) { return (int32_t)((n + FW_NT - 1) / FW_NT); }

}  // namespace srot
