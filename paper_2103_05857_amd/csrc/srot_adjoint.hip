// Adjoint of the semi-relaxed OT value V = min_T f(T) at the handle's plan,
// for gfx950.  At an optimal plan T* (residual r*, row multipliers mu) the
// envelope theorem gives the derivatives of V as those of the Lagrangian of
// the problem (App. D) with the plan held fixed:
//
//   dV/dC_ij = t*_ij              dV/db_j = -w r*_j
//   dV/da_i  = mu_i = min_j (c_ij + w r*_j)       (row minimum of the block
//                                                  gradient, eq. RelaxedGradient)
//   dV/dx_i  = 2 sum_j t*_ij (x_i - y_j)          (c_ij = ||x_i - y_j||^2)
//   dV/dy_j  = 2 sum_i t*_ij (y_j - x_i)
//
// every one scaled by the incoming gradient g.  The plan is read through its
// support bitmasks (the column ownership of the step kernels), so the point
// gradients cost O(nnz) gathers plus a scan of the masks; dC is the only
// dense output.  All sums run in FP64 in a fixed order: results are
// bit-reproducible run to run.
//
// Kernels
//   adjoint_rows_kernel   one 256-thread workgroup per row at a time: writes
//                         the row of dC (zeros off the support) and reduces
//                         dX_i over the row's support.
//   adjoint_cols_kernel   column sums for dY: each wave owns 64 mask slots and
//                         8 bit positions, i.e. 8 columns per lane, keeps
//                         their sums in registers over one slice of rows, and
//                         writes per-slice partial sums.
//   adjoint_final_kernel  adds the slices in order (dY), writes db and da.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "../../include/srot.h"
#include "srot_internal.h"

namespace srot {

namespace {

constexpr int ADJ_NT = 256;
constexpr int ADJ_BITS = 8;  // bit positions (columns) per lane in the column kernel

__device__ __forceinline__ int own_col(const Ownership &o, int u, int ts)
{
    return ((u / o.vec) * o.nt + ts) * o.vec + (u % o.vec);
}

// Fixed-order tree sum of three doubles over the 256 threads of a block.
__device__ __forceinline__ void block_sum3(double (&x)[3], double (*sh)[ADJ_NT])
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int d = 0; d < 3; ++d) sh[d][tid] = x[d];
    __syncthreads();
    for (int s = ADJ_NT / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int d = 0; d < 3; ++d) sh[d][tid] += sh[d][tid + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = sh[d][0];
    __syncthreads();
}

template <typename CT>
__global__ __launch_bounds__(ADJ_NT) void adjoint_rows_kernel(ProblemView P, const double *__restrict__ T,
                                                              const uint32_t *__restrict__ M,
                                                              Ownership own, double g,
                                                              CT *__restrict__ dC,
                                                              float *__restrict__ dX)
{
    __shared__ double sh[3][ADJ_NT];
    const int tid = threadIdx.x;
    const int n = P.n;
    const int slots = own.words * own.nt;
    for (int i = blockIdx.x; i < P.m; i += gridDim.x) {
        const size_t base = (size_t)i * (size_t)n;
        double acc[3] = {0.0, 0.0, 0.0};
        double x[3] = {0.0, 0.0, 0.0};
        if (dX) {
            x[0] = P.X[3 * i]; x[1] = P.X[3 * i + 1]; x[2] = P.X[3 * i + 2];
        }
        for (int s = tid; s < slots; s += ADJ_NT) {
            const int wd = s / own.nt, ts = s - wd * own.nt;
            const uint32_t word = M[(size_t)i * slots + s];
            if (dC) {
                for (int bt = 0; bt < 32; ++bt) {
                    const int u = wd * 32 + bt;
                    if (u >= own.cpt) break;
                    const int j = own_col(own, u, ts);
                    if (j < n) dC[base + j] = ((word >> bt) & 1u) ? (CT)(g * T[base + j]) : (CT)0;
                }
            }
            if (dX) {
                uint32_t mk = word;
                while (mk) {
                    const int bt = __ffs(mk) - 1;
                    mk &= mk - 1u;
                    const int j = own_col(own, wd * 32 + bt, ts);
                    const double t = T[base + j];
                    acc[0] += t * (x[0] - (double)P.Y[3 * j]);
                    acc[1] += t * (x[1] - (double)P.Y[3 * j + 1]);
                    acc[2] += t * (x[2] - (double)P.Y[3 * j + 2]);
                }
            }
        }
        if (dX) {  // uniform over the block
            block_sum3(acc, sh);
            if (tid == 0) {
                dX[3 * i] = (float)(2.0 * g * acc[0]);
                dX[3 * i + 1] = (float)(2.0 * g * acc[1]);
                dX[3 * i + 2] = (float)(2.0 * g * acc[2]);
            }
        }
    }
}

// part[(slice * 3 + d) * n + j] = sum over the slice's rows of t_ij (y_jd - x_id).
__global__ __launch_bounds__(ADJ_NT) void adjoint_cols_kernel(ProblemView P, const double *__restrict__ T,
                                                              const uint32_t *__restrict__ M,
                                                              Ownership own, int rows_per_slice,
                                                              double *__restrict__ part)
{
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;  // q: bit group of this wave
    const int n = P.n;
    const int slots = own.words * own.nt;
    const int s = blockIdx.x * 64 + lane;
    const int slice = blockIdx.y;
    const int i0 = slice * rows_per_slice;
    const int i1 = min(P.m, i0 + rows_per_slice);
    const bool live = s < slots;
    const int wd = live ? s / own.nt : 0;
    const int ts = live ? s - wd * own.nt : 0;

    int col[ADJ_BITS];
    double y[ADJ_BITS][3];
    double acc[ADJ_BITS][3];
#pragma unroll
    for (int e = 0; e < ADJ_BITS; ++e) {
        const int u = wd * 32 + q * ADJ_BITS + e;
        int j = (live && u < own.cpt) ? own_col(own, u, ts) : -1;
        if (j >= n) j = -1;
        col[e] = j;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            y[e][d] = (j >= 0) ? (double)P.Y[3 * j + d] : 0.0;
            acc[e][d] = 0.0;
        }
    }
    if (live) {
        for (int i = i0; i < i1; i += 8) {
            uint32_t wv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                wv[k] = (i + k < i1) ? M[(size_t)(i + k) * slots + s] : 0u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t bits = (wv[k] >> (q * ADJ_BITS)) & ((1u << ADJ_BITS) - 1u);
                if (bits == 0u) continue;
                const int ii = i + k;
                const double x0 = P.X[3 * ii], x1 = P.X[3 * ii + 1], x2 = P.X[3 * ii + 2];
                const size_t base = (size_t)ii * (size_t)n;
#pragma unroll
                for (int e = 0; e < ADJ_BITS; ++e) {
                    if (((bits >> e) & 1u) && col[e] >= 0) {
                        const double t = T[base + col[e]];
                        acc[e][0] += t * (y[e][0] - x0);
                        acc[e][1] += t * (y[e][1] - x1);
                        acc[e][2] += t * (y[e][2] - x2);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < ADJ_BITS; ++e) {
        if (col[e] < 0) continue;
#pragma unroll
        for (int d = 0; d < 3; ++d) part[((size_t)slice * 3 + d) * (size_t)n + col[e]] = acc[e][d];
    }
}

__global__ __launch_bounds__(ADJ_NT) void adjoint_final_kernel(ProblemView P, const double *__restrict__ part,
                                                               int slices, const double *__restrict__ r,
                                                               const double *__restrict__ row_G, double g,
                                                               float *__restrict__ dY,
                                                               double *__restrict__ da,
                                                               double *__restrict__ db)
{
    const int n = P.n, m = P.m;
    const int top = max(m, n);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < top; e += gridDim.x * blockDim.x) {
        if (e < n) {
            if (dY) {
                double sum[3] = {0.0, 0.0, 0.0};
                for (int sl = 0; sl < slices; ++sl) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) sum[d] += part[((size_t)sl * 3 + d) * (size_t)n + e];
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) dY[3 * e + d] = (float)(2.0 * g * sum[d]);
            }
            if (db) db[e] = -g * P.w * r[e];
        }
        if (e < m && da) da[e] = g * row_G[e];
    }
}

// Barycentric projection (eq. barycentric_projection): one workgroup per
// row, FP64 sums over the support in a fixed order.  A row without mass
// keeps its own point.
__global__ __launch_bounds__(ADJ_NT) void barycentric_kernel(ProblemView P, const double *__restrict__ T,
                                                             const uint32_t *__restrict__ M, Ownership own,
                                                             float *__restrict__ Xhat)
{
    __shared__ double sh[4][ADJ_NT];
    const int tid = threadIdx.x;
    const int n = P.n;
    const int slots = own.words * own.nt;
    for (int i = blockIdx.x; i < P.m; i += gridDim.x) {
        const size_t base = (size_t)i * (size_t)n;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int s = tid; s < slots; s += ADJ_NT) {
            const int wd = s / own.nt, ts = s - wd * own.nt;
            uint32_t mk = M[(size_t)i * slots + s];
            while (mk) {
                const int bt = __ffs(mk) - 1;
                mk &= mk - 1u;
                const int j = own_col(own, wd * 32 + bt, ts);
                const double t = T[base + j];
                acc[0] += t * (double)P.Y[3 * j];
                acc[1] += t * (double)P.Y[3 * j + 1];
                acc[2] += t * (double)P.Y[3 * j + 2];
                acc[3] += t;
            }
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) sh[d][tid] = acc[d];
        __syncthreads();
        for (int h = ADJ_NT / 2; h > 0; h >>= 1) {
            if (tid < h) {
#pragma unroll
                for (int d = 0; d < 4; ++d) sh[d][tid] += sh[d][tid + h];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double den = sh[3][0];
            for (int d = 0; d < 3; ++d)
                Xhat[3 * i + d] = den > 0.0 ? (float)(sh[d][0] / den) : P.X[3 * i + d];
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_barycentric(const ProblemView &P, const DeviceState &S, float *Xhat, hipStream_t stream)
{
    hipLaunchKernelGGL(barycentric_kernel, dim3((int)std::min<int64_t>(P.m, 4096)), dim3(ADJ_NT), 0, stream, P,
                       (const double *)S.T, (const uint32_t *)S.mask, S.own, Xhat);
    return hipGetLastError();
}

int32_t adjoint_slices_cap(int64_t m) { return (int32_t)std::min<int64_t>(m, 32); }

// Row slices of the dY column sums: enough (slice x column-group)
// workgroups to fill the chip, at most adjoint_slices_cap(m).
static int adjoint_slices(const ProblemView &P, const Ownership &own, int *rows_per_slice)
{
    const int slots = own.words * own.nt;
    const int gx = (slots + 63) / 64;
    const int want = std::max(1, (1024 + gx - 1) / gx);
    const int cap = adjoint_slices_cap(P.m);
    const int rps = (int)((P.m + std::min(want, cap) - 1) / std::min(want, cap));
    if (rows_per_slice) *rows_per_slice = rps;
    return (int)((P.m + rps - 1) / rps);
}

size_t adjoint_part_doubles(const ProblemView &P, const Ownership &own)
{
    return (size_t)adjoint_slices(P, own, nullptr) * 3 * (size_t)P.n;
}

hipError_t launch_adjoint(const ProblemView &P, const DeviceState &S, double g, void *dC,
                          float *dX, float *dY, double *da, double *db, hipStream_t stream)
{
    const Ownership own = S.own;
    if (dC || dX) {
        const int grid = (int)std::min<int64_t>(P.m, 4096);
        if (P.cost == SROT_COST_F64)
            hipLaunchKernelGGL(adjoint_rows_kernel<double>, dim3(grid), dim3(ADJ_NT), 0, stream, P,
                               (const double *)S.T, (const uint32_t *)S.mask, own, g, (double *)dC, dX);
        else
            hipLaunchKernelGGL(adjoint_rows_kernel<float>, dim3(grid), dim3(ADJ_NT), 0, stream, P,
                               (const double *)S.T, (const uint32_t *)S.mask, own, g, (float *)dC, dX);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    int slices = 0;
    if (dY) {
        const int slots = own.words * own.nt;
        const int gx = (slots + 63) / 64;
        int rows_per_slice = 1;
        slices = adjoint_slices(P, own, &rows_per_slice);
        hipLaunchKernelGGL(adjoint_cols_kernel, dim3(gx, slices), dim3(ADJ_NT), 0, stream, P,
                           (const double *)S.T, (const uint32_t *)S.mask, own, rows_per_slice,
                           S.adj_part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (dY || da || db) {
        const int top = (int)std::max<int64_t>(P.m, P.n);
        const int grid = std::max(1, std::min((top + ADJ_NT - 1) / ADJ_NT, 1024));
        hipLaunchKernelGGL(adjoint_final_kernel, dim3(grid), dim3(ADJ_NT), 0, stream, P,
                           (const double *)S.adj_part, slices, (const double *)S.r,
                           (const double *)S.row_G, g, dY, da, db);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace srot
