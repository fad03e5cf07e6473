// The plan in compressed sparse rows, for gfx950: each row's support (the
// active set of Sec. 4.1, eq. ActiveSet: the columns with t_ij > 0) read
// from the support bitmasks, in ascending column order, with its plan
// entries.  Three launches on the handle's stream:
//   plan_count_kernel  one wave per row adds the popcounts of its mask words
//                      into row_ptr[i + 1];
//   plan_scan_kernel   one workgroup turns the counts into row offsets in
//                      place (integer sums: exact in any order), -1 from the
//                      first offset past 2^31 - 1 on;
//   plan_fill_kernel   one wave per row walks its columns 64 at a time: each
//                      lane tests its column's mask bit, the ballot's prefix
//                      popcount gives the entry's place in the row.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/srot.h"
#include "srot_internal.h"

namespace srot {

namespace {

constexpr int PLAN_NT = 256;  // four waves, one row each at a time
constexpr int PLAN_WAVES = PLAN_NT / 64;
constexpr int SCAN_NT = 1024;

__global__ __launch_bounds__(PLAN_NT) void plan_count_kernel(int32_t m, int32_t slots,
                                                             const uint32_t *__restrict__ M,
                                                             int32_t *__restrict__ row_ptr)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * PLAN_WAVES;
    for (int64_t i = (int64_t)blockIdx.x * PLAN_WAVES + (threadIdx.x >> 6); i < m; i += stride) {
        const uint32_t *__restrict__ mrow = M + i * (int64_t)slots;
        int c = 0;
        for (int sl = lane; sl < slots; sl += 64) c += __popc(mrow[sl]);
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) row_ptr[i + 1] = c;
    }
}

__global__ __launch_bounds__(SCAN_NT) void plan_scan_kernel(int32_t m, int32_t *__restrict__ row_ptr)
{
    __shared__ long long sh[SCAN_NT];
    const int t = threadIdx.x;
    const int64_t L = ((int64_t)m + SCAN_NT - 1) / SCAN_NT;
    const int64_t q0 = std::min<int64_t>(m, t * L), q1 = std::min<int64_t>(m, q0 + L);
    long long s = 0;
    for (int64_t q = q0; q < q1; ++q) s += row_ptr[q + 1];
    sh[t] = s;
    __syncthreads();
    if (t == 0) {
        long long run = 0;
        for (int k = 0; k < SCAN_NT; ++k) {
            const long long v = sh[k];
            sh[k] = run;
            run += v;
        }
    }
    __syncthreads();
    long long run = sh[t];
    for (int64_t q = q0; q < q1; ++q) {
        run += row_ptr[q + 1];
        row_ptr[q + 1] = run <= 0x7fffffffLL ? (int32_t)run : -1;
    }
    if (t == 0) row_ptr[0] = 0;
}

__global__ __launch_bounds__(PLAN_NT) void plan_fill_kernel(int32_t m, int32_t n, Ownership own,
                                                            const uint32_t *__restrict__ M,
                                                            const double *__restrict__ T,
                                                            const int32_t *__restrict__ row_ptr,
                                                            int32_t *__restrict__ col, double *__restrict__ val)
{
    const int lane = threadIdx.x & 63;
    const int slots = own.words * own.nt;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t stride = (int64_t)gridDim.x * PLAN_WAVES;
    for (int64_t i = (int64_t)blockIdx.x * PLAN_WAVES + (threadIdx.x >> 6); i < m; i += stride) {
        const uint32_t *__restrict__ mrow = M + i * (int64_t)slots;
        const double *__restrict__ trow = T + i * (int64_t)n;
        int64_t base = row_ptr[i];
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int j = j0 + lane;
            bool bit = false;
            if (j < n) {
                // the mask slot and bit of column j in the ownership layout
                const int jg = j / own.vec;
                const int u = (jg / own.nt) * own.vec + j % own.vec;
                bit = (mrow[(u >> 5) * own.nt + jg % own.nt] >> (u & 31)) & 1u;
            }
            const unsigned long long b = __ballot(bit);
            if (bit) {
                const int64_t e = base + __popcll(b & below);
                col[e] = j;
                val[e] = trow[j];
            }
            base += __popcll(b);
        }
    }
}

}  // namespace

hipError_t launch_plan_count(const ProblemView &P, const DeviceState &S, int32_t *row_ptr, hipStream_t st)
{
    const int slots = S.own.words * S.own.nt;
    const int blocks = (int)std::min<int64_t>(((int64_t)P.m + PLAN_WAVES - 1) / PLAN_WAVES, 4096);
    hipLaunchKernelGGL(plan_count_kernel, dim3(blocks), dim3(PLAN_NT), 0, st, P.m, slots, (const uint32_t *)S.mask,
                       row_ptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(plan_scan_kernel, dim3(1), dim3(SCAN_NT), 0, st, P.m, row_ptr);
    return hipGetLastError();
}

hipError_t launch_plan_fill(const ProblemView &P, const DeviceState &S, const int32_t *row_ptr, int32_t *col,
                            double *val, hipStream_t st)
{
    const int blocks = (int)std::min<int64_t>(((int64_t)P.m + PLAN_WAVES - 1) / PLAN_WAVES, 4096);
    hipLaunchKernelGGL(plan_fill_kernel, dim3(blocks), dim3(PLAN_NT), 0, st, P.m, P.n, S.own,
                       (const uint32_t *)S.mask, (const double *)S.T, row_ptr, col, val);
    return hipGetLastError();
}

}  // namespace srot
