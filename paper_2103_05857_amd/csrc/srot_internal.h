// Internal declarations shared by the kernel and API translation units of
// libsrot.  Not part of the public interface (include/srot.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace srot {

// Everything a launch needs about one problem.  Device pointers only.
struct ProblemView {
    int32_t m, n;
    int32_t cost;          // SROT_COST_F32 / F64 / SQEUCLID
    const void *C;         // m x n (float or double), or nullptr
    const float *X;        // m x 3
    const float *Y;        // n x 3
    const double *a;       // m
    const double *b;       // n
    double w;
};

// Device state carved out of the caller's workspace.
struct DeviceState {
    double *T;             // m x n dense plan
    double *r;             // n, residual T^T 1 - b
    int32_t *idx;          // index buffer (idx_cap entries)
    int64_t idx_cap;
    double *row_G;         // m, min_j of the block gradient (gap sweep)
    int32_t *row_j;        // m, its lowest argmin
    double *row_g;         // m, per-row gap g_i
    double *partials;      // gap_blocks x 4
    int32_t gap_blocks;
    double *scalars;       // 8: g, f, D, ...
    int32_t *flags;        // 8: [0] validation/index error flag
};

// Launch wrappers (srot_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
hipError_t launch_validate(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_check_indices(const int32_t *idx, int64_t count, int32_t m, int32_t *flag,
                                hipStream_t stream);
hipError_t launch_init_plan(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_residual(const ProblemView &P, const DeviceState &S, hipStream_t stream);
hipError_t launch_sample_uniform(uint64_t seed, int64_t k0, int64_t count, int32_t m,
                                 int32_t *out, hipStream_t stream);
hipError_t launch_sample_permute(uint64_t seed, int64_t p0, int64_t npasses, int32_t m,
                                 int32_t *out, hipStream_t stream);
hipError_t launch_chain(const ProblemView &P, const DeviceState &S, const int32_t *idx,
                        int64_t k0, int64_t nsteps, int rule, int32_t *trace_j,
                        double *trace_gamma, hipStream_t stream);
hipError_t launch_gap(const ProblemView &P, const DeviceState &S, hipStream_t stream);

// Number of workgroups used by the gap sweep for an m-row problem.
int32_t gap_blocks_for(int64_t m);

}  // namespace srot
