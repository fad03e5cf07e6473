// Plain device-to-device copy of a known size (256 MiB read, 256 MiB
// written, three launches).  Profiling it with the FETCH_SIZE and WRITE_SIZE
// counters gives the factors that turn those counter readings into HBM bytes
// for the solver's kernels.
#include <hip/hip_runtime.h>
#include <cstdio>

__global__ void copy_calibrate_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                      size_t count) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = src[i];
}

int main() {
    const size_t bytes = 256ull << 20;
    float4 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, bytes) != hipSuccess) {
        std::fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemset(src, 1, bytes) != hipSuccess) return 1;
    for (int rep = 0; rep < 3; ++rep)
        hipLaunchKernelGGL(copy_calibrate_kernel, dim3(4096), dim3(256), 0, 0,
                           (const float4 *)src, dst, bytes / sizeof(float4));
    hipError_t e = hipDeviceSynchronize();
    std::printf("copy_calibrate: 3 x %zu bytes read and written: %s\n", bytes, hipGetErrorString(e));
    (void)hipFree(src);
    (void)hipFree(dst);
    return e == hipSuccess ? 0 : 1;
}
