// Bandwidth probe: the HBM bandwidth a plain streaming kernel reaches on this device.
// It gives the measured ceiling the matrix-product kernels are compared against, and a
// copy of known size for calibrating hardware byte counters.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hprlp.h"

namespace {

constexpr int kThreads = 256;

// sum of all float4 entries (one partial per block, so nothing is optimised away)
__global__ __launch_bounds__(kThreads) void stream_read_kernel(const float4* __restrict__ a, int64_t n, float* out) {
    float s = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float4 v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    __shared__ float sh[kThreads];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kThreads) void stream_copy_kernel(const float4* __restrict__ a, float4* __restrict__ b,
                                                               int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        b[i] = a[i];
}

__global__ void fill_kernel(float4* a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        a[i] = make_float4(1.f, 2.f, 3.f, 4.f);
}

}  // namespace

extern "C" int hpr_probe_stream(int64_t bytes, int32_t reps, double* read_gbs, double* copy_gbs) {
    if (bytes < (1 << 20) || reps < 1 || !read_gbs || !copy_gbs) return HPR_ERR_INVALID;
    const int64_t n = bytes / 16;
    float4 *a = nullptr, *b = nullptr;
    float* part = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = HPR_OK;
    const int blocks = 256 * 16;   // 16 blocks per compute unit
    float ms = 0.f;
    if (hipMalloc(&a, n * 16) != hipSuccess || hipMalloc(&b, n * 16) != hipSuccess ||
        hipMalloc(&part, sizeof(float) * blocks) != hipSuccess) {
        rc = HPR_ERR_NOMEM;
        goto done;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = HPR_ERR_HIP;
        goto done;
    }
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(kThreads), 0, 0, a, n);
    hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(kThreads), 0, 0, a, n, part);   // warm-up
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(kThreads), 0, 0, a, n, part);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) {
        rc = HPR_ERR_HIP;
        goto done;
    }
    (void)hipEventElapsedTime(&ms, e0, e1);
    *read_gbs = (double)n * 16 * reps / (ms * 1e-3) / 1e9;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(kThreads), 0, 0, a, b, n);      // warm-up
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(kThreads), 0, 0, a, b, n);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) {
        rc = HPR_ERR_HIP;
        goto done;
    }
    (void)hipEventElapsedTime(&ms, e0, e1);
    *copy_gbs = (double)n * 32 * reps / (ms * 1e-3) / 1e9;   // read + write
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(part);
    return rc;
}
