// Copy-bandwidth probe: the HBM rate a plain streaming kernel reaches on this device, the
// achievable ceiling the rooflines are read against (next to the published 8 TB/s), and the
// reference dispatch of known size for scaling the FETCH_SIZE / WRITE_SIZE counters.
#include <algorithm>

#include "pn_host.hpp"

namespace pn {

// dst[i] = src[i] over n float4s, grid-stride, four independent 16-byte loads in flight per
// thread before their stores.
__global__ void __launch_bounds__(256) copy_probe_kernel(const float4* __restrict__ src,
                                                         float4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                     d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace pn

using namespace pn;

extern "C" pn_status pn_copy_probe(const void* src, void* dst, size_t bytes, int reps,
                                   void* stream, double* gbs) {
    if (!src || !dst || !gbs || reps < 1 || bytes < 16 || (bytes & 15) ||
        ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) {
        set_error("pn_copy_probe: src, dst and gbs must be non-NULL, 16-byte aligned, bytes a "
                  "positive multiple of 16, reps >= 1");
        return PN_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)(bytes / 16);
    const int grid = (int)std::min<int64_t>(8 * (int64_t)cu_count(), (n + 255) / 256);
    hipEvent_t e0, e1;
    PN_HIP(hipEventCreate(&e0));
    PN_HIP(hipEventCreate(&e1));
    // one untimed launch first (first-touch and clocks)
    hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(256), 0, st, (const float4*)src,
                       (float4*)dst, n);
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(256), 0, st,
                           (const float4*)src, (float4*)dst, n);
    (void)hipEventRecord(e1, st);
    pn_status status = PN_OK;
    float ms = 0.f;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) {
        set_error("pn_copy_probe: timing failed");
        status = PN_ERR_HIP;
    } else {
        *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}
