// Copy-bandwidth probe: the HBM rate a plain streaming kernel reaches on this device, the
// achievable ceiling the rooflines are read against (next to the published 8 TB/s), and
// reference dispatches of known size for scaling the FETCH_SIZE / WRITE_SIZE counters.
#include <algorithm>

#include "pn_host.hpp"

namespace pn {

typedef float pnv4 __attribute__((ext_vector_type(4)));

// dst[i] = src[i] over n 16-byte elements, grid-stride.  FORM 0: four independent loads in
// flight per thread (a grid stride apart) before their stores; FORM 1: one element per thread
// and iteration, loads and stores with the non-temporal hint.  Which one streams faster
// depends on the grid (DRAM page locality of the waves in flight), so the probe times both.
template <int FORM>
__global__ void __launch_bounds__(256) copy_probe_kernel(const pnv4* __restrict__ src,
                                                         pnv4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (FORM == 0) {
        for (; i + 3 * stride < n; i += 4 * stride) {
            const pnv4 a = src[i], b = src[i + stride], c = src[i + 2 * stride],
                       d = src[i + 3 * stride];
            dst[i] = a;
            dst[i + stride] = b;
            dst[i + 2 * stride] = c;
            dst[i + 3 * stride] = d;
        }
        for (; i < n; i += stride) dst[i] = src[i];
    } else {
        for (; i < n; i += stride)
            __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    }
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
    hipEvent_t e0, e1;
    PN_HIP(hipEventCreate(&e0));
    PN_HIP(hipEventCreate(&e1));
    pn_status status = PN_OK;
    double best = 0.0;
    for (int form = 0; form < 2 && status == PN_OK; ++form) {
        void (*k)(const pnv4*, pnv4*, int64_t) =
            form == 0 ? copy_probe_kernel<0> : copy_probe_kernel<1>;
        for (int per_cu : {1, 2, 3, 4, 6, 8}) {
            const int grid = (int)std::max<int64_t>(
                1, std::min<int64_t>((int64_t)per_cu * cu_count(), (n + 255) / 256));
            // one untimed launch first (first touch, clocks)
            hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, (const pnv4*)src, (pnv4*)dst, n);
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps; ++r)
                hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, st, (const pnv4*)src,
                                   (pnv4*)dst, n);
            (void)hipEventRecord(e1, st);
            float ms = 0.f;
            if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) {
                set_error("pn_copy_probe: timing failed");
                status = PN_ERR_HIP;
                break;
            }
            best = std::max(best, 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9);
        }
    }
    if (status == PN_OK) *gbs = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}
