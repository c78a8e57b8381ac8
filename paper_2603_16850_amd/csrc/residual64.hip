// FP64 residual of an FP32 trajectory: max_t |s_t - f(s_{t-1}, x_t)| per sequence with the
// state, input and parameters upcast to FP64 (eq. r_def evaluated in double precision).  It
// confirms the FP32 stopping test of a solve and gives the residual that is reported.
#include <algorithm>
#include <cstring>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

// One thread per step; the parameters are read through the cache.
template <int CELL>
__global__ void residual64_kernel(const float* x, const float* s0, const float* s,
                                  const float* params, const int64_t* offsets, int B, int D,
                                  int Dx, unsigned long long* out) {
    const int64_t N = offsets[B];
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = B;           // sequence of row n: last b with offsets[b] <= n
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offsets[mid] <= n) lo = mid; else hi = mid;
        }
        while (lo + 1 < B && offsets[lo + 1] <= n) ++lo;   // skip empty sequences
        const int b = lo;
        const float* h = (n == offsets[b]) ? s0 + (size_t)b * D : s + (size_t)(n - 1) * D;
        const float* xv = x + (size_t)n * Dx;
        double rmax = 0.0;
        for (int j = 0; j < D; ++j) {
            double f;
            if (CELL == PN_CELL_TANH || CELL == PN_CELL_MEANFIELD) {
                const float* W = params;
                const float* U = W + D * D;
                const float* bb = U + D * Dx;
                double acc = bb[j];
                for (int k = 0; k < D; ++k)
                    acc += (double)W[j * D + k] *
                           (CELL == PN_CELL_TANH ? (double)h[k] : tanh((double)h[k]));
                for (int k = 0; k < Dx; ++k) acc += (double)U[j * Dx + k] * (double)xv[k];
                f = CELL == PN_CELL_TANH ? tanh(acc) : acc;
            } else {
                const float* W = params;
                const float* U = W + 3 * D * Dx;
                const float* bb = U + 3 * D * D;
                double az = bb[j], ar = bb[D + j], an = bb[2 * D + j], aq = bb[3 * D + j];
                for (int k = 0; k < Dx; ++k) {
                    az += (double)W[j * Dx + k] * xv[k];
                    ar += (double)W[(D + j) * Dx + k] * xv[k];
                    an += (double)W[(2 * D + j) * Dx + k] * xv[k];
                }
                for (int k = 0; k < D; ++k) {
                    az += (double)U[j * D + k] * h[k];
                    ar += (double)U[(D + j) * D + k] * h[k];
                    aq += (double)U[(2 * D + j) * D + k] * h[k];
                }
                const double z = 1.0 / (1.0 + exp(-az)), r = 1.0 / (1.0 + exp(-ar));
                const double nn = tanh(an + r * aq);
                f = (1.0 - z) * nn + z * (double)h[j];
            }
            const double res = (double)s[(size_t)n * D + j] - f;
            rmax = fmax(rmax, (res == res) ? fabs(res) : INFINITY);
        }
        atomicMax(&out[b], (unsigned long long)__double_as_longlong(rmax));
    }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

bool residual64_supported(int cell, int D, int Dx) {
    return (cell == PN_CELL_TANH || cell == PN_CELL_GRU || cell == PN_CELL_MEANFIELD) && D >= 1 &&
           D <= 256 && Dx >= 1 &&
           Dx <= 256;
}

size_t residual64_workspace(int, int, int, const HostBatch& hb) {
    Carver c(nullptr);
    c.take<int64_t>(hb.B + 1);
    c.take<unsigned long long>(hb.B);
    return c.bytes();
}

pn_status residual64_device(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                            const float* s0, const float* s, void* ws, hipStream_t stream,
                            double* max_resid) {
    Carver c(ws);
    int64_t* doff = c.take<int64_t>(hb.B + 1);
    unsigned long long* out = c.take<unsigned long long>(hb.B);
    PN_HIP(hipMemcpyAsync(doff, hb.offsets.data(), sizeof(int64_t) * (hb.B + 1),
                          hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, stream, out, hb.B);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4 * cu_count(), (hb.N + 255) / 256));
    if (hb.N > 0) {
        if (cd.cell == PN_CELL_TANH)
            hipLaunchKernelGGL(residual64_kernel<PN_CELL_TANH>, dim3(grid), dim3(256), 0, stream, x,
                               s0, s, (const float*)cd.params, (const int64_t*)doff, hb.B, cd.D,
                               cd.Dx, out);
        else if (cd.cell == PN_CELL_MEANFIELD)
            hipLaunchKernelGGL(residual64_kernel<PN_CELL_MEANFIELD>, dim3(grid), dim3(256), 0,
                               stream, x, s0, s, (const float*)cd.params, (const int64_t*)doff,
                               hb.B, cd.D, cd.Dx, out);
        else
            hipLaunchKernelGGL(residual64_kernel<PN_CELL_GRU>, dim3(grid), dim3(256), 0, stream, x,
                               s0, s, (const float*)cd.params, (const int64_t*)doff, hb.B, cd.D,
                               cd.Dx, out);
    }
    PN_HIP(hipGetLastError());
    std::vector<unsigned long long> h(hb.B);
    PN_HIP(hipMemcpyAsync(h.data(), out, sizeof(unsigned long long) * hb.B,
                          hipMemcpyDeviceToHost, stream));
    PN_HIP(hipStreamSynchronize(stream));
    for (int b = 0; b < hb.B; ++b) {
        double v;
        std::memcpy(&v, &h[b], sizeof(double));
        max_resid[b] = v;
    }
    return PN_OK;
}

pn_status residual64_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                         const float* s0, const float* s, void* ws, hipStream_t stream,
                         double* max_resid) {
    return residual64_device(cd, hb, x, s0, s, ws, stream, max_resid);
}

}  // namespace pn
