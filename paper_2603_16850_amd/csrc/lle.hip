// Largest Lyapunov exponent along a trajectory (Alg. LLE_estimate, Ch. 5): a unit vector is
// pushed through the Jacobians A_t = df/ds_{t-1} of the trajectory, renormalised each step,
// and the log stretch factors are averaged.  One wave per sequence, D = Dx = 16: lane
// (r, q) = (l & 15, l >> 4) holds row r of W (and U) at columns 4q .. 4q+3; every lane holds
// u[r] of its row, matrix-vector products meet by shuffles.  The trajectory is read four rows
// per load, one load ahead.
#include <algorithm>
#include <cstring>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

namespace {
constexpr int LD = 16;

// sum over the four column quarters of a row (lanes r, r + 16, r + 32, r + 48)
PN_DEV float rowsum(float v) { return sum_halves(sum_rows16(v)); }
// (M v)[r] for M's row slice m (columns 4q..4q+3) and v held as lane r's value
PN_DEV float matvec(float4 m, float v, int q) {
    return rowsum(m.x * __shfl(v, 4 * q) + m.y * __shfl(v, 4 * q + 1) +
                  m.z * __shfl(v, 4 * q + 2) + m.w * __shfl(v, 4 * q + 3));
}
}  // namespace

template <bool MF>
__global__ void __launch_bounds__(64) lle_kernel(const float* __restrict__ x,
                                                 const float* __restrict__ s0,
                                                 const float* __restrict__ s,
                                                 const float* __restrict__ u0,
                                                 const float* __restrict__ params,
                                                 const int64_t* offsets, int B, double* out) {
    const int b = blockIdx.x;
    if (b >= B) return;
    const int l = threadIdx.x, r = l & 15, q = l >> 4;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    const float* W = params;
    const float* U = W + LD * LD;
    const float4 wr = *(const float4*)(W + r * LD + 4 * q);
    const float4 ur = *(const float4*)(U + r * LD + 4 * q);
    const float br = (U + LD * LD)[r];
    float u = u0[(size_t)b * LD + r];
    {
        float n2 = u * u;
        for (int off = 1; off < 16; off <<= 1) n2 += __shfl_xor(n2, off);
        u = u / sqrtf(n2);
    }
    double total = 0.0;
    // rows r0-1 .. r0+T-1 of the trajectory (row r0-1 is s_0): chunk j holds rows
    // r0-1+4j .. r0+2+4j, lane (r, q) the entry r of the chunk's row q; x likewise from row r0
    auto srow = [&](int64_t i) -> float {        // entry r of s_{i} (i = -1: s_0), i < T
        return i < 0 ? s0[(size_t)b * LD + r] : s[(size_t)(r0 + i) * LD + r];
    };
    auto load_chunk = [&](int64_t j, float& sv, float& xv) {
        const int64_t i = 4 * j + q - 1;          // step index of the previous state
        sv = (i < T) ? srow(i) : 0.f;
        xv = (i + 1 < T) ? x[(size_t)(r0 + i + 1) * LD + r] : 0.f;
    };
    float sc = 0.f, xc = 0.f, sn = 0.f, xn = 0.f;
    if (T > 0) load_chunk(0, sn, xn);
    for (int64_t t = 0; t < T; ++t) {
        const int j = (int)(t & 3);
        if (j == 0) {
            sc = sn;
            xc = xn;
            if (t + 4 < T) load_chunk((t >> 2) + 1, sn, xn);
        }
        const float prev = __shfl(sc, r + 16 * j);      // s_{t-1}[r]
        float v;
        if (MF) {
            const float th = tanhf_(prev);
            v = matvec(wr, (1.f - th * th) * u, q);      // W diag(1 - tanh^2) u
        } else {
            const float xv = __shfl(xc, r + 16 * j);
            const float f = tanhf_(matvec(wr, prev, q) + matvec(ur, xv, q) + br);
            v = (1.f - f * f) * matvec(wr, u, q);        // diag(1 - f^2) W u
        }
        float n2 = v * v;
        for (int off = 1; off < 16; off <<= 1) n2 += __shfl_xor(n2, off);
        const float nrm = sqrtf(n2);
        total += (double)logf(nrm);
        u = v / nrm;
    }
    if (l == 0) out[b] = T > 0 ? total / (double)T : 0.0;
}

bool lle_supported(int cell, int D, int Dx) {
    return ((cell == PN_CELL_TANH || cell == PN_CELL_MEANFIELD) && D == LD && Dx == LD) ||
           (cell == PN_CELL_MEANFIELD && mf_dense_supported(D, Dx));
}

size_t lle_workspace(const HostBatch& hb) {
    Carver c(nullptr);
    c.take<int64_t>(hb.B + 1);
    c.take<double>(std::max(hb.B, 1));
    return c.bytes();
}

pn_status lle_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x, const float* s0,
                  const float* s, const float* u0, void* ws, hipStream_t stream, double* lle) {
    if (hb.B == 0) return PN_OK;
    if (cd.D != LD) return mf_lle_run(cd, hb, s0, s, u0, ws, stream, lle);
    Carver c(ws);
    int64_t* doff = c.take<int64_t>(hb.B + 1);
    double* out = c.take<double>(std::max(hb.B, 1));
    PN_HIP(hipMemcpyAsync(doff, hb.offsets.data(), sizeof(int64_t) * (hb.B + 1),
                          hipMemcpyHostToDevice, stream));
    if (cd.cell == PN_CELL_MEANFIELD)
        hipLaunchKernelGGL(lle_kernel<true>, dim3(hb.B), dim3(64), 0, stream, x, s0, s, u0,
                           (const float*)cd.params, (const int64_t*)doff, hb.B, out);
    else
        hipLaunchKernelGGL(lle_kernel<false>, dim3(hb.B), dim3(64), 0, stream, x, s0, s, u0,
                           (const float*)cd.params, (const int64_t*)doff, hb.B, out);
    PN_HIP(hipGetLastError());
    PN_HIP(hipMemcpyAsync(lle, out, sizeof(double) * hb.B, hipMemcpyDeviceToHost, stream));
    PN_HIP(hipStreamSynchronize(stream));
    return PN_OK;
}

}  // namespace pn
