// Carry scan over the group maps (see carry.hpp).
#include <algorithm>

#include "carry.hpp"

namespace pn {

// One wave per (sequence, 4 units).  Lane h = lane % 16 of unit slot q = lane / 16 owns a
// chunk of consecutive groups: it composes them (phase 1), the 16 chunk maps are scanned
// across lanes (phase 2), and the chunk is walked again from its carry-in to write every
// group's carry (phase 3).  Loads are issued eight at a time, so a sequence of G groups costs
// about 2 G / 128 memory round trips per lane.
__global__ void __launch_bounds__(64) carry_scan_kernel(const float2* __restrict__ agg,
                                                        float* __restrict__ carry,
                                                        const Ctrl* ctrl, const SeqState* seq,
                                                        const int32_t* group_start, int B,
                                                        int D) {
    if (ld_i32(&ctrl->all_done)) return;
    const int nblk = (D + 3) / 4;
    const int b = blockIdx.x / nblk;
    const int lane = threadIdx.x, q = lane >> 4, h = lane & 15;
    const int j = (blockIdx.x % nblk) * 4 + q;
    if (b >= B || seq[b].status != kActive) return;
    const bool unit_ok = j < D;
    const int g0 = group_start[b], G = group_start[b + 1] - g0;
    const int ch = (G + 15) / 16;
    const int c0 = g0 + min(G, h * ch), c1 = g0 + min(G, (h + 1) * ch);
    constexpr int K = 8;

    // phase 1: chunk map (A, C): Delta after the chunk = A * Delta before it + C
    float A = 1.f, C = 0.f;
    if (unit_ok) {
        for (int g = c0; g < c1; g += K) {
            float2 v[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] = (g + k < c1) ? agg[(size_t)(g + k) * D + j] : make_float2(1.f, 0.f);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                C = v[k].x * C + v[k].y;
                A = v[k].x * A;
            }
        }
    }
    // phase 2: inclusive scan of the chunk maps over h (16-lane segments), then the
    // exclusive value: the carry entering chunk h (the sequence starts from Delta = 0)
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
        const float pa = __shfl_up(A, off), pc = __shfl_up(C, off);
        if (h >= off) { C = A * pc + C; A = A * pa; }
    }
    float cin = __shfl_up(C, 1);
    if (h == 0) cin = 0.f;
    // phase 3: every group's carry-in
    if (unit_ok) {
        float cv = cin;
        for (int g = c0; g < c1; g += K) {
            float2 v[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] = (g + k < c1) ? agg[(size_t)(g + k) * D + j] : make_float2(1.f, 0.f);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (g + k < c1) {
                    carry[(size_t)(g + k) * D + j] = cv;
                    cv = v[k].x * cv + v[k].y;
                }
        }
    }
}

void launch_carry_scan(const float2* agg, float* carry, const IterState& st, int B, int D,
                       hipStream_t stream) {
    const int nblk = (D + 3) / 4;
    hipLaunchKernelGGL(carry_scan_kernel, dim3((unsigned)(B * nblk)), dim3(64), 0, stream, agg,
                       carry, (const Ctrl*)st.ctrl, (const SeqState*)st.seq,
                       (const int32_t*)st.group_start, B, D);
}

}  // namespace pn
