// Carry scan over the group maps (see carry.hpp).
#include <algorithm>

#include "carry.hpp"

namespace pn {

// One wave per (sequence, 4 units).  Lane h = lane % 16 of unit slot q = lane / 16 owns a
// chunk of consecutive groups: it composes them (phase 1), the 16 chunk maps are scanned
// across lanes (phase 2), and the chunk is walked again from its carry-in to write every
// group's carry (phase 3).  Loads are issued eight at a time, so a sequence of G groups costs
// about 2 G / 128 memory round trips per lane.
//
// Converged-prefix skipping (grmax non-null): the sequence's leading groups whose residual
// max (the maximum of the grmax entries of their waves) is below tol are frozen, from the
// first group on; every wave of the sequence finds the same count, the first writes it to the
// sequence state.  The maps of frozen groups are replaced by (0, 0), so the carry into the
// first open group is 0: the scan restarts there as at a sequence head.
__global__ void __launch_bounds__(64) carry_scan_kernel(const float2* __restrict__ agg,
                                                        float* __restrict__ carry,
                                                        const Ctrl* ctrl, SeqState* seq,
                                                        const int32_t* group_start, int B,
                                                        int D, const uint32_t* grmax, int nw) {
    if (ld_i32(&ctrl->all_done)) return;
    const int nblk = (D + 3) / 4;
    const int b = blockIdx.x / nblk;
    const int lane = threadIdx.x, q = lane >> 4, h = lane & 15;
    const int j = (blockIdx.x % nblk) * 4 + q;
    if (b >= B || seq[b].status != kActive) return;
    const bool unit_ok = j < D;
    const int g0 = group_start[b], G = group_start[b + 1] - g0;
    int nf = 0;               // frozen leading groups
    if (grmax) {
        const float tol = ctrl->tol;
        for (int base = 0; base < G; base += 64) {
            const int gg = base + lane;
            bool open = false;
            if (gg < G) {
                uint32_t m = 0;
                for (int w = 0; w < nw; ++w) m = max(m, grmax[(size_t)(g0 + gg) * nw + w]);
                open = !(__uint_as_float(m) < tol);
            }
            const uint64_t bad = __ballot(open);
            if (bad) {
                nf = base + __ffsll((unsigned long long)bad) - 1;
                break;
            }
            nf = min(G, base + 64);
        }
        if (blockIdx.x % nblk == 0 && lane == 0) {
            seq[b].frozen_prev = seq[b].frozen;
            seq[b].frozen = nf;
        }
    }
    const int gopen = g0 + nf;        // groups before it contribute the map (0, 0)
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
                v[k] = (g + k < c1) ? (g + k < gopen ? make_float2(0.f, 0.f)
                                                     : agg[(size_t)(g + k) * D + j])
                                    : make_float2(1.f, 0.f);
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
                v[k] = (g + k < c1) ? (g + k < gopen ? make_float2(0.f, 0.f)
                                                     : agg[(size_t)(g + k) * D + j])
                                    : make_float2(1.f, 0.f);
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
                       hipStream_t stream, const uint32_t* grmax, int nw) {
    const int nblk = (D + 3) / 4;
    hipLaunchKernelGGL(carry_scan_kernel, dim3((unsigned)(B * nblk)), dim3(64), 0, stream, agg,
                       carry, (const Ctrl*)st.ctrl, st.seq, (const int32_t*)st.group_start, B,
                       D, grmax, nw);
}

}  // namespace pn
