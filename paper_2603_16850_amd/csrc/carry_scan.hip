// Carry scan over group aggregates and the apply pass (see carry.hpp).
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

// One workgroup of 256 threads per tile, each thread a few float4s of the tile's rows.
template <int D, int L>
__global__ void __launch_bounds__(256) apply_kernel(float* buf0, float* buf1,
                                                    const float2* __restrict__ lac,
                                                    const float* __restrict__ carry,
                                                    const Ctrl* ctrl, SeqState* seq,
                                                    const TileInfo* tiles, int ntiles) {
    constexpr int Q = D / 4;
    constexpr int NI = (L * Q + 255) / 256;
    __shared__ int rowbad[L];
    if (ld_i32(&ctrl->all_done)) return;
    const int par = ctrl->iter & 1;
    const float* __restrict__ in = par ? buf1 : buf0;
    float* __restrict__ out = par ? buf0 : buf1;
    const float reset_abs = ctrl->reset_abs;
    const int tid = threadIdx.x;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const TileInfo ti = tiles[t];
        if (seq[ti.b].status != kActive) continue;       // same on every thread
        for (int r = tid; r < L; r += 256) rowbad[r] = 0;
        __syncthreads();
        float4 v[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int idx = tid + 256 * i;
            const int r = idx / Q, c4 = idx % Q;
            v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (idx < L * Q && r < ti.len) {
                const size_t e = (size_t)(ti.row0 + r) * D + 4 * c4;
                const float4 s4 = *(const float4*)(in + e);
                const float4 p0 = *(const float4*)(lac + e);        // (la, lc) of units 0, 1
                const float4 p1 = *(const float4*)(lac + e + 2);    // units 2, 3
                const float4 cv = *(const float4*)(carry + (size_t)ti.gslot * D + 4 * c4);
                v[i] = make_float4(s4.x + (p0.x * cv.x + p0.y), s4.y + (p0.z * cv.y + p0.w),
                                   s4.z + (p1.x * cv.z + p1.y), s4.w + (p1.z * cv.w + p1.w));
                const bool bad = !(fabsf(v[i].x) <= reset_abs) || !(fabsf(v[i].y) <= reset_abs) ||
                                 !(fabsf(v[i].z) <= reset_abs) || !(fabsf(v[i].w) <= reset_abs);
                if (bad) rowbad[r] = 1;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int idx = tid + 256 * i;
            const int r = idx / Q, c4 = idx % Q;
            if (idx < L * Q && r < ti.len) {
                const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                *(float4*)(out + (size_t)(ti.row0 + r) * D + 4 * c4) = rowbad[r] ? z : v[i];
            }
        }
        if (tid < 64) {
            int nb = 0;
            for (int base = 0; base < L; base += 64) {
                const int r = base + tid;
                nb += __popcll(__ballot(r < ti.len && rowbad[r]));
            }
            if (tid == 0 && nb) atomicAdd(&seq[ti.b].resets_pending, nb);
        }
        __syncthreads();
    }
}

typedef void (*ApplyKernel)(float*, float*, const float2*, const float*, const Ctrl*,
                            SeqState*, const TileInfo*, int);

static ApplyKernel apply_lookup(int D, int L) {
#define PN_AP(d, ll) if (D == d && L == ll) return apply_kernel<d, ll>;
#define PN_APL(d) PN_AP(d, 32) PN_AP(d, 64) PN_AP(d, 128)
    PN_APL(16) PN_APL(32) PN_APL(48) PN_APL(64)
#undef PN_APL
#undef PN_AP
    return nullptr;
}

void launch_apply(float* buf0, float* buf1, const float2* lac, const float* carry,
                  const IterState& st, int ntiles, int D, int L, hipStream_t stream) {
    ApplyKernel k = apply_lookup(D, L);
    if (!k || ntiles <= 0) return;
    const int grid = std::min(ntiles, cu_count() * 8);
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), 0, stream, buf0, buf1, lac, carry,
                       (const Ctrl*)st.ctrl, st.seq, (const TileInfo*)st.tiles, ntiles);
}

}  // namespace pn
