// Sequential GPU baseline: the rollout s_t = f(s_{t-1}, x_t) one step after another (Ch. 2,
// Problem Statement "Unrolling an SSM"), one workgroup per sequence.
//
// As in library RNN layers, the input projections W x_t + b of every step are computed first
// by a parallel kernel; the recurrence then only evaluates the h-dependent part.  For the GRU,
// four lanes of one wave serve each unit (z, r and U_n h dot products, the fourth idle), meet
// by cross-lane shuffles, and one barrier per step publishes the new state in LDS.
#include <algorithm>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

// P[n][O] = Wcat x_n + bcat, Wcat [O x DX] row-major, one output per thread.
template <int O, int DX>
__global__ void __launch_bounds__(256) xproj_kernel(const float* x, const float* Wcat,
                                                    const float* bcat, float* P, int64_t N) {
    constexpr int R = 32;
    __shared__ float xs[R][DX];
    const int tid = threadIdx.x;
    float w[DX];
    float bias = 0.f;
    if (tid < O) {
#pragma unroll
        for (int k = 0; k < DX; ++k) w[k] = Wcat[tid * DX + k];
        bias = bcat[tid];
    }
    for (int64_t n0 = (int64_t)blockIdx.x * R; n0 < N; n0 += (int64_t)gridDim.x * R) {
        __syncthreads();
        for (int idx = tid; idx < R * DX; idx += blockDim.x) {
            const int r = idx / DX, c = idx % DX;
            xs[r][c] = (n0 + r < N) ? x[(n0 + r) * DX + c] : 0.f;
        }
        __syncthreads();
        if (tid < O) {
            for (int r = 0; r < R && n0 + r < N; ++r) {
                float acc = bias;
#pragma unroll
                for (int k = 0; k < DX; ++k) acc += w[k] * xs[r][k];
                P[(n0 + r) * O + tid] = acc;
            }
        }
    }
}

template <int D>
__global__ void __launch_bounds__(4 * D) gru_seq_kernel(const float* P, const float* s0,
                                                        const float* U, const float* bhn,
                                                        float* s, const int64_t* offsets) {
    constexpr int CH = 32;
    __shared__ __attribute__((aligned(16))) float hbuf[2][D];
    __shared__ float pch[CH][3 * D];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int j = tid >> 2, role = tid & 3, base = (threadIdx.x & 63) & ~3;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    float w[D];
    const int wrow = role == 0 ? j : (role == 1 ? D + j : 2 * D + j);   // U_z, U_r, U_n rows
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = role < 3 ? U[wrow * D + k] : 0.f;
    const float b_hn = bhn[j];
    if (tid < D) hbuf[0][tid] = s0[(size_t)b * D + tid];
    __syncthreads();
    for (int64_t t = 0; t < T; ++t) {
        if (t % CH == 0) {
            for (int idx = tid; idx < CH * 3 * D; idx += blockDim.x) {
                const int r = idx / (3 * D), c = idx % (3 * D);
                pch[r][c] = (t + r < T) ? P[(size_t)(r0 + t + r) * 3 * D + c] : 0.f;
            }
            __syncthreads();
        }
        const int cur = (int)(t & 1);
        const float* h = hbuf[cur];
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < D; k += 4) {
            const float4 h4 = *(const float4*)(h + k);
            acc += w[k] * h4.x + w[k + 1] * h4.y + w[k + 2] * h4.z + w[k + 3] * h4.w;
        }
        const float zp = __shfl(acc, base + 0), rp = __shfl(acc, base + 1),
                    qp = __shfl(acc, base + 2);
        if (role == 0) {
            const float* pr = pch[t % CH];
            const float z = sigmoidf_(zp + pr[j]);
            const float r = sigmoidf_(rp + pr[D + j]);
            const float q = qp + b_hn;
            const float n = tanhf_(pr[2 * D + j] + r * q);
            const float hn = (1.f - z) * n + z * h[j];
            hbuf[cur ^ 1][j] = hn;
            s[(size_t)(r0 + t) * D + j] = hn;
        }
        __syncthreads();
    }
}

// tanh-RNN (MF = false): s_t = tanh(W s_{t-1} + P_t); mean-field RNN (MF = true):
// s_t = W tanh(s_{t-1}) + P_t, with tanh(s) kept in LDS as the next step's operand
template <int D, bool MF>
__global__ void __launch_bounds__(D < 64 ? 64 : D) tanh_seq_kernel(const float* P,
                                                                   const float* s0,
                                                                   const float* W, float* s,
                                                                   const int64_t* offsets) {
    constexpr int CH = 32;
    __shared__ __attribute__((aligned(16))) float hbuf[2][D];
    __shared__ float pch[CH][D];
    const int b = blockIdx.x;
    const int j = threadIdx.x;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    float w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = j < D ? W[j * D + k] : 0.f;
    if (j < D) hbuf[0][j] = MF ? tanhf_(s0[(size_t)b * D + j]) : s0[(size_t)b * D + j];
    __syncthreads();
    for (int64_t t = 0; t < T; ++t) {
        if (t % CH == 0) {
            for (int idx = j; idx < CH * D; idx += blockDim.x) {
                const int r = idx / D, c = idx % D;
                pch[r][c] = (t + r < T) ? P[(size_t)(r0 + t + r) * D + c] : 0.f;
            }
            __syncthreads();
        }
        const int cur = (int)(t & 1);
        if (j < D) {
            const float* h = hbuf[cur];
            float acc = pch[t % CH][j];
#pragma unroll
            for (int k = 0; k < D; k += 4) {
                const float4 h4 = *(const float4*)(h + k);
                acc += w[k] * h4.x + w[k + 1] * h4.y + w[k + 2] * h4.z + w[k + 3] * h4.w;
            }
            if (MF) {
                hbuf[cur ^ 1][j] = tanhf_(acc);
                s[(size_t)(r0 + t) * D + j] = acc;
            } else {
                const float hn = tanhf_(acc);
                hbuf[cur ^ 1][j] = hn;
                s[(size_t)(r0 + t) * D + j] = hn;
            }
        }
        __syncthreads();
    }
}

// ---- host -----------------------------------------------------------------------------------

struct SeqKern {
    void (*xproj)(const float*, const float*, const float*, float*, int64_t);
    int O;
    void (*gru)(const float*, const float*, const float*, const float*, float*, const int64_t*);
    void (*tanh)(const float*, const float*, const float*, float*, const int64_t*);
    int nt;
};

template <int D, int DX>
static SeqKern seq_gru_get() {
    SeqKern k{};
    k.xproj = xproj_kernel<3 * D, DX>;
    k.O = 3 * D;
    k.gru = gru_seq_kernel<D>;
    k.nt = 4 * D;
    return k;
}
template <int D, int DX, bool MF = false>
static SeqKern seq_tanh_get() {
    SeqKern k{};
    k.xproj = xproj_kernel<D, DX>;
    k.O = D;
    k.tanh = tanh_seq_kernel<D, MF>;
    k.nt = D < 64 ? 64 : D;
    return k;
}

static bool seq_lookup(int cell, int D, int Dx, SeqKern* k) {
    if (cell == PN_CELL_GRU) {
#define PN_SG(d, dx) if (D == d && Dx == dx) { *k = seq_gru_get<d, dx>(); return true; }
        PN_SG(64, 32) PN_SG(48, 24) PN_SG(32, 16) PN_SG(16, 8) PN_SG(16, 16) PN_SG(64, 64)
        PN_SG(32, 32) PN_SG(48, 48) PN_SG(64, 16) PN_SG(32, 8)
#undef PN_SG
    } else if (cell == PN_CELL_TANH) {
#define PN_ST(d, dx) if (D == d && Dx == dx) { *k = seq_tanh_get<d, dx>(); return true; }
        PN_ST(16, 16) PN_ST(32, 16) PN_ST(32, 32) PN_ST(64, 32) PN_ST(16, 8) PN_ST(4, 4)
#undef PN_ST
    } else if (cell == PN_CELL_MEANFIELD) {
        if (D == 16 && Dx == 16) { *k = seq_tanh_get<16, 16, true>(); return true; }
    }
    return false;
}

bool seq_supported(int cell, int D, int Dx) {
    SeqKern k;
    return seq_lookup(cell, D, Dx, &k);
}

size_t gru_adjoint_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);

size_t seq_workspace(int cell, int D, int Dx, const HostBatch& hb) {
    Carver c(nullptr);
    c.take<int64_t>(hb.B + 1);
    c.take<float>((size_t)hb.N * (cell == PN_CELL_GRU ? 3 * D : D));
    size_t n = c.bytes();
    pn_opts o;
    pn_default_opts(&o);
    if (cell == PN_CELL_GRU) n = std::max(n, gru_adjoint_workspace(D, Dx, hb, o));
    if (cell == PN_CELL_TANH && tanh_dense_supported(D, Dx))
        n = std::max(n, tanh_adjoint_workspace(D, Dx, hb, o));
    return n;
}

pn_status seq_rollout_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                          const float* s0, float* s, void* ws, hipStream_t stream) {
    SeqKern k;
    if (!seq_lookup(cd.cell, cd.D, cd.Dx, &k)) return PN_ERR_UNSUPPORTED;
    if (hb.N == 0) return PN_OK;
    const int D = cd.D, Dx = cd.Dx;
    Carver c(ws);
    int64_t* doff = c.take<int64_t>(hb.B + 1);
    float* P = c.take<float>((size_t)hb.N * k.O);
    PN_HIP(hipMemcpyAsync(doff, hb.offsets.data(), sizeof(int64_t) * (hb.B + 1),
                          hipMemcpyHostToDevice, stream));
    const float* prm = (const float*)cd.params;
    const int xg = (int)std::min<int64_t>(4 * cu_count(), (hb.N + 31) / 32);
    if (cd.cell == PN_CELL_GRU) {
        // Wcat = [W_z;W_r;W_n] is the head of the packed parameters, bcat = [b_z;b_r;b_n]
        const float* U = prm + 3 * D * Dx;
        hipLaunchKernelGGL(k.xproj, dim3(xg), dim3(256), 0, stream, x, prm, U + 3 * D * D, P,
                           hb.N);
        prof_launch("seq_rollout", stream, [&](hipStream_t s2) {
            hipLaunchKernelGGL(k.gru, dim3(hb.B), dim3(k.nt), 0, s2, (const float*)P, s0, U,
                               U + 3 * D * D + 3 * D, s, (const int64_t*)doff);
        });
    } else {
        const float* W = prm;
        const float* Ux = prm + D * D;
        hipLaunchKernelGGL(k.xproj, dim3(xg), dim3(256), 0, stream, x, Ux, Ux + D * Dx, P, hb.N);
        prof_launch("seq_rollout", stream, [&](hipStream_t s2) {
            hipLaunchKernelGGL(k.tanh, dim3(hb.B), dim3(k.nt), 0, s2, (const float*)P, s0, W, s,
                               (const int64_t*)doff);
        });
    }
    PN_HIP(hipGetLastError());
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    return PN_OK;
}

}  // namespace pn
