// Sequential GPU baseline: the rollout s_t = f(s_{t-1}, x_t) one step after another (Ch. 2,
// Problem Statement "Unrolling an SSM"), one workgroup per sequence.
//
// As in library RNN layers, the input projections W x_t + b of every step are computed first
// by a parallel kernel; the recurrence then only evaluates the h-dependent part, in one wave
// per sequence with no workgroup barrier on the step chain.
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

// One wave per sequence, lane j owns unit j: the rows j of U_z, U_r and U_n live in the lane's
// registers, the state is exchanged through LDS (a single wave's LDS operations complete in
// order, so no barrier is needed), and the input projections of the next PF steps are
// prefetched into registers while the current step computes.  Per step a lane issues 3 D
// FMAs (three independent dot-product chains) and one LDS write; nothing else waits.
template <int D>
__global__ void __launch_bounds__(64) gru_seq_kernel(const float* __restrict__ P,
                                                     const float* __restrict__ s0,
                                                     const float* __restrict__ U,
                                                     const float* __restrict__ bhn,
                                                     float* __restrict__ s,
                                                     const int64_t* __restrict__ offsets) {
    static_assert(D % 4 == 0 && D <= 64, "one lane per unit");
    constexpr int PF = 4;                    // prefetch depth (steps)
    __shared__ __attribute__((aligned(16))) float hbuf[2][D];
    const int b = blockIdx.x;
    const int j = threadIdx.x;
    const bool act = j < D;
    const int jj = act ? j : 0;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    if (T == 0) return;                      // nothing to walk (and no row to prefetch)
    float wz[D], wr[D], wq[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        wz[k] = U[(size_t)jj * D + k];
        wr[k] = U[(size_t)(D + jj) * D + k];
        wq[k] = U[(size_t)(2 * D + jj) * D + k];
    }
    const float b_hn = bhn[jj];
    float h = act ? s0[(size_t)b * D + j] : 0.f;
    if (act) hbuf[0][j] = h;
    float pz[PF], pr[PF], pn[PF];
    // Step t: the gates from the state in hbuf[t & 1] and the projections (cz, cr, cn); the
    // new state goes to hbuf[(t + 1) & 1] and to s.  Same gate arithmetic as the parallel
    // solver's GRU kernels (exponential and hardware reciprocal).
    auto step = [&](int64_t t, float cz, float cr, float cn) {
        const float* hc = hbuf[t & 1];
        float az0 = 0.f, ar0 = 0.f, aq0 = 0.f, az1 = 0.f, ar1 = 0.f, aq1 = 0.f;
#pragma unroll
        for (int k = 0; k < D; k += 4) {
            const float4 h4 = *(const float4*)(hc + k);
            az0 = fmaf(wz[k], h4.x, az0);
            ar0 = fmaf(wr[k], h4.x, ar0);
            aq0 = fmaf(wq[k], h4.x, aq0);
            az1 = fmaf(wz[k + 1], h4.y, az1);
            ar1 = fmaf(wr[k + 1], h4.y, ar1);
            aq1 = fmaf(wq[k + 1], h4.y, aq1);
            az0 = fmaf(wz[k + 2], h4.z, az0);
            ar0 = fmaf(wr[k + 2], h4.z, ar0);
            aq0 = fmaf(wq[k + 2], h4.z, aq0);
            az1 = fmaf(wz[k + 3], h4.w, az1);
            ar1 = fmaf(wr[k + 3], h4.w, ar1);
            aq1 = fmaf(wq[k + 3], h4.w, aq1);
        }
        const float z = sigmoid_rcp(az0 + az1 + cz);
        const float r = sigmoid_rcp(ar0 + ar1 + cr);
        const float q = aq0 + aq1 + b_hn;
        const float n = tanh_rcp(cn + r * q);
        h = (1.f - z) * n + z * h;
        if (act) {
            hbuf[(t + 1) & 1][j] = h;
            s[(size_t)(r0 + t) * D + j] = h;
        }
        __builtin_amdgcn_wave_barrier();
    };
    const int64_t Tm = T - T % PF;           // steps covered by whole prefetch rounds
#pragma unroll
    for (int i = 0; i < PF; ++i) {
        const float* row = P + (size_t)(r0 + (i < Tm ? i : 0)) * 3 * D;
        pz[i] = row[jj];
        pr[i] = row[D + jj];
        pn[i] = row[2 * D + jj];
    }
    __builtin_amdgcn_wave_barrier();
    for (int64_t t0 = 0; t0 < Tm; t0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const float cz = pz[i], cr = pr[i], cn = pn[i];
            // the slot is free again: fetch step t + PF (clamped to a valid row at the end)
            const int64_t tn = t0 + i + PF < Tm ? t0 + i + PF : t0 + i;
            const float* row = P + (size_t)(r0 + tn) * 3 * D;
            pz[i] = row[jj];
            pr[i] = row[D + jj];
            pn[i] = row[2 * D + jj];
            step(t0 + i, cz, cr, cn);
        }
    }
    for (int64_t t = Tm; t < T; ++t) {
        const float* row = P + (size_t)(r0 + t) * 3 * D;
        step(t, row[jj], row[D + jj], row[2 * D + jj]);
    }
}

// tanh-RNN (MF = false): s_t = tanh(W s_{t-1} + P_t); mean-field RNN (MF = true):
// s_t = W tanh(s_{t-1}) + P_t, with tanh(s) kept in LDS as the next step's operand.  One wave
// per sequence, lane j owns unit j (row j of W in registers), the state exchanged through LDS
// without barriers, the projections P of the next PF steps prefetched into registers.
template <int D, bool MF>
__global__ void __launch_bounds__(64) tanh_seq_kernel(const float* __restrict__ P,
                                                      const float* __restrict__ s0,
                                                      const float* __restrict__ W,
                                                      float* __restrict__ s,
                                                      const int64_t* __restrict__ offsets) {
    static_assert(D % 4 == 0 && D <= 64, "one lane per unit");
    constexpr int PF = 4;
    __shared__ __attribute__((aligned(16))) float hbuf[2][D];
    const int b = blockIdx.x;
    const int j = threadIdx.x;
    const bool act = j < D;
    const int jj = act ? j : 0;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    if (T == 0) return;                      // nothing to walk (and no row to prefetch)
    float w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = W[(size_t)jj * D + k];
    if (act) hbuf[0][j] = MF ? tanhf_(s0[(size_t)b * D + j]) : s0[(size_t)b * D + j];
    auto step = [&](int64_t t, float pt) {
        const float* hc = hbuf[t & 1];
        float a0 = pt, a1 = 0.f;
#pragma unroll
        for (int k = 0; k < D; k += 4) {
            const float4 h4 = *(const float4*)(hc + k);
            a0 = fmaf(w[k], h4.x, a0);
            a1 = fmaf(w[k + 1], h4.y, a1);
            a0 = fmaf(w[k + 2], h4.z, a0);
            a1 = fmaf(w[k + 3], h4.w, a1);
        }
        const float acc = a0 + a1;
        const float sn = MF ? acc : tanhf_(acc);
        if (act) {
            hbuf[(t + 1) & 1][j] = MF ? tanhf_(acc) : sn;
            s[(size_t)(r0 + t) * D + j] = sn;
        }
        __builtin_amdgcn_wave_barrier();
    };
    const int64_t Tm = T - T % PF;
    float pf[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i) pf[i] = P[(size_t)(r0 + (i < Tm ? i : 0)) * D + jj];
    __builtin_amdgcn_wave_barrier();
    for (int64_t t0 = 0; t0 < Tm; t0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const float pt = pf[i];
            const int64_t tn = t0 + i + PF < Tm ? t0 + i + PF : t0 + i;
            pf[i] = P[(size_t)(r0 + tn) * D + jj];
            step(t0 + i, pt);
        }
    }
    for (int64_t t = Tm; t < T; ++t) step(t, P[(size_t)(r0 + t) * D + jj]);
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
    k.nt = 64;
    return k;
}
template <int D, int DX, bool MF = false>
static SeqKern seq_tanh_get() {
    SeqKern k{};
    k.xproj = xproj_kernel<D, DX>;
    k.O = D;
    k.tanh = tanh_seq_kernel<D, MF>;
    k.nt = 64;
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
    return seq_lookup(cell, D, Dx, &k) || (cell == PN_CELL_MEANFIELD && mf_dense_supported(D, Dx));
}

size_t gru_adjoint_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);

size_t seq_workspace(int cell, int D, int Dx, const HostBatch& hb) {
    SeqKern k;
    if (cell == PN_CELL_MEANFIELD && !seq_lookup(cell, D, Dx, &k)) return mf_seq_workspace(D, hb);
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
    if (!seq_lookup(cd.cell, cd.D, cd.Dx, &k)) {
        if (cd.cell == PN_CELL_MEANFIELD && mf_dense_supported(cd.D, cd.Dx))
            return mf_seq_run(cd, hb, x, s0, s, ws, stream);
        return PN_ERR_UNSUPPORTED;
    }
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
