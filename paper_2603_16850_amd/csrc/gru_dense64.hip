// DEER with dense Jacobians in FP64 for a small GRU state (D <= 4): the whole Newton loop of
// Alg. alg:deer runs inside one 1024-thread workgroup per sequence, so an iteration costs no
// kernel launch (the workload is launch-latency bound, not bandwidth or compute bound).
//
// Each iteration walks the sequence in chunks of 1024 steps, one step per thread:
//   1. linearise: f_t(s_{t-1}), r_t = s_t - f_t (eq. r_def) and the dense A_t = df_t/ds_{t-1}
//      (eq. lil_j) from the closed-form GRU Jacobian;
//   2. scan the affine maps Delta -> A_t Delta + c_t, c_t = -r_t (eq. lin_rr) with the
//      composition of eq. bin_op_affine: inside a wave by shuffles (Hillis-Steele), across the
//      16 waves through LDS, and across chunks by the carried Delta of the chunk's last step;
//   3. write s^(i+1) = s^(i) + Delta (overflow reset guard) into the other ping-pong buffer.
// The stopping test reads max |r(s^(i))| over the whole sequence before s^(i+1) is used.
#include <algorithm>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

template <int D>
struct Aff {
    double P[D][D];
    double q[D];
};

// later o earlier: Delta -> L.P (E.P Delta + E.q) + L.q
template <int D>
PN_DEV Aff<D> compose(const Aff<D>& E, const Aff<D>& Lm) {
    Aff<D> o;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double acc = Lm.q[i];
#pragma unroll
        for (int k = 0; k < D; ++k) acc += Lm.P[i][k] * E.q[k];
        o.q[i] = acc;
#pragma unroll
        for (int jj = 0; jj < D; ++jj) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) a += Lm.P[i][k] * E.P[k][jj];
            o.P[i][jj] = a;
        }
    }
    return o;
}

template <int D>
PN_DEV Aff<D> shfl_up_aff(const Aff<D>& a, int delta) {
    Aff<D> o;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        o.q[i] = __shfl_up(a.q[i], delta);
#pragma unroll
        for (int jj = 0; jj < D; ++jj) o.P[i][jj] = __shfl_up(a.P[i][jj], delta);
    }
    return o;
}

template <int D>
PN_DEV Aff<D> identity_aff() {
    Aff<D> o;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        o.q[i] = 0.0;
#pragma unroll
        for (int jj = 0; jj < D; ++jj) o.P[i][jj] = (i == jj) ? 1.0 : 0.0;
    }
    return o;
}

struct Dense64Args {
    const double* x;
    const double* s0;
    double* sbuf[2];
    const double* params;
    const int64_t* offsets;
    SeqState* seq;
    int Dx;
    int max_iters;
    double tol;
    double reset_abs;
};

template <int D>
__global__ void __launch_bounds__(1024) gru_dense64_kernel(Dense64Args a) {
    constexpr int NT = 1024, NWV = NT / 64;
    constexpr int MAXDX = 16;
    __shared__ double Wz[D][MAXDX], Wr[D][MAXDX], Wn[D][MAXDX];
    __shared__ double Uz[D][D], Ur[D][D], Un[D][D];
    __shared__ double bz[D], br[D], bn[D], bhn[D];
    __shared__ Aff<D> wave_tot[NWV];
    __shared__ double carry[D];
    __shared__ double red[NWV];
    __shared__ int rowbad_any[NWV];
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int Dx = a.Dx;
    const double* W = a.params;
    const double* U = W + 3 * D * Dx;
    const double* bias = U + 3 * D * D;
    for (int idx = tid; idx < D * Dx; idx += NT) {
        const int i = idx / Dx, k = idx % Dx;
        Wz[i][k] = W[(0 * D + i) * Dx + k];
        Wr[i][k] = W[(1 * D + i) * Dx + k];
        Wn[i][k] = W[(2 * D + i) * Dx + k];
    }
    for (int idx = tid; idx < D * D; idx += NT) {
        const int i = idx / D, k = idx % D;
        Uz[i][k] = U[(0 * D + i) * D + k];
        Ur[i][k] = U[(1 * D + i) * D + k];
        Un[i][k] = U[(2 * D + i) * D + k];
    }
    if (tid < D) {
        bz[tid] = bias[tid];
        br[tid] = bias[D + tid];
        bn[tid] = bias[2 * D + tid];
        bhn[tid] = bias[3 * D + tid];
    }
    __syncthreads();
    const int64_t r0 = a.offsets[b], T = a.offsets[b + 1] - r0;
    int final_par = 0, iters = 0, resets = 0, conv = 0;
    double final_r = 0.0;
    for (int it = 0;; ++it) {
        const int cur = it & 1;
        const double* sin = a.sbuf[cur] + r0 * D;
        double* sout = a.sbuf[cur ^ 1] + r0 * D;
        if (tid < D) carry[tid] = 0.0;
        double rmax = 0.0;
        int nreset = 0;
        __syncthreads();
        for (int64_t c0 = 0; c0 < T; c0 += NT) {
            const int64_t t = c0 + tid;
            const bool valid = t < T;
            // ---- linearise step t
            Aff<D> m = identity_aff<D>();
            double scur[D];
            if (valid) {
                double h[D], xv[MAXDX];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    h[i] = (t == 0) ? a.s0[(size_t)b * D + i] : sin[(t - 1) * D + i];
                    scur[i] = sin[t * D + i];
                }
                for (int k = 0; k < Dx; ++k) xv[k] = a.x[(r0 + t) * Dx + k];
                double z[D], r[D], q[D], n[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double az = bz[i], ar = br[i], an = bn[i], aq = bhn[i];
                    for (int k = 0; k < Dx; ++k) {
                        az += Wz[i][k] * xv[k];
                        ar += Wr[i][k] * xv[k];
                        an += Wn[i][k] * xv[k];
                    }
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        az += Uz[i][k] * h[k];
                        ar += Ur[i][k] * h[k];
                        aq += Un[i][k] * h[k];
                    }
                    z[i] = 1.0 / (1.0 + exp(-az));
                    r[i] = 1.0 / (1.0 + exp(-ar));
                    q[i] = aq;
                    n[i] = tanh(an + r[i] * aq);
                }
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const double f = (1.0 - z[i]) * n[i] + z[i] * h[i];
                    const double res = scur[i] - f;
                    rmax = fmax(rmax, (res == res) ? fabs(res) : INFINITY);
                    m.q[i] = -res;
                    const double al = (h[i] - n[i]) * z[i] * (1.0 - z[i]);
                    const double e = (1.0 - z[i]) * (1.0 - n[i] * n[i]);
                    const double be = e * r[i], ga = e * q[i] * r[i] * (1.0 - r[i]);
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        m.P[i][k] = (t == 0) ? 0.0
                                             : ((i == k ? z[i] : 0.0) + al * Uz[i][k] +
                                                be * Un[i][k] + ga * Ur[i][k]);
                }
            }
            // ---- inclusive scan over the chunk: wave, then across waves
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const Aff<D> prev = shfl_up_aff(m, d);
                if (lane >= d) m = compose(prev, m);
            }
            if (lane == 63) wave_tot[wv] = m;
            __syncthreads();
            Aff<D> pre;     // composed maps of earlier waves applied to the carry
            {
                double v[D];
#pragma unroll
                for (int i = 0; i < D; ++i) v[i] = carry[i];
                for (int w2 = 0; w2 < wv; ++w2) {
                    double nv[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        double acc = wave_tot[w2].q[i];
#pragma unroll
                        for (int k = 0; k < D; ++k) acc += wave_tot[w2].P[i][k] * v[k];
                        nv[i] = acc;
                    }
#pragma unroll
                    for (int i = 0; i < D; ++i) v[i] = nv[i];
                }
#pragma unroll
                for (int i = 0; i < D; ++i) pre.q[i] = v[i];
            }
            double dl[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double acc = m.q[i];
#pragma unroll
                for (int k = 0; k < D; ++k) acc += m.P[i][k] * pre.q[k];
                dl[i] = acc;
            }
            __syncthreads();   // everyone has read carry / wave_tot
            const int64_t last = std::min<int64_t>(T, c0 + NT) - 1;
            if (t == last) {
#pragma unroll
                for (int i = 0; i < D; ++i) carry[i] = dl[i];
            }
            if (valid) {
                double sn[D];
                bool bad = false;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    sn[i] = scur[i] + dl[i];
                    bad = bad || !(fabs(sn[i]) <= a.reset_abs);
                }
                if (bad) ++nreset;
#pragma unroll
                for (int i = 0; i < D; ++i) sout[t * D + i] = bad ? 0.0 : sn[i];
            }
            __syncthreads();
        }
        // ---- stopping test on r(s^(it))
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
        int nr = nreset;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nr += __shfl_xor(nr, off);
        if (lane == 0) { red[wv] = rmax; rowbad_any[wv] = nr; }
        __syncthreads();
        double tot = 0.0;
        int rs = 0;
        for (int w2 = 0; w2 < NWV; ++w2) { tot = fmax(tot, red[w2]); rs += rowbad_any[w2]; }
        __syncthreads();
        if (tot < a.tol || it >= a.max_iters) {
            final_par = cur;
            iters = it;
            final_r = tot;
            conv = tot < a.tol;
            break;
        }
        resets += rs;
    }
    if (final_par == 1) {
        for (int64_t i = tid; i < T * D; i += NT) a.sbuf[0][r0 * D + i] = a.sbuf[1][r0 * D + i];
    }
    if (tid == 0) {
        SeqState q;
        q.status = conv ? kConverged : kCapped;
        q.iters = iters;
        q.resets = resets;
        q.resets_pending = 0;
        q.parity = 0;
        q.maxr = 0;
        q.final_resid = (float)final_r;
        q.frozen = 0;
        q.frozen_prev = 0;
        q.maxd = 0;
        a.seq[b] = q;
    }
}

bool gru_dense64_supported(int D, int Dx) { return D >= 1 && D <= 4 && Dx >= 1 && Dx <= 16; }

size_t gru_dense64_workspace(int D, int Dx, const HostBatch& hb, const pn_opts&) {
    Carver c(nullptr);
    c.take<SeqState>(hb.B);
    c.take<int64_t>(hb.B + 1);
    c.take<double>((size_t)hb.N * D);
    c.take<double>(hb.B);
    return c.bytes();
}

pn_status gru_dense64_forward(const pn_cell_desc& cd, const HostBatch& hb, const double* x,
                              const double* s0, double* s, const pn_opts& o, void* ws,
                              hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    const int D = cd.D;
    Carver c(ws);
    SeqState* seq = c.take<SeqState>(hb.B);
    int64_t* doff = c.take<int64_t>(hb.B + 1);
    double* salt = c.take<double>((size_t)hb.N * D);
    double* fres = c.take<double>(hb.B);
    (void)fres;
    PN_HIP(hipMemcpyAsync(doff, hb.offsets.data(), sizeof(int64_t) * (hb.B + 1),
                          hipMemcpyHostToDevice, stream));
    Dense64Args a;
    a.x = x;
    a.s0 = s0;
    a.sbuf[0] = s;
    a.sbuf[1] = salt;
    a.params = (const double*)cd.params;
    a.offsets = doff;
    a.seq = seq;
    a.Dx = cd.Dx;
    a.max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    a.tol = o.tol;
    a.reset_abs = o.reset_abs;
    void (*k)(Dense64Args) = nullptr;
    switch (D) {
        case 1: k = gru_dense64_kernel<1>; break;
        case 2: k = gru_dense64_kernel<2>; break;
        case 3: k = gru_dense64_kernel<3>; break;
        case 4: k = gru_dense64_kernel<4>; break;
        default: return PN_ERR_UNSUPPORTED;
    }
    prof_launch("gru_dense64_solve", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(k, dim3(hb.B), dim3(1024), 0, s2, a);
    });
    PN_HIP(hipGetLastError());
    std::vector<SeqState> hs(hb.B);
    PN_HIP(hipMemcpyAsync(hs.data(), seq, sizeof(SeqState) * hb.B, hipMemcpyDeviceToHost, stream));
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    bool allc = true;
    for (int b = 0; b < hb.B; ++b) {
        const bool cv = hs[b].status == kConverged || hb.len(b) == 0;
        allc = allc && cv;
        if (info) {
            info[b].iters = hs[b].iters;
            info[b].converged = cv;
            info[b].resets = hs[b].resets;
            info[b].pad_ = 0;
            info[b].max_resid = hs[b].final_resid;
        }
    }
    *all_conv = allc;
    return PN_OK;
}

}  // namespace pn
