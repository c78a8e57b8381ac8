// The mean-field RNN of the predictability experiments (Ch. 5 "Experiments") at state sizes
// up to 128 (the thesis uses D = 100): DEER with dense Jacobians, the sequential rollout and
// the largest-Lyapunov-exponent estimate.
//
//   f(s, x) = W tanh(s) + U x + b,   A_t = df/ds_{t-1} = W diag(d_t),  d_t = 1 - tanh^2(s_{t-1}).
//
// DEER (Alg. alg:deer) in the Delta form of eq. lin_rr: at the iterate s^(k),
//   r_t = s_t - f(s_{t-1}, x_t),   Delta_t = A_t Delta_{t-1} - r_t  (zero before the sequence),
//   s^(k+1) = s^(k) + Delta,
// stopping when max |r| < tol (the residual of the iterate itself).  The linear recurrence is
// solved by the work-efficient two-level scan over groups of consecutive steps:
//   map pass   - per group the product M_q = A_hi ... A_lo (D x D, MFMA: BF16 operands with
//                FP32 accumulation, or FP32) and the chain v_q from Delta = 0 (FP32), with the
//                residual and d_t of every step (kept for the apply pass);
//   walk       - w_0 = 0, w_{q+1} = M_q w_q + v_q: the Delta entering each group;
//   apply pass - the exact FP32 recurrence from w_q inside every group, s^(k+1) written.
// With BF16 maps the carries are those of a slightly different linear system: the step is
// then a quasi-Newton step, and the next iteration's exact FP32 residual corrects it (the
// compose-precision option of the dense scans).  States are padded to 128 on chip (zero rows
// and columns of W beyond D keep the padded coordinates at zero).
#include <algorithm>
#include <cmath>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MP = 128;           // padded state size
constexpr int MNB = MP / 16;      // 16-row blocks
constexpr int MKK = MP / 32;      // K chunks of the BF16 16x16x32 product

struct MfArgs {
    const float* x;
    const float* s0;
    const float* W;               // [D][D]
    const float* U;               // [D][Dx]
    const float* bias;            // [D]
    int D, Dx;
    float* ub;                    // [N][D]  U x_t + b (once per solve)
    float* sbuf[2];               // s^(k) in sbuf[k & 1]; sbuf[0] is the caller's s
    float* rd;                    // [N][2][D]  r_t and d_t of the current linearisation
    float* mbuf;                  // [ngroups][MP][MP]  group maps, row-major
    float* vbuf;                  // [ngroups][MP]
    float* wcar;                  // [ngroups][MP]  Delta entering each group
    Ctrl* ctrl;
    SeqState* seq;
    const TileInfo* tiles;
    const GroupInfo* groups;
    const int32_t* group_start;
    int ngroups;
    int B;
};

// rows [row_lo, row_lo + len) of group slot gi (groups in time order from the sequence start)
PN_DEV void mf_group_rows(const MfArgs& a, int gi, int64_t& row_lo, int& len, int& b,
                          bool& first) {
    const GroupInfo gr = a.groups[gi];
    const TileInfo t0 = a.tiles[gr.tile0], t1 = a.tiles[gr.tile0 + gr.ntl - 1];
    row_lo = t0.row0;
    len = (int)(t1.row0 + t1.len - t0.row0);
    b = gr.b;
    first = (t0.flags & kTileTimeFirst) != 0;
}

// Thread (i, h) = (tid >> 1, tid & 1) of a 256-thread workgroup holds row i of W at columns
// 64h .. 64h + 63 (zero beyond D); (W v)_i is its partial sum plus its pair lane's.
struct MfRow {
    float w[64];
    PN_DEV void load(const float* W, int D, int i, int h) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            const int col = 64 * h + k;
            w[k] = (i < D && col < D) ? W[(size_t)i * D + col] : 0.f;
        }
    }
    // partial sum over this thread's columns of v (LDS, 16-byte aligned, MP entries)
    PN_DEV float dot(const float* v, int h) const {
        float p0 = 0.f, p1 = 0.f;
#pragma unroll
        for (int k = 0; k < 64; k += 4) {
            const float4 q = *(const float4*)(v + 64 * h + k);
            p0 = fmaf(w[k], q.x, p0);
            p1 = fmaf(w[k + 1], q.y, p1);
            p0 = fmaf(w[k + 2], q.z, p0);
            p1 = fmaf(w[k + 3], q.w, p1);
        }
        return p0 + p1;
    }
};
PN_DEV float pair_sum(float p) { return p + __shfl_xor(p, 1); }

__global__ void __launch_bounds__(256) mf_ub_kernel(const float* __restrict__ x,
                                                    const float* __restrict__ U,
                                                    const float* __restrict__ bias,
                                                    float* __restrict__ ub, int64_t N, int D,
                                                    int Dx) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N * D;
         e += (int64_t)gridDim.x * 256) {
        const int64_t t = e / D;
        const int i = (int)(e % D);
        const float* xr = x + t * Dx;
        const float* ur = U + (size_t)i * Dx;
        float acc = bias[i];
        for (int k = 0; k < Dx; ++k) acc = fmaf(ur[k], xr[k], acc);
        ub[e] = acc;
    }
}

// ---- map pass: one workgroup (4 waves) per group ---------------------------------------------
// M is held in the MFMA output layout, wave w owning the column blocks 2w and 2w + 1: lane
// (c, g) = (l & 15, l >> 4) holds M[4g + r + 16 bi][c + 16 cb].  The product's K order is the
// rows a lane holds (slot j of chunk kk <-> row 4g + (j & 3) + 16 (2 kk + (j >> 2)) in BF16,
// slot s <-> row 4g + (s & 3) + 16 (s >> 2) in FP32), so d (.) M is formed from the lane's
// own entries and no transpose is needed between steps; the A operand (W in that column order)
// is staged once per workgroup in LDS.
template <bool BF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1)))
mf_map_kernel(MfArgs a) {
    __shared__ __attribute__((aligned(16))) bf16x8 wb[BF ? MNB * MKK * 64 : 1];
    __shared__ __attribute__((aligned(16))) float wf[BF ? 1 : MP * (MP + 1)];
    __shared__ __attribute__((aligned(16))) float th[MP];
    __shared__ __attribute__((aligned(16))) float dk[MP];
    __shared__ __attribute__((aligned(16))) float vv[MP];
    __shared__ __attribute__((aligned(16))) float dv[MP];
    if (ld_i32(&a.ctrl->all_done)) return;
    const int gi = blockIdx.x;
    if (gi >= a.ngroups) return;                        // (an empty batch launches one)
    int64_t row_lo;
    int len, b;
    bool first;
    mf_group_rows(a, gi, row_lo, len, b, first);
    if (a.seq[b].status != kActive) return;            // same on every thread
    const int k = a.ctrl->iter;
    const float* __restrict__ s = a.sbuf[k & 1];
    const int D = a.D;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
    const int mi = tid >> 1, mh = tid & 1;
    MfRow wr;
    wr.load(a.W, D, mi, mh);
    if constexpr (BF) {
        for (int e = tid; e < MNB * MKK * 64; e += 256) {
            const int el = e & 63, kk = (e >> 6) % MKK, bo = (e >> 6) / MKK;
            const int i = (el & 15) + 16 * bo, eg = el >> 4;
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int kr = 4 * eg + (j & 3) + 16 * (2 * kk + (j >> 2));
                v[j] = (__bf16)((i < D && kr < D) ? a.W[(size_t)i * D + kr] : 0.f);
            }
            wb[e] = v;
        }
    } else {
        for (int e = tid; e < MP * MP; e += 256) {
            const int i = e / MP, kr = e % MP;
            wf[i * (MP + 1) + kr] = (i < D && kr < D) ? a.W[(size_t)i * D + kr] : 0.f;
        }
    }
    if (tid < MP) vv[tid] = 0.f;
    floatx4 M[MNB][2];
#pragma unroll
    for (int bi = 0; bi < MNB; ++bi)
#pragma unroll
        for (int cl = 0; cl < 2; ++cl)
#pragma unroll
            for (int r = 0; r < 4; ++r) M[bi][cl][r] = (bi == 2 * w + cl && 4 * g + r == c) ? 1.f : 0.f;
    uint32_t mr = 0;
    // the step's operands, loaded one step ahead: s_{t-1} (thread tid < D), s_t and U x_t + b
    // (thread (mi, 0), mi < D)
    float sp_n = 0.f, sc_n = 0.f, ub_n = 0.f;
    auto fetch = [&](int st) {
        const int64_t row = row_lo + st;
        if (tid < D)
            sp_n = (st == 0 && first) ? a.s0[(size_t)b * D + tid] : s[(size_t)(row - 1) * D + tid];
        if (mh == 0 && mi < D) {
            sc_n = s[(size_t)row * D + mi];
            ub_n = a.ub[(size_t)row * D + mi];
        }
    };
    fetch(0);
    __syncthreads();
    for (int st = 0; st < len; ++st) {
        const int64_t row = row_lo + st;
        const float sp = sp_n, sc = sc_n, ubv = ub_n;
        fetch(min(st + 1, len - 1));                      // (the last step re-reads)
        if (tid < MP) {                                   // tanh and d of s_{t-1}
            const float t_ = tid < D ? tanhf_(sp) : 0.f;
            const float d_ = tid < D ? 1.f - t_ * t_ : 0.f;
            th[tid] = t_;
            dk[tid] = d_;
            dv[tid] = d_ * vv[tid];
        }
        __syncthreads();
        // f_i - ub_i = (W tanh s_{t-1})_i and (A_t v)_i = (W (d (.) v))_i
        const float pf = pair_sum(wr.dot(th, mh));
        const float pv = pair_sum(wr.dot(dv, mh));
        // M <- W (d (.) M): the lane's rows of d
        float4 dr[MNB];
#pragma unroll
        for (int bi = 0; bi < MNB; ++bi) dr[bi] = *(const float4*)(dk + 16 * bi + 4 * g);
        floatx4 Mn[MNB][2];
        if constexpr (BF) {
            bf16x8 Bb[MKK][2];
#pragma unroll
            for (int kk = 0; kk < MKK; ++kk)
#pragma unroll
                for (int cl = 0; cl < 2; ++cl)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int bi = 2 * kk + (j >> 2), r = j & 3;
                        const float dd = r == 0 ? dr[bi].x : (r == 1 ? dr[bi].y : (r == 2 ? dr[bi].z : dr[bi].w));
                        Bb[kk][cl][j] = (__bf16)(dd * M[bi][cl][r]);
                    }
#pragma unroll
            for (int bo = 0; bo < MNB; ++bo) {
#pragma unroll
                for (int cl = 0; cl < 2; ++cl) Mn[bo][cl] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < MKK; ++kk) {
                    const bf16x8 av = wb[(bo * MKK + kk) * 64 + l];
#pragma unroll
                    for (int cl = 0; cl < 2; ++cl)
                        Mn[bo][cl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, Bb[kk][cl],
                                                                             Mn[bo][cl], 0, 0, 0);
                }
            }
        } else {
            float Bf[MNB][2][4];
#pragma unroll
            for (int bi = 0; bi < MNB; ++bi)
#pragma unroll
                for (int cl = 0; cl < 2; ++cl) {
                    Bf[bi][cl][0] = dr[bi].x * M[bi][cl][0];
                    Bf[bi][cl][1] = dr[bi].y * M[bi][cl][1];
                    Bf[bi][cl][2] = dr[bi].z * M[bi][cl][2];
                    Bf[bi][cl][3] = dr[bi].w * M[bi][cl][3];
                }
#pragma unroll
            for (int bo = 0; bo < MNB; ++bo) {
#pragma unroll
                for (int cl = 0; cl < 2; ++cl) Mn[bo][cl] = floatx4{0.f, 0.f, 0.f, 0.f};
                const float* wrow = wf + (c + 16 * bo) * (MP + 1) + 4 * g;
#pragma unroll
                for (int sk = 0; sk < MP / 4; ++sk) {
                    const float av = wrow[(sk & 3) + 16 * (sk >> 2)];
#pragma unroll
                    for (int cl = 0; cl < 2; ++cl)
                        Mn[bo][cl] = mfma16x4(av, Bf[sk >> 2][cl][sk & 3], Mn[bo][cl]);
                }
            }
        }
#pragma unroll
        for (int bi = 0; bi < MNB; ++bi)
#pragma unroll
            for (int cl = 0; cl < 2; ++cl) M[bi][cl] = Mn[bi][cl];
        __syncthreads();                                  // th, dk, dv, vv read by everyone
        if (mh == 0 && mi < D) {
            const float f = pf + ubv;
            const float r = sc - f;
            mr = max(mr, absbits(r));
            vv[mi] = pv - r;
            a.rd[((size_t)row * 2 + 0) * D + mi] = r;
            a.rd[((size_t)row * 2 + 1) * D + mi] = dk[mi];
        }
        __syncthreads();
    }
    float* mp = a.mbuf + (size_t)gi * MP * MP;
#pragma unroll
    for (int bi = 0; bi < MNB; ++bi)
#pragma unroll
        for (int cl = 0; cl < 2; ++cl)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                mp[(size_t)(4 * g + r + 16 * bi) * MP + c + 16 * (2 * w + cl)] = M[bi][cl][r];
    if (tid < MP) a.vbuf[(size_t)gi * MP + tid] = vv[tid];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mr = max(mr, (uint32_t)__shfl_xor((int)mr, off));
    if (l == 0) atomicMax(&a.seq[b].maxr, mr);
}

// ---- walk: one workgroup per sequence (after the decision of this iteration) ----------------
// Thread (i, p) = (tid >> 3, tid & 7) of 1024 holds columns 16p .. 16p + 15 of row i of the
// next WPF maps (every load unconditional, clamped to the last map, so that the compiler's
// waits keep them in flight): the walk is a chain of dependent mat-vecs.
constexpr int WPF = 5;
__global__ void __launch_bounds__(1024) mf_walk_kernel(MfArgs a) {
    __shared__ __attribute__((aligned(16))) float wsh[MP];
    if (ld_i32(&a.ctrl->all_done)) return;
    const int b = blockIdx.x;
    if (a.seq[b].status != kActive) return;
    const int g0 = a.group_start[b], G = a.group_start[b + 1] - g0;
    const int tid = threadIdx.x, mi = tid >> 3, mp = tid & 7;
    if (tid < MP) {
        wsh[tid] = 0.f;
        if (G > 0) a.wcar[(size_t)g0 * MP + tid] = 0.f;
    }
    const int nq = G - 1;                                // maps applied
    if (nq <= 0) return;                                 // (uniform)
    float4 ring[WPF][4];
    float rv[WPF];
    auto fetch = [&](int q, int j) {
        const float* mrow = a.mbuf + (size_t)(g0 + q) * MP * MP + (size_t)mi * MP + 16 * mp;
#pragma unroll
        for (int k = 0; k < 4; ++k) ring[j][k] = *(const float4*)(mrow + 4 * k);
        rv[j] = a.vbuf[(size_t)(g0 + q) * MP + mi];
    };
#pragma unroll
    for (int j = 0; j < WPF; ++j) fetch(min(j, nq - 1), j);
    __syncthreads();
    for (int q0 = 0; q0 < nq; q0 += WPF) {
#pragma unroll
        for (int j = 0; j < WPF; ++j) {
            const int q = q0 + j;
            float p0 = 0.f, p1 = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 u = *(const float4*)(wsh + 16 * mp + 4 * k);
                p0 = fmaf(ring[j][k].x, u.x, p0);
                p1 = fmaf(ring[j][k].y, u.y, p1);
                p0 = fmaf(ring[j][k].z, u.z, p0);
                p1 = fmaf(ring[j][k].w, u.w, p1);
            }
            float p = p0 + p1;
            p += __shfl_xor(p, 1);
            p += __shfl_xor(p, 2);
            p += __shfl_xor(p, 4);
            const float y = p + rv[j];
            fetch(min(q + WPF, nq - 1), j);
            __syncthreads();
            if (q < nq && mp == 0) {
                wsh[mi] = y;
                a.wcar[(size_t)(g0 + q + 1) * MP + mi] = y;
            }
            __syncthreads();
        }
    }
}

// ---- apply pass: one workgroup per group ------------------------------------------------------
// s^(k+1)_t = s^(k)_t + Delta_t.  Reset guard (the heuristic of the other solvers): a step
// whose new state has an entry that is not finite or exceeds reset_abs in magnitude is set to
// zero, and the recurrence continues from the Delta that leads there.
__global__ void __launch_bounds__(256) mf_apply_kernel(MfArgs a) {
    __shared__ __attribute__((aligned(16))) float dl[MP];
    __shared__ __attribute__((aligned(16))) float dd[MP];
    __shared__ int bad[2];
    if (ld_i32(&a.ctrl->all_done)) return;
    const int gi = blockIdx.x;
    if (gi >= a.ngroups) return;                        // (an empty batch launches one)
    int64_t row_lo;
    int len, b;
    bool first;
    mf_group_rows(a, gi, row_lo, len, b, first);
    if (a.seq[b].status != kActive) return;
    const int k1 = a.ctrl->iter;                        // the decision has counted iteration k
    const float reset_abs = a.ctrl->reset_abs;
    const float* __restrict__ sold = a.sbuf[(k1 + 1) & 1];
    float* __restrict__ snew = a.sbuf[k1 & 1];
    const int D = a.D;
    const int tid = threadIdx.x, mi = tid >> 1, mh = tid & 1;
    MfRow wr;
    wr.load(a.W, D, mi, mh);
    if (tid < MP) dl[tid] = a.wcar[(size_t)gi * MP + tid];
    if (tid < 2) bad[tid] = 0;
    int resets = 0;
    // d_t (thread tid < D), r_t and s^(k)_t (thread (mi, 0)), one step ahead
    float d_n = 0.f, r_n = 0.f, so_n = 0.f;
    auto fetch = [&](int st) {
        const int64_t row = row_lo + st;
        if (tid < D) d_n = a.rd[((size_t)row * 2 + 1) * D + tid];
        if (mh == 0 && mi < D) {
            r_n = a.rd[((size_t)row * 2 + 0) * D + mi];
            so_n = sold[(size_t)row * D + mi];
        }
    };
    fetch(0);
    __syncthreads();
    for (int st = 0; st < len; ++st) {
        const int64_t row = row_lo + st;
        const float dv_ = d_n, rv = r_n, so = so_n;
        fetch(min(st + 1, len - 1));
        if (tid < MP) dd[tid] = tid < D ? dv_ * dl[tid] : 0.f;
        __syncthreads();
        const float y = pair_sum(wr.dot(dd, mh));
        float del = 0.f, sn = 0.f;
        if (mh == 0 && mi < D) {
            del = y - rv;
            sn = so + del;
            if (!(fabsf(sn) <= reset_abs)) bad[st & 1] = 1;   // NaN fails the test too
        }
        if (tid == 0) bad[(st + 1) & 1] = 0;             // the next step's flag
        __syncthreads();
        const bool reset = bad[st & 1] != 0;
        if (mh == 0 && mi < D) {
            if (reset) {
                sn = 0.f;
                del = -so;
            }
            dl[mi] = del;
            snew[(size_t)row * D + mi] = sn;
        }
        resets += reset ? 1 : 0;
        __syncthreads();
    }
    if (tid == 0 && resets) atomicAdd(&a.seq[b].resets_pending, resets);
}

// ---- sequential rollout and LLE (one workgroup per sequence) ----------------------------------
__global__ void __launch_bounds__(256) mf_seq_kernel(const float* __restrict__ ub,
                                                     const float* __restrict__ s0,
                                                     const float* __restrict__ W, int D,
                                                     float* __restrict__ s,
                                                     const int64_t* __restrict__ offsets) {
    __shared__ __attribute__((aligned(16))) float th[MP];
    const int b = blockIdx.x, tid = threadIdx.x, mi = tid >> 1, mh = tid & 1;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    MfRow wr;
    wr.load(W, D, mi, mh);
    float sv = (tid < D) ? s0[(size_t)b * D + tid] : 0.f;   // threads tid < MP own s[tid]
    for (int64_t t = 0; t < T; ++t) {
        if (tid < MP) th[tid] = tid < D ? tanhf_(sv) : 0.f;
        __syncthreads();
        const float y = pair_sum(wr.dot(th, mh));
        __syncthreads();
        // thread (mi, 0) has row mi; hand it to thread mi (which keeps s[mi]) through LDS
        if (mh == 0) th[mi] = mi < D ? y + ub[(size_t)(r0 + t) * D + mi] : 0.f;
        __syncthreads();
        if (tid < MP) {
            sv = th[tid];
            if (tid < D) s[(size_t)(r0 + t) * D + tid] = sv;
        }
        __syncthreads();
    }
}

// Alg. LLE_estimate: u pushed through A_t = W diag(1 - tanh^2(s_{t-1})), renormalised each
// step; the mean log stretch.
__global__ void __launch_bounds__(256) mf_lle_kernel(const float* __restrict__ s0,
                                                     const float* __restrict__ s,
                                                     const float* __restrict__ u0,
                                                     const float* __restrict__ W, int D,
                                                     const int64_t* __restrict__ offsets,
                                                     double* out) {
    __shared__ __attribute__((aligned(16))) float du[MP];
    __shared__ float red[4];
    const int b = blockIdx.x, tid = threadIdx.x, mi = tid >> 1, mh = tid & 1;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    MfRow wr;
    wr.load(W, D, mi, mh);
    float u = (tid < D) ? u0[(size_t)b * D + tid] : 0.f;    // threads tid < MP own u[tid]
    auto block_sum = [&](float v) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        const float tot = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
        return tot;
    };
    {
        const float n2 = block_sum(tid < MP ? u * u : 0.f);
        u = u / sqrtf(n2);
    }
    double total = 0.0;
    for (int64_t t = 0; t < T; ++t) {
        if (tid < MP) {
            float sp = 0.f;
            if (tid < D) sp = t == 0 ? s0[(size_t)b * D + tid] : s[(size_t)(r0 + t - 1) * D + tid];
            const float th = tanhf_(sp);
            du[tid] = tid < D ? (1.f - th * th) * u : 0.f;
        }
        __syncthreads();
        const float y = pair_sum(wr.dot(du, mh));
        __syncthreads();
        if (mh == 0) du[mi] = y;                          // (W d u)[mi] to thread mi
        __syncthreads();
        const float v = tid < MP ? du[tid] : 0.f;
        const float n2 = block_sum(v * v);
        const float nrm = sqrtf(n2);
        total += (double)logf(nrm);
        u = v / nrm;
    }
    if (tid == 0) out[b] = T > 0 ? total / (double)T : 0.0;
}

// ---- host ---------------------------------------------------------------------------------------
namespace {
constexpr int kMfTile = 32;

struct MfLayout {
    IterState st;
    float *ub, *salt, *rd, *mbuf, *vbuf, *wcar;
    size_t bytes;
};

MfLayout mf_layout(void* ws, int D, const HostBatch& hb, int ntiles, int ngroups) {
    Carver c(ws);
    MfLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles, ngroups);
    lay.ub = c.take<float>((size_t)hb.N * D);
    lay.salt = c.take<float>((size_t)hb.N * D);
    lay.rd = c.take<float>((size_t)hb.N * 2 * D);
    const size_t ng = (size_t)std::max(ngroups, 1);
    lay.mbuf = c.take<float>(ng * MP * MP);
    lay.vbuf = c.take<float>(ng * MP);
    lay.wcar = c.take<float>(ng * MP);
    lay.bytes = c.bytes();
    return lay;
}

// Group length (measured per step and group at D = 100): the map and apply passes walk a
// group's steps one after another, one workgroup per group and CU (about 2.5 us per step with
// BF16 maps, 10 us with FP32 maps, in rounds of one group per CU), the walk one group after
// another (about 0.9 us per group of the longest sequence).  The default minimises that
// estimate over powers of two.
int mf_group_tiles(const std::vector<int32_t>& ts, const HostBatch& hb, const pn_opts& o) {
    if (o.group > 0) return o.group;
    int tmax = 0;
    for (int b = 0; b < hb.B; ++b) tmax = std::max(tmax, ts[b + 1] - ts[b]);
    const double step_us = o.compose == PN_COMPOSE_BF16 ? 2.5 : 10.0;
    int best = 1;
    double best_us = 1e300;
    for (int gt = 1; gt <= 64; gt *= 2) {
        const int ng = count_groups(ts, hb.B, gt);
        const double rounds = std::ceil((double)std::max(ng, 1) / cu_count());
        const double us = rounds * kMfTile * gt * step_us + 0.9 * ((tmax + gt - 1) / gt);
        if (us < best_us) best_us = us, best = gt;
    }
    return best;
}

void mf_upload_offsets(int64_t* doff, const HostBatch& hb, hipStream_t stream) {
    (void)hipMemcpyAsync(doff, hb.offsets.data(), sizeof(int64_t) * (hb.B + 1),
                         hipMemcpyHostToDevice, stream);
}
}  // namespace

bool mf_dense_supported(int D, int Dx) { return D > 16 && D <= MP && Dx >= 1 && Dx <= 1024; }

size_t mf_dense_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    (void)Dx;
    const std::vector<int32_t> ts = tile_starts(hb, kMfTile);
    const int gt = mf_group_tiles(ts, hb, o);
    return mf_layout(nullptr, D, hb, ts[hb.B], count_groups(ts, hb.B, gt)).bytes;
}

pn_status mf_dense_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                           const float* s0, float* s, const pn_opts& o, void* ws,
                           hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    const int D = cd.D, Dx = cd.Dx;
    if (!mf_dense_supported(D, Dx)) {
        set_error("dense DEER for the mean-field cell is built for 16 < D <= %d", MP);
        return PN_ERR_UNSUPPORTED;
    }
    const std::vector<int32_t> ts = tile_starts(hb, kMfTile);
    const int ntiles = ts[hb.B];
    const int gt = mf_group_tiles(ts, hb, o);
    const int ngroups = count_groups(ts, hb.B, gt);
    MfLayout lay = mf_layout(ws, D, hb, ntiles, ngroups);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, kMfTile, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream, gt));
    MfArgs a;
    a.x = x;
    a.s0 = s0;
    a.W = (const float*)cd.params;
    a.U = a.W + (size_t)D * D;
    a.bias = a.U + (size_t)D * Dx;
    a.D = D;
    a.Dx = Dx;
    a.ub = lay.ub;
    a.sbuf[0] = s;
    a.sbuf[1] = lay.salt;
    a.rd = lay.rd;
    a.mbuf = lay.mbuf;
    a.vbuf = lay.vbuf;
    a.wcar = lay.wcar;
    a.ctrl = lay.st.ctrl;
    a.seq = lay.st.seq;
    a.tiles = lay.st.tiles;
    a.groups = lay.st.groups;
    a.group_start = lay.st.group_start;
    a.ngroups = ngroups;
    a.B = hb.B;
    if (hb.N > 0) {
        const int ug = (int)std::min<int64_t>(8 * cu_count(), (hb.N * D + 255) / 256);
        hipLaunchKernelGGL(mf_ub_kernel, dim3(ug), dim3(256), 0, stream, x, a.U, a.bias, lay.ub,
                           hb.N, D, Dx);
        PN_HIP(hipGetLastError());
    }
    const bool bf = o.compose == PN_COMPOSE_BF16;
    void (*mapk)(MfArgs) = bf ? mf_map_kernel<true> : mf_map_kernel<false>;
    const int grid = std::max(1, ngroups);
    auto one_iter = [&](hipStream_t st) {
        prof_launch("mf_dense_map", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(mapk, dim3(grid), dim3(256), 0, s2, a);
        });
        launch_decide(lay.st, hb.B, st, true);
        prof_launch("mf_dense_walk", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(mf_walk_kernel, dim3(hb.B), dim3(1024), 0, s2, a);
        });
        prof_launch("mf_dense_apply", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(mf_apply_kernel, dim3(grid), dim3(256), 0, s2, a);
        });
    };
    std::vector<uintptr_t> key = {0x4D46u, (uintptr_t)hb.N, lay.bytes, (uintptr_t)mapk,
                                  (uintptr_t)grid, (uintptr_t)x, (uintptr_t)s0, (uintptr_t)s,
                                  (uintptr_t)cd.params, (uintptr_t)ws, (uintptr_t)hb.B,
                                  (uintptr_t)D, (uintptr_t)Dx, (uintptr_t)ngroups};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    return finish_iterations(lay.st, hb, D, sizeof(float), s, lay.salt, stream, info, all_conv);
}

size_t mf_seq_workspace(int D, const HostBatch& hb) {
    Carver c(nullptr);
    c.take<int64_t>(hb.B + 1);
    c.take<float>((size_t)hb.N * D);
    c.take<double>(std::max(hb.B, 1));
    return c.bytes();
}

pn_status mf_seq_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                     const float* s0, float* s, void* ws, hipStream_t stream) {
    const int D = cd.D, Dx = cd.Dx;
    if (hb.N == 0) return PN_OK;
    Carver c(ws);
    int64_t* doff = c.take<int64_t>(hb.B + 1);
    float* ub = c.take<float>((size_t)hb.N * D);
    mf_upload_offsets(doff, hb, stream);
    const float* W = (const float*)cd.params;
    const float* U = W + (size_t)D * D;
    const int ug = (int)std::min<int64_t>(8 * cu_count(), (hb.N * D + 255) / 256);
    hipLaunchKernelGGL(mf_ub_kernel, dim3(ug), dim3(256), 0, stream, x, U, U + (size_t)D * Dx,
                       ub, hb.N, D, Dx);
    prof_launch("seq_rollout", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(mf_seq_kernel, dim3(hb.B), dim3(256), 0, s2, (const float*)ub, s0, W,
                           D, s, (const int64_t*)doff);
    });
    PN_HIP(hipGetLastError());
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    return PN_OK;
}

pn_status mf_lle_run(const pn_cell_desc& cd, const HostBatch& hb, const float* s0,
                     const float* s, const float* u0, void* ws, hipStream_t stream, double* lle) {
    if (hb.B == 0) return PN_OK;
    Carver c(ws);                                   // the layout of lle_workspace
    int64_t* doff = c.take<int64_t>(hb.B + 1);
    double* out = c.take<double>(std::max(hb.B, 1));
    mf_upload_offsets(doff, hb, stream);
    hipLaunchKernelGGL(mf_lle_kernel, dim3(hb.B), dim3(256), 0, stream, s0, s, u0,
                       (const float*)cd.params, cd.D, (const int64_t*)doff, out);
    PN_HIP(hipGetLastError());
    PN_HIP(hipMemcpyAsync(lle, out, sizeof(double) * hb.B, hipMemcpyDeviceToHost, stream));
    PN_HIP(hipStreamSynchronize(stream));
    return PN_OK;
}

}  // namespace pn
