// ELK (Ch. 4): each Newton iteration replaces the DEER step by the filtered means of the
// linear-Gaussian SSM of Prop. prop:ELK, written in step coordinates Delta_t = s_t - s^(i)_t:
//   Delta_t = A_t Delta_{t-1} - r_t + w_t, w_t ~ N(0, I);   0 = Delta_t + v_t, v_t ~ N(0, I/lambda)
// whose Kalman filter (Sec. "Dynamics perspective on ELK") is
//   P- = A_t P A_t^T + I,  Gamma_t = (lambda P- + I)^-1,  P = Gamma_t P-,  m = Gamma_t (A_t m - r_t).
// For the tanh-RNN (D = 16) A_t = diag(1 - f_t^2) W is rebuilt on chip from the iterate.
//
// The filter is parallelised over time as an associative scan of 5-tuple elements
// (A, b, C, eta, J) -- the parallel Kalman filter the thesis cites (Ch. 2).  One single-wave
// workgroup takes a chunk of L steps:
//   1. linearise the chunk (FP32 MFMA GEMM for the pre-activations, residual, d_t);
//   2. fold the chunk's leaves into its aggregate element (one 16x16 inverse and nine 16x16
//      products per step, products on FP32 MFMA 16x16x4, the inverse by Gauss-Jordan with
//      partial pivoting in LDS) and publish it;
//   3. look back over the preceding chunks for the filtered (m, P) at the chunk boundary;
//   4. run the exact filter over the chunk from that (m, P), write s + m (reset guard) and
//      publish the chunk's final (m, P).
// lambda = 0 gives Gamma_t = I: the DEER step.
#include <algorithm>
#include <cstring>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

constexpr int ED = 16;                 // state size
constexpr int ES = 17;                 // LDS row stride of a 16x16 matrix
constexpr int EM = ED * ES;            // floats per stored matrix
constexpr int MW = ED * ED / 2;        // u64 words per published matrix
constexpr int EAGG = 3 * MW + ED;      // A, C, J, b, eta
constexpr int EINC = MW + ED / 2;      // P, m

// C = alpha * op(X) op(Y) + [Add] + addI * I (16x16, LDS, C may alias X, Y or Add)
PN_DEV void mm16(float* C, const float* X, bool tx, const float* Y, bool ty, float alpha,
                 const float* Add, float addI) {
    const int l = threadIdx.x & 63, g = l >> 4, u = l & 15;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + g;
        const float av = tx ? X[k * ES + u] : X[u * ES + k];
        const float bv = ty ? Y[u * ES + k] : Y[k * ES + u];
        acc = mfma16x4(av, bv, acc);
    }
    float out[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * g + i;
        float v = alpha * acc[i];
        if (Add) v += Add[r * ES + u];
        if (r == u) v += addI;
        out[i] = v;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) C[(4 * g + i) * ES + u] = out[i];
    __syncthreads();
}

// y = alpha * op(M) x + beta * add   (16-vectors in LDS; y may alias x or add)
PN_DEV void mv16(float* y, const float* M, bool tm, const float* x, float alpha, const float* add,
                 float beta) {
    const int l = threadIdx.x & 63;
    float v = 0.f;
    if (l < ED) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < ED; ++k) acc += (tm ? M[k * ES + l] : M[l * ES + k]) * x[k];
        v = alpha * acc + (add ? beta * add[l] : 0.f);
    }
    __syncthreads();
    if (l < ED) y[l] = v;
    __syncthreads();
}

// G = M^-1 by Gauss-Jordan with partial pivoting on [M | I] (aug: 16 x 33 floats).
PN_DEV void inv16(float* G, const float* M, float* aug, float* fac) {
    const int l = threadIdx.x & 63;
    constexpr int AS = 33;
    for (int idx = l; idx < ED * 32; idx += 64) {
        const int r = idx / 32, c = idx % 32;
        aug[r * AS + c] = c < ED ? M[r * ES + c] : (c - ED == r ? 1.f : 0.f);
    }
    __syncthreads();
    for (int k = 0; k < ED; ++k) {
        float v = (l < ED && l >= k) ? fabsf(aug[l * AS + k]) : -1.f;
        int idx = l;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const float ov = __shfl_xor(v, off);
            const int oi = __shfl_xor(idx, off);
            if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
        }
        const int p = __shfl(idx, 0);
        if (p != k && l < 32) {
            const float a0 = aug[k * AS + l], a1 = aug[p * AS + l];
            aug[k * AS + l] = a1;
            aug[p * AS + l] = a0;
        }
        __syncthreads();
        if (l < ED) fac[l] = aug[l * AS + k];
        __syncthreads();
        const float inv = 1.f / fac[k];
        if (l < 32) aug[k * AS + l] *= inv;
        __syncthreads();
        {
            const int c = l & 31;
            for (int r = l >> 5; r < ED; r += 2)
                if (r != k) aug[r * AS + c] -= fac[r] * aug[k * AS + c];
        }
        __syncthreads();
    }
    for (int idx = l; idx < ED * ED; idx += 64) {
        const int r = idx / ED, c = idx % ED;
        G[r * ES + c] = aug[r * AS + ED + c];
    }
    __syncthreads();
}

PN_DEV void publish_mat(uint64_t* dst, const float* M) {
    const int l = threadIdx.x & 63;
    for (int w = l; w < MW; w += 64) {
        const int r = w / 8, c = 2 * (w % 8);
        st_u64(&dst[w], pack2(M[r * ES + c], M[r * ES + c + 1]));
    }
}
PN_DEV void publish_vec(uint64_t* dst, const float* v) {
    const int l = threadIdx.x & 63;
    if (l < ED / 2) st_u64(&dst[l], pack2(v[2 * l], v[2 * l + 1]));
}
PN_DEV void load_mat(float* M, const uint64_t* src) {
    const int l = threadIdx.x & 63;
    for (int w = l; w < MW; w += 64) {
        const uint64_t v = ld_u64(&src[w]);
        const int r = w / 8, c = 2 * (w % 8);
        M[r * ES + c] = lo_of(v);
        M[r * ES + c + 1] = hi_of(v);
    }
}
PN_DEV void load_vec(float* x, const uint64_t* src) {
    const int l = threadIdx.x & 63;
    if (l < ED / 2) {
        const uint64_t v = ld_u64(&src[l]);
        x[2 * l] = lo_of(v);
        x[2 * l + 1] = hi_of(v);
    }
}
PN_DEV bool words_ready(const uint64_t* src, int n) {
    const int l = threadIdx.x & 63;
    bool ok = true;
    for (int w = l; w < n; w += 64) ok = ok && ready64(ld_u64(&src[w]));
    return __all(ok);
}

struct ElkArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];
    const float* params;     // W (16x16) | U (16xDx) | b (16)
    uint64_t* agg[2];
    uint64_t* incl[2];
    Ctrl* ctrl;
    SeqState* seq;
    const int64_t* offsets;
    const int32_t* tile_start;
    const int32_t* order;
    int B;
    int ntiles;
    float lam;
    int res64;               // nonzero: the stopping residual is evaluated in FP64
    int diag;                // nonzero: quasi-ELK, the LGSSM uses diag(A_t)
};

template <int DX, int L>
__global__ void __launch_bounds__(64) elk_iter_kernel(ElkArgs a) {
    constexpr int KT = ED + DX;
    constexpr int SS = ED + 4, XS = DX + 4;
    static_assert(L % 16 == 0 && KT % 4 == 0, "shape");
    __shared__ __attribute__((aligned(16))) float sst[(L + 1) * SS];
    __shared__ __attribute__((aligned(16))) float xst[L * XS];
    __shared__ float dsh[L * ED], rsh[L * ED];
    __shared__ float Wm[EM], Ai[EM], Ci[EM], Ji[EM], At[EM], Jj[EM], Gm[EM], T1[EM], T2[EM];
    __shared__ float aug[ED * 33];
    __shared__ float fac[ED];
    __shared__ float bi[ED], ei[ED], vx[ED], vy[ED], vz[ED];
    __shared__ int tinfo[5];

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k_it = a.ctrl->iter;
    const int par = k_it & 1;
    const float reset_abs = a.ctrl->reset_abs;
    const float lam = a.lam;
    const float s1 = 1.f / (1.f + lam);           // 1 / (1 + lambda)
    const float kap = lam / (1.f + lam);         // kappa
    const float* __restrict__ sin = a.sbuf[par];
    float* __restrict__ sout = a.sbuf[par ^ 1];
    const int l = threadIdx.x, g = l >> 4, u = l & 15;

    const float* W = a.params;
    const float* U = W + ED * ED;
    const float* bvec = U + ED * DX;
    for (int idx = l; idx < ED * ED; idx += 64) Wm[(idx / ED) * ES + idx % ED] = W[idx];
    float blin[KT / 4];                          // B operand [W | U]^T, unit u, k = 4kb + g
#pragma unroll
    for (int kb = 0; kb < KT / 4; ++kb) {
        const int kk = 4 * kb + g;
        blin[kb] = kk < ED ? W[u * ED + kk] : U[u * DX + (kk - ED)];
    }
    const float bias_u = bvec[u];

    for (;;) {
        __syncthreads();
        if (l == 0) {
            const int idx = (int)atomicAdd(&a.ctrl->tile_counter, 1u);
            tinfo[0] = idx;
            if (idx < a.ntiles) {
                const int slot = a.order[idx];
                int lo = 0, hi = a.B;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (a.tile_start[mid] <= slot) lo = mid; else hi = mid;
                }
                const int lt = slot - a.tile_start[lo];
                tinfo[1] = lo;
                tinfo[2] = lt;
                tinfo[3] = (a.seq[lo].status == kActive)
                               ? (int)std::min<int64_t>(L, a.offsets[lo + 1] - a.offsets[lo] - (int64_t)lt * L)
                               : -1;
                tinfo[4] = slot;
            }
        }
        __syncthreads();
        if (tinfo[0] >= a.ntiles) break;
        const int tile = tinfo[4];
        const int b = tinfo[1], lt = tinfo[2], len = tinfo[3];
        if (len < 0) continue;
        const bool first = lt == 0;
        const int64_t row0 = a.offsets[b] + (int64_t)lt * L;
        for (int w = l; w < EAGG; w += 64) st_u64(&a.agg[par ^ 1][(size_t)tile * EAGG + w], kSent64);
        for (int w = l; w < EINC; w += 64) st_u64(&a.incl[par ^ 1][(size_t)tile * EINC + w], kSent64);

        // ---- stage and linearise
        for (int idx = l; idx < (L + 1) * (ED / 4); idx += 64) {
            const int r = idx / (ED / 4), c4 = idx % (ED / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r == 0) v = first ? *(const float4*)(a.s0 + (size_t)b * ED + 4 * c4)
                                  : *(const float4*)(sin + (size_t)(row0 - 1) * ED + 4 * c4);
            else if (r - 1 < len) v = *(const float4*)(sin + (size_t)(row0 + r - 1) * ED + 4 * c4);
            *(float4*)(sst + r * SS + 4 * c4) = v;
        }
        for (int idx = l; idx < L * (DX / 4); idx += 64) {
            const int r = idx / (DX / 4), c4 = idx % (DX / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
            *(float4*)(xst + r * XS + 4 * c4) = v;
        }
        __syncthreads();
        uint32_t rmax = 0;
#pragma unroll
        for (int mb = 0; mb < L / 16; ++mb) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KT / 4; ++kb) {
                const int kk = 4 * kb + g, tr = mb * 16 + u;
                const float av = kk < ED ? sst[tr * SS + kk] : xst[tr * XS + (kk - ED)];
                acc = mfma16x4(av, blin[kb], acc);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = mb * 16 + 4 * g + i;
                const float f = tanhf_(acc[i] + bias_u);
                const float res = sst[(t + 1) * SS + u] - f;
                dsh[t * ED + u] = (first && t == 0) ? 0.f : 1.f - f * f;
                rsh[t * ED + u] = res;
                if (t < len && !a.res64) rmax = max(rmax, absbits(res));
            }
        }
        if (a.res64) {
            // The stopping test of this iterate in FP64: s, x and the parameters upcast, the
            // same quantity the final FP64 residual reports.  The FP32 residual above still
            // drives the update; its rounding (~1e-7 here) would otherwise let an iterate
            // pass a 1e-6 test that it fails in FP64.  The bound is rounded up to FP32.
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = 4 * g + i;
                for (int tt = t; tt < L && tt < len; tt += 16) {
                    double acc = (double)bias_u;
                    for (int kk = 0; kk < ED; ++kk)
                        acc += (double)Wm[u * ES + kk] * (double)sst[tt * SS + kk];
                    for (int kk = 0; kk < DX; ++kk)
                        acc += (double)U[u * DX + kk] * (double)xst[tt * XS + kk];
                    const double r = (double)sst[(tt + 1) * SS + u] - tanh(acc);
                    const double ar = fabs(r);
                    float fr = (float)ar;
                    if ((double)fr < ar) fr = nextafterf(fr, INFINITY);
                    rmax = max(rmax, (r == r) ? absbits(fr) : 0x7F800000u);
                }
            }
        }
        __syncthreads();

        auto build_At = [&](int t) {
            for (int idx = l; idx < ED * ED; idx += 64) {
                const int r = idx / ED, c = idx % ED;
                At[r * ES + c] = (a.diag && r != c) ? 0.f : dsh[t * ED + r] * Wm[r * ES + c];
            }
            __syncthreads();
        };

        // ---- fold the chunk into its aggregate element and publish it
        if (!first) {
            // leaf of the chunk's first step
            build_At(0);
            for (int idx = l; idx < ED * ED; idx += 64) {
                const int r = idx / ED, c = idx % ED;
                Ai[r * ES + c] = s1 * At[r * ES + c];
                Ci[r * ES + c] = (r == c) ? s1 : 0.f;
            }
            if (l < ED) { bi[l] = -s1 * rsh[l]; vx[l] = rsh[l]; }
            __syncthreads();
            mv16(ei, At, true, vx, kap, nullptr, 0.f);            // eta = kappa A^T r
            mm16(Ji, At, true, At, false, kap, nullptr, 0.f);     // J = kappa A^T A
            for (int t = 1; t < len; ++t) {
                build_At(t);
                if (l < ED) vx[l] = rsh[t * ED + l];
                __syncthreads();
                mm16(Jj, At, true, At, false, kap, nullptr, 0.f);     // J_j
                mv16(vy, At, true, vx, kap, nullptr, 0.f);            // eta_j
                mm16(T1, Ci, false, Jj, false, 1.f, nullptr, 1.f);    // I + C_i J_j
                inv16(Gm, T1, aug, fac);                              // G
                mm16(T2, At, false, Gm, false, s1, nullptr, 0.f);     // A_j G
                // eta, J use the old A_i
                mv16(vz, Jj, false, bi, -1.f, vy, 1.f);               // eta_j - J_j b_i
                mv16(vz, Gm, true, vz, 1.f, nullptr, 0.f);            // G^T (.)
                mv16(ei, Ai, true, vz, 1.f, ei, 1.f);                 // eta = A_i^T (.) + eta_i
                mm16(T1, Jj, false, Ai, false, 1.f, nullptr, 0.f);    // J_j A_i
                mm16(T1, Gm, true, T1, false, 1.f, nullptr, 0.f);     // G^T J_j A_i
                mm16(Ji, Ai, true, T1, false, 1.f, Ji, 0.f);          // J = A_i^T (.) + J_i
                mv16(vz, Ci, false, vy, 1.f, bi, 1.f);                // b_i + C_i eta_j
                mv16(bi, T2, false, vz, 1.f, vx, -s1);                // b = A_j G (.) + b_j
                mm16(T1, T2, false, Ci, false, 1.f, nullptr, 0.f);    // A_j G C_i
                mm16(Ci, T1, false, At, true, s1, nullptr, s1);       // C = (.) A_j^T + C_j
                mm16(Ai, T2, false, Ai, false, 1.f, nullptr, 0.f);    // A = A_j G A_i
            }
            uint64_t* ag = a.agg[par] + (size_t)tile * EAGG;
            publish_mat(ag, Ai);
            publish_mat(ag + MW, Ci);
            publish_mat(ag + 2 * MW, Ji);
            publish_vec(ag + 3 * MW, bi);
            publish_vec(ag + 3 * MW + ED / 2, ei);
        }

        // ---- filtered state (m, P) at the chunk boundary: Ci <- P, bi <- m
        for (int idx = l; idx < ED * ED; idx += 64) Ci[(idx / ED) * ES + idx % ED] = 0.f;
        if (l < ED) bi[l] = 0.f;
        __syncthreads();
        if (!first) {
            int pred = tile - 1, spins = 0;
            for (;;) {
                if (words_ready(a.incl[par] + (size_t)pred * EINC, EINC)) break;
                if (words_ready(a.agg[par] + (size_t)pred * EAGG, EAGG)) { --pred; continue; }
                if (++spins > (1 << 20) || ld_i32(&a.ctrl->error)) { if (l == 0) atomicExch(&a.ctrl->error, 1); break; }
                __builtin_amdgcn_s_sleep(1);
            }
            load_mat(Ci, a.incl[par] + (size_t)pred * EINC);
            load_vec(bi, a.incl[par] + (size_t)pred * EINC + MW);
            __syncthreads();
            for (int p2 = pred + 1; p2 < tile; ++p2) {
                const uint64_t* ag = a.agg[par] + (size_t)p2 * EAGG;
                load_mat(Ai, ag);
                load_mat(T2, ag + MW);       // C_p
                load_mat(Jj, ag + 2 * MW);   // J_p
                load_vec(vx, ag + 3 * MW);   // b_p
                load_vec(vy, ag + 3 * MW + ED / 2);  // eta_p
                __syncthreads();
                mm16(T1, Ci, false, Jj, false, 1.f, nullptr, 1.f);    // I + P J_p
                inv16(Gm, T1, aug, fac);
                mm16(T1, Ai, false, Gm, false, 1.f, nullptr, 0.f);    // A_p G
                mv16(vz, Ci, false, vy, 1.f, bi, 1.f);                // m + P eta_p
                mv16(bi, T1, false, vz, 1.f, vx, 1.f);                // m' = A_p G (.) + b_p
                mm16(Gm, T1, false, Ci, false, 1.f, nullptr, 0.f);    // A_p G P
                mm16(Ci, Gm, false, Ai, true, 1.f, T2, 0.f);          // P' = (.) A_p^T + C_p
            }
        }

        // ---- exact filter over the chunk from (m, P); write s + m; publish (m, P)
        int nreset = 0;
        for (int t = 0; t < len; ++t) {
            build_At(t);
            mm16(T1, At, false, Ci, false, 1.f, nullptr, 0.f);        // A P
            mm16(T2, T1, false, At, true, 1.f, nullptr, 1.f);         // P- = A P A^T + I
            mm16(T1, T2, false, T2, false, 0.f, T2, 0.f);             // copy P- (alpha 0 + add)
            for (int idx = l; idx < ED * ED; idx += 64) {
                const int r = idx / ED, c = idx % ED;
                Jj[r * ES + c] = lam * T2[r * ES + c] + (r == c ? 1.f : 0.f);   // lambda P- + I
            }
            __syncthreads();
            inv16(Gm, Jj, aug, fac);                                  // Gamma
            mm16(Ci, Gm, false, T1, false, 1.f, nullptr, 0.f);        // P = Gamma P-
            for (int idx = l; idx < ED * ED; idx += 64) {              // symmetrise
                const int r = idx / ED, c = idx % ED;
                if (r < c) {
                    const float v = 0.5f * (Ci[r * ES + c] + Ci[c * ES + r]);
                    Ci[r * ES + c] = v;
                    Ci[c * ES + r] = v;
                }
            }
            __syncthreads();
            if (l < ED) vx[l] = -rsh[t * ED + l];
            __syncthreads();
            mv16(vy, At, false, bi, 1.f, vx, 1.f);                    // A m - r
            mv16(bi, Gm, false, vy, 1.f, nullptr, 0.f);               // m = Gamma (.)
            if (l < ED) {
                const float v = sst[(t + 1) * SS + l] + bi[l];
                vz[l] = v;
            }
            __syncthreads();
            const bool bad = (l < ED) && !(fabsf(vz[l]) <= reset_abs);
            const bool rowbad = __any(bad);
            if (l < ED) sout[(size_t)(row0 + t) * ED + l] = rowbad ? 0.f : vz[l];
            nreset += rowbad ? 1 : 0;
        }
        publish_mat(a.incl[par] + (size_t)tile * EINC, Ci);
        publish_vec(a.incl[par] + (size_t)tile * EINC + MW, bi);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) {
            atomicMax(&a.seq[b].maxr, rmax);
            if (nreset) atomicAdd(&a.seq[b].resets_pending, nreset);
        }
    }
}

// ---- host ---------------------------------------------------------------------------------------

constexpr int kElkL = 16;

struct ElkLayout {
    IterState st;
    float* salt;
    uint64_t* agg[2];
    uint64_t* incl[2];
    char* r64;
    size_t bytes;
};

static ElkLayout elk_layout(void* ws, const HostBatch& hb, int ntiles) {
    Carver c(ws);
    ElkLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles);
    lay.salt = c.take<float>((size_t)hb.N * ED);
    for (int p = 0; p < 2; ++p) lay.agg[p] = c.take<uint64_t>((size_t)ntiles * EAGG);
    for (int p = 0; p < 2; ++p) lay.incl[p] = c.take<uint64_t>((size_t)ntiles * EINC);
    lay.r64 = c.take<char>(residual64_workspace(PN_CELL_TANH, ED, 16, hb));   // FP64 residual
    lay.bytes = c.bytes();
    return lay;
}

bool elk_supported(int D, int Dx) { return D == ED && Dx == 16; }

size_t elk_workspace(int, int, const HostBatch& hb, const pn_opts&) {
    return elk_layout(nullptr, hb, tile_starts(hb, kElkL)[hb.B]).bytes;
}

__global__ void elk_fill_kernel(uint64_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = kSent64;
}

pn_status residual64_device(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                            const float* s0, const float* s, void* ws, hipStream_t stream,
                            double* max_resid);

pn_status elk_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                      const float* s0, float* s, double lambda, const pn_opts& o, void* ws,
                      hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    void (*kern)(ElkArgs) = elk_iter_kernel<16, kElkL>;
    const std::vector<int32_t> ts = tile_starts(hb, kElkL);
    const int ntiles = ts[hb.B];
    ElkLayout lay = elk_layout(ws, hb, ntiles);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, kElkL, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream));
    if (ntiles > 0) {
        const size_t na = (size_t)ntiles * EAGG, ni = (size_t)ntiles * EINC;
        hipLaunchKernelGGL(elk_fill_kernel, dim3((unsigned)std::min<size_t>(4096, (na + 255) / 256)),
                           dim3(256), 0, stream, lay.agg[0], na);
        hipLaunchKernelGGL(elk_fill_kernel, dim3((unsigned)std::min<size_t>(4096, (ni + 255) / 256)),
                           dim3(256), 0, stream, lay.incl[0], ni);
        PN_HIP(hipGetLastError());
    }
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, 64, 0) != hipSuccess || occ < 1)
        occ = 1;
    const int grid = std::max(1, std::min(ntiles, cu_count() * occ));
    ElkArgs args;
    args.x = x;
    args.s0 = s0;
    args.sbuf[0] = s;
    args.sbuf[1] = lay.salt;
    args.params = (const float*)cd.params;
    for (int p = 0; p < 2; ++p) { args.agg[p] = lay.agg[p]; args.incl[p] = lay.incl[p]; }
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.offsets = lay.st.offsets;
    args.tile_start = lay.st.tile_start;
    args.order = lay.st.order;
    args.B = hb.B;
    args.ntiles = ntiles;
    args.lam = (float)lambda;
    args.res64 = o.fp64_final_residual ? 1 : 0;
    args.diag = o.jac == PN_JAC_DIAG ? 1 : 0;
    auto one_iter = [&](hipStream_t st) {
        prof_launch("elk_iter", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, s2, args);
        });
        launch_decide(lay.st, hb.B, st);
    };
    uint32_t lam_bits = 0;
    std::memcpy(&lam_bits, &args.lam, sizeof lam_bits);
    std::vector<uintptr_t> key = {0x454Cu, (uintptr_t)kern, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)cd.params,
                                  (uintptr_t)ws, (uintptr_t)hb.B, (uintptr_t)ntiles,
                                  (uintptr_t)lam_bits, (uintptr_t)args.res64,
                                  (uintptr_t)args.diag};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    int derr = 0;
    PN_TRY(finish_iterations(lay.st, hb, ED, sizeof(float), s, lay.salt, stream, info, all_conv,
                             &derr));
    if (derr) {
        set_error("look-back watchdog expired in the ELK scan");
        return PN_ERR_INTERNAL;
    }
    if (o.fp64_final_residual && info) {
        // the reported residual is the FP64 one; the stopping test is re-checked in FP64
        std::vector<double> r64(hb.B);
        PN_TRY(residual64_device(cd, hb, x, s0, s, lay.r64, stream, r64.data()));
        bool allc = true;
        for (int b = 0; b < hb.B; ++b) {
            info[b].max_resid = r64[b];
            if (hb.len(b) > 0 && !(r64[b] < o.tol)) info[b].converged = 0;
            allc = allc && (info[b].converged != 0);
        }
        *all_conv = allc;
    }
    return PN_OK;
}

}  // namespace pn
