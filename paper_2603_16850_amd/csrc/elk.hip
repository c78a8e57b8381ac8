// ELK (Ch. 4): each Newton iteration replaces the DEER step by the filtered means of the
// linear-Gaussian SSM of Prop. prop:ELK, written in step coordinates Delta_t = s_t - s^(i)_t:
//   Delta_t = A_t Delta_{t-1} - r_t + w_t, w_t ~ N(0, I);   0 = Delta_t + v_t, v_t ~ N(0, I/lambda)
// whose Kalman filter (Sec. "Dynamics perspective on ELK") is
//   P- = A_t P A_t^T + I,  Gamma_t = (lambda P- + I)^-1,  P = Gamma_t P-,  m = Gamma_t (A_t m - r_t).
// For the tanh-RNN (D = 16) A_t = diag(1 - f_t^2) W is rebuilt on chip from the iterate (its
// diagonal only for quasi-ELK).
//
// The filter is parallelised over time through 5-tuple elements (A, b, C, eta, J) -- the
// parallel Kalman filter the thesis cites (Ch. 2) -- with the same two-pass structure as the
// diagonal and dense DEER paths.  Steps are cut into chunks of 16 and the chunks of a sequence
// into groups of consecutive chunks (see IterState).  Iteration k:
//   local pass, one single-wave workgroup per group, chunk by chunk:
//     1. (k >= 1) apply the previous step: re-linearise at s^(k-1) and run the exact filter
//        from the filtered state (m, P) entering the group, s^(k) = s^(k-1) + m (reset guard);
//     2. linearise at s^(k) (FP32 MFMA GEMM for the pre-activations, residual, d_t);
//     3. fold the steps' leaves into the group's element (one 16x16 inverse and nine 16x16
//        products per step, products on FP32 MFMA 16x16x4, the inverse by Gauss-Jordan with
//        partial pivoting in LDS);
//   carry pass, one workgroup per sequence: the filtered state entering every group, by
//   applying the group elements in order from (m, P) = (0, 0).
// Converged-prefix skipping (optional; convergence is causal, Prop. global_convergence): the
// carry pass also finds the sequence's leading groups whose residual is below tol.  Those are
// frozen: the step there is taken as exactly zero, so the filter restarts after them from
// (m, P) = (0, 0), the next local pass copies each newly frozen group once into the other
// iterate buffer, and later passes skip it.
// lambda = 0 gives Gamma_t = I: the DEER step.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

constexpr int ED = 16;                 // state size
constexpr int ES = 17;                 // LDS row stride of a 16x16 matrix
constexpr int EM = ED * ES;            // floats per stored matrix
constexpr int EL = 16;                 // chunk length
constexpr int EGEL = 3 * ED * ED + 2 * ED;   // group element: A, C, J (row-major), b, eta
constexpr int ECAR = ED * ED + ED;           // filtered state: P (row-major), m

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

// G = M^-1 (16x16 in LDS) by Gauss-Jordan with partial pivoting, held in registers: lane l
// keeps row r = l & 15 of [M | I], columns 8q .. 8q + 7 (q = l >> 4).  Rows are not swapped:
// the pivot of column k is the unused row of largest |entry| (found by a rotate-and-max over
// each 16-lane row of the wave; ties and the last 4 mantissa bits go to the higher row), and
// the row that pivoted column k ends holding row k of the inverse in its right half.
PN_DEV void inv16(float* G, const float* M) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int c = 8 * q + j;
        a[j] = c < ED ? M[r * ES + c] : (c - ED == r ? 1.f : 0.f);
    }
    bool used = false;
    int myk = 0;
#pragma unroll 2
    for (int k = 0; k < ED; ++k) {
        const int kq = k >> 3, kc = k & 7;
        float ak = a[0];
#pragma unroll
        for (int j = 1; j < 8; ++j) ak = kc == j ? a[j] : ak;
        uint32_t key = used ? 0u
                            : ((max(__float_as_uint(fabsf(ak)), 0x10u) & ~0xFu) | (uint32_t)r);
        key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x121, 0xF, 0xF, false));
        key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x122, 0xF, 0xF, false));
        key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x124, 0xF, 0xF, false));
        key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x128, 0xF, 0xF, false));
        const int p = __builtin_amdgcn_readlane((int)key, 16 * kq) & 15;
        const float piv = __int_as_float(
            __builtin_amdgcn_readlane(__float_as_int(ak), 16 * kq + p));
        const float fk = __int_as_float(
            __builtin_amdgcn_ds_bpermute((r + 16 * kq) << 2, __float_as_int(ak)));
        float prow[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            prow[j] = __int_as_float(
                __builtin_amdgcn_ds_bpermute((16 * q + p) << 2, __float_as_int(a[j])));
        const float inv = 1.f / piv;
        const float g = -fk * inv;
        const bool me = r == p;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = me ? a[j] * inv : fmaf(g, prow[j], a[j]);
        if (me) { used = true; myk = k; }
    }
    if (q >= 2) {
#pragma unroll
        for (int j = 0; j < 8; ++j) G[myk * ES + 8 * (q - 2) + j] = a[j];
    }
    __syncthreads();
}

PN_DEV void store_mat(float* dst, const float* M) {       // LDS (stride ES) -> row-major
    const int l = threadIdx.x & 63;
    for (int w = l; w < ED * ED; w += 64) dst[w] = M[(w / ED) * ES + w % ED];
}
PN_DEV void fetch_mat(float* M, const float* src) {       // row-major -> LDS (stride ES)
    const int l = threadIdx.x & 63;
    for (int w = l; w < ED * ED; w += 64) M[(w / ED) * ES + w % ED] = src[w];
}

struct ElkArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];          // ping-pong iterates: s^(k) lives in sbuf[k & 1]
    const float* params;     // W (16x16) | U (16xDx) | b (16)
    float* gel;              // [ngroups][EGEL] group elements of this iteration
    const float* gcar;       // [ngroups][ECAR] filtered state entering every group (previous)
    Ctrl* ctrl;
    SeqState* seq;
    const TileInfo* tiles;   // by slot (chunks)
    const GroupInfo* groups;
    const int32_t* group_start;
    uint32_t* grmax;         // [ngroups] residual bound of every group's latest iterate (bits)
    int ngroups;
    int freeze;              // converged-prefix skipping
    float lam;
    int res64;               // nonzero: the stopping residual is evaluated in FP64
    int diag;                // nonzero: quasi-ELK, the LGSSM uses diag(A_t)
};

template <int DX>
__global__ void __launch_bounds__(64) elk_local_kernel(ElkArgs a) {
    constexpr int L = EL;
    constexpr int KT = ED + DX;
    constexpr int SS = ED + 4, XS = DX + 4;
    static_assert(KT % 4 == 0, "shape");
    __shared__ __attribute__((aligned(16))) float sst[(L + 1) * SS];
    __shared__ __attribute__((aligned(16))) float xst[L * XS];
    __shared__ float dsh[L * ED], rsh[L * ED];
    __shared__ float Wm[EM], Ai[EM], Ci[EM], Ji[EM], At[EM], Jj[EM], Gm[EM], T1[EM], T2[EM];
    __shared__ float Pr[EM];                  // replay: filtered covariance
    __shared__ float bi[ED], ei[ED], vx[ED], vy[ED], vz[ED], mr[ED];
    __shared__ int badrow[L + 1];

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k_it = a.ctrl->iter;
    const bool fuse = k_it > 0;
    const float reset_abs = a.ctrl->reset_abs;
    const float lam = a.lam;
    const float s1 = 1.f / (1.f + lam);           // 1 / (1 + lambda)
    const float kap = lam / (1.f + lam);         // kappa
    const float* __restrict__ sprev = a.sbuf[(k_it + 1) & 1];   // s^(k-1)
    float* __restrict__ scur = a.sbuf[k_it & 1];                 // s^(k)
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

    // residual, d_t of the staged rows (FP64 stopping residual when asked for)
    auto linearise = [&](bool first, int len, bool track) -> uint32_t {
        uint32_t rm = 0;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KT / 4; ++kb) {
            const int kk = 4 * kb + g;
            const float av = kk < ED ? sst[u * SS + kk] : xst[u * XS + (kk - ED)];
            acc = mfma16x4(av, blin[kb], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = 4 * g + i;
            const float f = tanhf_(acc[i] + bias_u);
            const float res = sst[(t + 1) * SS + u] - f;
            dsh[t * ED + u] = (first && t == 0) ? 0.f : 1.f - f * f;
            rsh[t * ED + u] = res;
            if (track && t < len && !a.res64) rm = max(rm, absbits(res));
        }
        if (track && a.res64) {
            // The stopping test in FP64: s, x and the parameters upcast, the quantity the final
            // FP64 residual reports.  The FP32 residual still drives the update; its rounding
            // (~1e-7 here) would otherwise let an iterate pass a 1e-6 test it fails in FP64.
            // The bound is rounded up to FP32.
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = 4 * g + i;
                if (t < len) {
                    double acc64 = (double)bias_u;
                    for (int kk = 0; kk < ED; ++kk)
                        acc64 += (double)Wm[u * ES + kk] * (double)sst[t * SS + kk];
                    for (int kk = 0; kk < DX; ++kk)
                        acc64 += (double)U[u * DX + kk] * (double)xst[t * XS + kk];
                    const double r = (double)sst[(t + 1) * SS + u] - tanh(acc64);
                    const double ar = fabs(r);
                    float fr = (float)ar;
                    if ((double)fr < ar) fr = nextafterf(fr, INFINITY);
                    rm = max(rm, (r == r) ? absbits(fr) : 0x7F800000u);
                }
            }
        }
        __syncthreads();
        return rm;
    };
    auto build_At = [&](int t) {
        for (int idx = l; idx < ED * ED; idx += 64) {
            const int r = idx / ED, c = idx % ED;
            At[r * ES + c] = (a.diag && r != c) ? 0.f : dsh[t * ED + r] * Wm[r * ES + c];
        }
        __syncthreads();
    };

    for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
        const GroupInfo gr = a.groups[gi];
        if (a.seq[gr.b].status != kActive) continue;
        const int b = gr.b;
        if (a.freeze) {
            const int gg = gi - a.group_start[b];
            if (gg < a.seq[b].frozen_prev) continue;            // frozen, both buffers hold it
            if (gg < a.seq[b].frozen) {                         // frozen by the last carry pass
                if (fuse) {
                    for (int kt = 0; kt < gr.ntl; ++kt) {
                        const TileInfo ti = a.tiles[gr.tile0 + kt];
                        for (int idx = l; idx < ti.len * (ED / 4); idx += 64) {
                            const size_t o = (size_t)ti.row0 * ED + 4 * idx;
                            *(float4*)(scur + o) = *(const float4*)(sprev + o);
                        }
                    }
                }
                continue;
            }
        }
        uint32_t rmax = 0;
        int nreset = 0;
        bool have = false;                       // the group's element holds at least one step
        if (fuse) {                              // filtered state entering the group
            const float* cr = a.gcar + (size_t)gi * ECAR;
            fetch_mat(Pr, cr);
            if (l < ED) mr[l] = cr[ED * ED + l];
        }
        for (int kt = 0; kt < gr.ntl; ++kt) {
            const TileInfo ti = a.tiles[gr.tile0 + kt];
            const int len = ti.len;
            const int64_t row0 = ti.row0;
            const bool first = (ti.flags & kTileTimeFirst) != 0;
            __syncthreads();
            // ---- stage s_{t-1}, s_t (of s^(k-1), or the guess s^(0)) and x_t
            const float* src = fuse ? sprev : scur;
            for (int idx = l; idx < (L + 1) * (ED / 4); idx += 64) {
                const int r = idx / (ED / 4), c4 = idx % (ED / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r == 0) v = first ? *(const float4*)(a.s0 + (size_t)b * ED + 4 * c4)
                                      : *(const float4*)(src + (size_t)(row0 - 1) * ED + 4 * c4);
                else if (r - 1 < len) v = *(const float4*)(src + (size_t)(row0 + r - 1) * ED + 4 * c4);
                *(float4*)(sst + r * SS + 4 * c4) = v;
            }
            for (int idx = l; idx < L * (DX / 4); idx += 64) {
                const int r = idx / (DX / 4), c4 = idx % (DX / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
                *(float4*)(xst + r * XS + 4 * c4) = v;
            }
            if (l <= L) badrow[l] = 0;
            __syncthreads();

            if (fuse) {
                // ---- the previous iteration's step: the exact filter from the entering (m, P)
                linearise(first, len, false);
                float hv = 0.f;
                if (!first && l < ED) {
                    hv = sst[l] + mr[l];               // s^(k) of the row before the chunk
                    if (!(fabsf(hv) <= reset_abs)) badrow[0] = 1;
                }
                for (int t = 0; t < len; ++t) {
                    build_At(t);
                    mm16(T1, At, false, Pr, false, 1.f, nullptr, 0.f);        // A P
                    mm16(T2, T1, false, At, true, 1.f, nullptr, 1.f);         // P- = A P A^T + I
                    for (int idx = l; idx < ED * ED; idx += 64) {
                        const int r = idx / ED, c = idx % ED;
                        Jj[r * ES + c] = lam * T2[r * ES + c] + (r == c ? 1.f : 0.f);
                    }
                    __syncthreads();
                    inv16(Gm, Jj);                                  // Gamma
                    mm16(Pr, Gm, false, T2, false, 1.f, nullptr, 0.f);        // P = Gamma P-
                    for (int idx = l; idx < ED * ED; idx += 64) {              // symmetrise
                        const int r = idx / ED, c = idx % ED;
                        if (r < c) {
                            const float v = 0.5f * (Pr[r * ES + c] + Pr[c * ES + r]);
                            Pr[r * ES + c] = v;
                            Pr[c * ES + r] = v;
                        }
                    }
                    if (l < ED) vx[l] = -rsh[t * ED + l];
                    __syncthreads();
                    mv16(vy, At, false, mr, 1.f, vx, 1.f);                    // A m - r
                    mv16(mr, Gm, false, vy, 1.f, nullptr, 0.f);               // m = Gamma (.)
                    const float v = l < ED ? sst[(t + 1) * SS + l] + mr[l] : 0.f;
                    const bool rb = __any(l < ED && !(fabsf(v) <= reset_abs));
                    if (l < ED) sst[(t + 1) * SS + l] = rb ? 0.f : v;
                    nreset += rb ? 1 : 0;
                    __syncthreads();
                }
                if (!first && l < ED) sst[l] = badrow[0] ? 0.f : hv;
                __syncthreads();
                for (int idx = l; idx < len * (ED / 4); idx += 64) {
                    const int r = idx / (ED / 4), c4 = idx % (ED / 4);
                    *(float4*)(scur + (size_t)(row0 + r) * ED + 4 * c4) =
                        *(const float4*)(sst + (r + 1) * SS + 4 * c4);
                }
            }

            // ---- linearise at s^(k), then fold the chunk's leaves into the group's element
            rmax = max(rmax, linearise(first, len, true));
            for (int t = 0; t < len; ++t) {
                build_At(t);
                if (l < ED) vx[l] = rsh[t * ED + l];
                __syncthreads();
                if (!have) {
                    // leaf (A/(1+lambda), -r/(1+lambda), I/(1+lambda), kappa A^T r, kappa A^T A);
                    // at a sequence head A = 0, which folds in the prior Delta_0 = 0
                    for (int idx = l; idx < ED * ED; idx += 64) {
                        const int r = idx / ED, c = idx % ED;
                        Ai[r * ES + c] = s1 * At[r * ES + c];
                        Ci[r * ES + c] = (r == c) ? s1 : 0.f;
                    }
                    if (l < ED) bi[l] = -s1 * vx[l];
                    __syncthreads();
                    mv16(ei, At, true, vx, kap, nullptr, 0.f);            // eta = kappa A^T r
                    mm16(Ji, At, true, At, false, kap, nullptr, 0.f);     // J = kappa A^T A
                    have = true;
                    continue;
                }
                mm16(Jj, At, true, At, false, kap, nullptr, 0.f);     // J_j
                mv16(vy, At, true, vx, kap, nullptr, 0.f);            // eta_j
                mm16(T1, Ci, false, Jj, false, 1.f, nullptr, 1.f);    // I + C_i J_j
                inv16(Gm, T1);                              // G
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
        }
        // ---- the group's element
        float* ge = a.gel + (size_t)gi * EGEL;
        store_mat(ge, Ai);
        store_mat(ge + ED * ED, Ci);
        store_mat(ge + 2 * ED * ED, Ji);
        if (l < ED) {
            ge[3 * ED * ED + l] = bi[l];
            ge[3 * ED * ED + ED + l] = ei[l];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) {
            a.grmax[gi] = rmax;
            atomicMax(&a.seq[b].maxr, rmax);
            if (nreset) atomicAdd(&a.seq[b].resets_pending, nreset);
        }
    }
}

// ---- carry pass: the filtered state entering every group ------------------------------------
// One single-wave workgroup per sequence: (m, P) = (0, 0) before the first group; a group's
// element maps it on by  G = (I + P J)^-1,  m' = A G (m + P eta) + b,  P' = A G P A^T + C.
// The next group's element is fetched into registers while the current one is applied.
__global__ void __launch_bounds__(64) elk_carry_kernel(const float* __restrict__ gel,
                                                       float* __restrict__ gcar,
                                                       const Ctrl* ctrl, SeqState* seq,
                                                       const int32_t* group_start,
                                                       const uint32_t* grmax, int freeze,
                                                       int B) {
    __shared__ float Ae[EM], Ce[EM], Je[EM], P[EM], T1[EM], Gm[EM];
    __shared__ float be[ED], ee[ED], m[ED], vz[ED];
    if (ld_i32(&ctrl->all_done)) return;
    const int b = blockIdx.x;
    if (b >= B || seq[b].status != kActive) return;
    const int l = threadIdx.x;
    const int g0 = group_start[b], G = group_start[b + 1] - g0;
    int gstart = 0;                      // first group the step is taken on
    if (freeze) {
        // leading groups whose residual bound is below tol (NaN bounds are not)
        const uint32_t tolb = __float_as_uint(ctrl->tol);
        int fz = G;
        for (int base = 0; base < G; base += 64) {
            const bool open = base + l < G && !(grmax[g0 + base + l] < tolb);
            const uint64_t m = __ballot(open);
            if (m) {
                fz = base + __ffsll((unsigned long long)m) - 1;
                break;
            }
        }
        const int old = seq[b].frozen;
        gstart = max(fz, old);
        __syncthreads();
        if (l == 0) {
            seq[b].frozen_prev = old;
            seq[b].frozen = gstart;
        }
    }
    constexpr int PER = (EGEL + 63) / 64;
    float nxt[PER];
    auto prefetch = [&](int gg) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int w = l + 64 * i;
            nxt[i] = (gg < G && w < EGEL) ? gel[(size_t)(g0 + gg) * EGEL + w] : 0.f;
        }
    };
    for (int idx = l; idx < EM; idx += 64) P[idx] = 0.f;
    if (l < ED) m[l] = 0.f;
    prefetch(gstart);
    __syncthreads();
    for (int gg = gstart; gg < G; ++gg) {
        // carry into group gg
        float* cr = gcar + (size_t)(g0 + gg) * ECAR;
        store_mat(cr, P);
        if (l < ED) cr[ED * ED + l] = m[l];
        // this group's element into LDS, the next one into registers
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int w = l + 64 * i;
            if (w < 3 * ED * ED) {
                float* M = w < ED * ED ? Ae : (w < 2 * ED * ED ? Ce : Je);
                const int v = w % (ED * ED);
                M[(v / ED) * ES + v % ED] = nxt[i];
            } else if (w < 3 * ED * ED + ED) {
                be[w - 3 * ED * ED] = nxt[i];
            } else if (w < EGEL) {
                ee[w - 3 * ED * ED - ED] = nxt[i];
            }
        }
        prefetch(gg + 1);
        __syncthreads();
        mm16(T1, P, false, Je, false, 1.f, nullptr, 1.f);     // I + P J
        inv16(Gm, T1);                              // G
        mm16(T1, Ae, false, Gm, false, 1.f, nullptr, 0.f);    // A G
        mv16(vz, P, false, ee, 1.f, m, 1.f);                  // m + P eta
        mv16(m, T1, false, vz, 1.f, be, 1.f);                 // m' = A G (.) + b
        mm16(Gm, T1, false, P, false, 1.f, nullptr, 0.f);     // A G P
        mm16(P, Gm, false, Ae, true, 1.f, Ce, 0.f);           // P' = (.) A^T + C
    }
}

// ---- host ---------------------------------------------------------------------------------------

struct ElkLayout {
    IterState st;
    float* salt;
    float* gel;
    float* gcar;
    uint32_t* grmax;
    char* r64;
    size_t bytes;
};

static ElkLayout elk_layout(void* ws, const HostBatch& hb, int ntiles, int ngroups) {
    Carver c(ws);
    ElkLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles, ngroups);
    lay.salt = c.take<float>((size_t)hb.N * ED);
    lay.gel = c.take<float>((size_t)std::max(ngroups, 1) * EGEL);
    lay.gcar = c.take<float>((size_t)std::max(ngroups, 1) * ECAR);
    lay.grmax = c.take<uint32_t>((size_t)std::max(ngroups, 1));
    lay.r64 = c.take<char>(residual64_workspace(PN_CELL_TANH, ED, 16, hb));   // FP64 residual
    lay.bytes = c.bytes();
    return lay;
}

bool elk_supported(int D, int Dx) { return D == ED && Dx == 16; }

static int elk_resident() {
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)elk_local_kernel<16>, 64, 0) !=
            hipSuccess || occ < 1)
        occ = 1;
    return cu_count() * occ;
}

// Chunks per group.  An explicit tile (a multiple of 16 steps) fixes it.  Otherwise a cost
// model picks it: the local pass takes rounds * gt chunks of latency (rounds = groups per
// resident workgroup), the carry pass one element application per group of the longest
// sequence; a chunk of the local pass (replay and fold) costs about kLocalPerCarry carry steps.
static int elk_group_tiles(const HostBatch& hb, const std::vector<int32_t>& ts, int tile) {
    if (tile > 0) return tile / EL;
    constexpr double kLocalPerCarry = 36.0;
    const int resident = elk_resident();
    int maxc = 0;
    for (int b = 0; b < hb.B; ++b) maxc = std::max(maxc, ts[b + 1] - ts[b]);
    int best = 1;
    double best_cost = 1e300;
    for (int gt = 1; gt <= 64; gt *= 2) {
        const int ng = count_groups(ts, hb.B, gt);
        const double rounds = std::ceil((double)ng / resident);
        const double cost = rounds * gt * kLocalPerCarry + std::ceil((double)maxc / gt);
        if (cost < best_cost) { best_cost = cost; best = gt; }
    }
    return best;
}

size_t elk_workspace(int, int, const HostBatch& hb, const pn_opts& o) {
    const std::vector<int32_t> ts = tile_starts(hb, EL);
    const int gt = elk_group_tiles(hb, ts, o.tile);
    return elk_layout(nullptr, hb, ts[hb.B], count_groups(ts, hb.B, gt)).bytes;
}

pn_status residual64_device(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                            const float* s0, const float* s, void* ws, hipStream_t stream,
                            double* max_resid);

pn_status elk_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                      const float* s0, float* s, double lambda, const pn_opts& o, void* ws,
                      hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    void (*kern)(ElkArgs) = elk_local_kernel<16>;
    const std::vector<int32_t> ts = tile_starts(hb, EL);
    const int ntiles = ts[hb.B];
    const int resident = elk_resident();
    const int gt = elk_group_tiles(hb, ts, o.tile);
    const int ngroups = count_groups(ts, hb.B, gt);
    ElkLayout lay = elk_layout(ws, hb, ntiles, ngroups);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, EL, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream, gt));
    const int grid = std::max(1, std::min(ngroups, resident));
    ElkArgs args;
    args.x = x;
    args.s0 = s0;
    args.sbuf[0] = s;
    args.sbuf[1] = lay.salt;
    args.params = (const float*)cd.params;
    args.gel = lay.gel;
    args.gcar = lay.gcar;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.tiles = lay.st.tiles;
    args.groups = lay.st.groups;
    args.group_start = lay.st.group_start;
    args.grmax = lay.grmax;
    args.ngroups = ngroups;
    args.freeze = o.freeze_prefix ? 1 : 0;
    args.lam = (float)lambda;
    args.res64 = o.fp64_final_residual ? 1 : 0;
    args.diag = o.jac == PN_JAC_DIAG ? 1 : 0;
    auto one_iter = [&](hipStream_t st) {
        prof_launch("elk_local", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, s2, args);
        });
        prof_launch("elk_carry", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(elk_carry_kernel, dim3(std::max(1, hb.B)), dim3(64), 0, s2,
                               (const float*)lay.gel, lay.gcar, (const Ctrl*)lay.st.ctrl,
                               lay.st.seq, (const int32_t*)lay.st.group_start,
                               (const uint32_t*)lay.grmax, args.freeze, hb.B);
        });
        launch_decide(lay.st, hb.B, st, true);
    };
    std::vector<uintptr_t> key = {0x454Du, (uintptr_t)kern, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)cd.params,
                                  (uintptr_t)ws, (uintptr_t)hb.B, (uintptr_t)ntiles,
                                  (uintptr_t)ngroups, float_bits(args.lam),
                                  (uintptr_t)args.res64, (uintptr_t)args.diag,
                                  (uintptr_t)args.freeze};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    int derr = 0;
    PN_TRY(finish_iterations(lay.st, hb, ED, sizeof(float), s, lay.salt, stream, info, all_conv,
                             &derr));
    if (derr) {
        set_error("device-side check failed in the ELK iteration");
        return PN_ERR_INTERNAL;
    }
    if (o.fp64_final_residual && info) {
        // the reported residual is the FP64 one of the returned iterate
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
