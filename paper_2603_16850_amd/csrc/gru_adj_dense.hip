// Exact adjoint of the GRU recurrence as one reverse dense scan (the DEER backward pass).
//
// Ch. 3 ("Training and the backwards pass"): once the forward iteration has converged, the
// Jacobians A_t at the solution are exact, and the reverse-time linear recurrence
//   lambda_t = g_t + A_{t+1}^T lambda_{t+1},   lambda_T = g_T,
// is a linear dynamical system with transitions A_{t+1}^T that one parallel scan solves.  The
// scan here is the work-efficient two-level form, written in the carried vector
// w_t = A_t^T lambda_t (so that lambda_t = g_t + w_{t+1}):
//
//   1. chain pass, zero carry: every group of consecutive steps (taken from the sequence end)
//      walks its steps with w_in = 0, giving the affine part v_q of the group's map;
//   2. map pass: the linear part M_q = A_lo^T A_{lo+1}^T ... A_hi^T of the group's map, a chain
//      of dense D x D products on MFMA (BF16 operands or FP32, FP32 accumulation), A_t^T
//      rebuilt per step from the gate values;
//   3. carry walk: w into the first (latest) group is 0; w into group q+1 is M_q w_q + v_q;
//   4. chain pass from the carries: lambda_t = g_t + w exactly in FP32 inside every group.
//
// Inside a group the result is the sequential recurrence itself; across groups it is exact up
// to the products' rounding.  The residual of the recurrence,
// rho_t = lambda_t - g_t - A_{t+1}^T lambda_{t+1}, vanishes (to FP32 rounding) except at the
// group boundaries, where it equals the difference R_q between the vector the chain of group q
// handed on and the carry group q+1 started from.  If max |R_q| > tol * max(1, max |g|) the
// carries are refined by the same walk over the maps with R in place of v (the residual
// always exact, the maps possibly BF16: an iterative refinement, as the forward Newton
// iteration refines itself) and pass 4 runs again for the sequences still open.
//
// The VJP of one step, with the gate values (alpha, beta, gamma, z) of step t,
//   A_t^T u = z (.) u + U_z^T (alpha (.) u) + U_n^T (beta (.) u) + U_r^T (gamma (.) u),
// is a (D x 3D)(3D x n) product: n = 16 groups side by side in the chain passes (FP32 MFMA),
// n = D columns of one group's M in the map pass.
#include <algorithm>

#include "gru_common.hpp"
#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));


struct DenseAdjArgs {
    const float* gates;        // [N][4][D]: alpha, beta, gamma, z
    const float* gs;           // [N][D] g_t
    const float* U;            // [U_z; U_r; U_n] (3D x D), row-major
    float* lam;                // [N][D] output
    const TileInfo* tiles;     // by scan slot
    const GroupInfo* groups;   // by group slot (a sequence's groups from its end)
    const int32_t* group_start;
    int ngroups;
    float* mbuf;               // [ngroups][D][D] M_q, row-major
    float* vbuf;               // [ngroups][D] v_q (chain with zero carry)
    float* wcar;               // [ngroups][D] carry into each group
    float* wout;               // [ngroups][D] vector each group's chain hands on
    int* done;                 // [B] 1 once the sequence passed the residual test
    int* nopen;                // sequences left open by the last check
    const float* gmax;         // [B] max |g| per sequence
    SeqState* seq;
    float tol;
};

// rows [row_lo, row_hi] of group slot gi
PN_DEV void dense_group_rows(const DenseAdjArgs& a, int gi, int64_t& row_hi, int& len, int& b) {
    const GroupInfo gr = a.groups[gi];
    const TileInfo t0 = a.tiles[gr.tile0];                  // latest tile of the group
    const TileInfo t1 = a.tiles[gr.tile0 + gr.ntl - 1];     // earliest
    row_hi = t0.row0 + t0.len - 1;
    len = (int)(row_hi - t1.row0 + 1);
    b = gr.b;
}

// ---- chain pass ---------------------------------------------------------------------------
// One wave walks 16 groups side by side (lane l works on group column c = l % 16).  In the
// MFMA 16x16x4 layout the lane holds, for its column, the rows 4g + r + 16 bi of the carried
// vector (g = l / 16, r = 0..3, bi = 0..D/16-1).  The K index of the VJP product (3D long: the
// alpha, beta, gamma terms) is permuted so that at K step s each lane group supplies a row it
// already holds: slot s <-> matrix s / (D/4), row 4g + (s % 4) + 16 ((s % (D/4)) / 4).  The
// product's output rows are then again the lane's own rows, and no transpose is needed
// between steps.  The A operands (the transposed U blocks in that order) sit in LDS, one
// float4 (four K steps) per lane and read.
template <int D>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(D <= 48 ? 2 : 1)))
gru_adj_dchain_kernel(DenseAdjArgs a) {
    constexpr int NB = D / 16, KQ = D / 4, NS = 3 * KQ, NQ = NS / 4;
    static_assert(D % 16 == 0, "D multiple of 16");
    __shared__ __attribute__((aligned(16))) float4 ua[NB * NQ * 64];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
    for (int e = tid; e < NB * NQ * 64; e += 256) {
        const int el = e & 63, sq = (e >> 6) % NQ, bo = (e >> 6) / NQ;
        const int eg = el >> 4, i = (el & 15) + 16 * bo;
        const int s0 = 4 * sq, m = s0 / KQ, kb = (s0 % KQ) / 4;
        const int blk = m == 0 ? 0 : (m == 1 ? 2 : 1);       // alpha-U_z, beta-U_n, gamma-U_r
        float4 v;
        v.x = a.U[(size_t)(blk * D + 4 * eg + 0 + 16 * kb) * D + i];
        v.y = a.U[(size_t)(blk * D + 4 * eg + 1 + 16 * kb) * D + i];
        v.z = a.U[(size_t)(blk * D + 4 * eg + 2 + 16 * kb) * D + i];
        v.w = a.U[(size_t)(blk * D + 4 * eg + 3 + 16 * kb) * D + i];
        ua[e] = v;
    }
    __syncthreads();
    const int gi = (blockIdx.x * 4 + w) * 16 + c;
    int64_t row_hi = 0;
    int len = 0, b = 0;
    if (gi < a.ngroups) {
        dense_group_rows(a, gi, row_hi, len, b);
        if (a.done[b]) len = 0;
    }
    int nsteps = len;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) nsteps = max(nsteps, __shfl_xor(nsteps, off));
    if (nsteps == 0) return;
    float x[NB][4];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (len > 0) v = *(const float4*)(a.wcar + (size_t)gi * D + 16 * bi + 4 * g);
        x[bi][0] = v.x;
        x[bi][1] = v.y;
        x[bi][2] = v.z;
        x[bi][3] = v.w;
    }
    // operands of step st: g_t and the gate values of this lane's rows
    float4 gv[NB], ga[4][NB];
    auto fetch = [&](int st) {
        const int64_t row = row_hi - min(st, max(len - 1, 0));
        const float* gp = a.gs + (size_t)row * D + 4 * g;
        const float* gr = a.gates + (size_t)row * 4 * D + 4 * g;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            gv[bi] = *(const float4*)(gp + 16 * bi);
#pragma unroll
            for (int m = 0; m < 4; ++m) ga[m][bi] = *(const float4*)(gr + m * D + 16 * bi);
        }
    };
    fetch(0);
    for (int st = 0; st < nsteps; ++st) {
        const bool act = st < len;
        float lm[NB][4], bop[NS];
        floatx4 acc[NB];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            lm[bi][0] = gv[bi].x + x[bi][0];
            lm[bi][1] = gv[bi].y + x[bi][1];
            lm[bi][2] = gv[bi].z + x[bi][2];
            lm[bi][3] = gv[bi].w + x[bi][3];
            acc[bi][0] = ga[3][bi].x * lm[bi][0];
            acc[bi][1] = ga[3][bi].y * lm[bi][1];
            acc[bi][2] = ga[3][bi].z * lm[bi][2];
            acc[bi][3] = ga[3][bi].w * lm[bi][3];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int m = s / KQ, kb = (s % KQ) / 4, r = s % 4;
            const float4 q = ga[m][kb];
            const float wv = r == 0 ? q.x : (r == 1 ? q.y : (r == 2 ? q.z : q.w));
            bop[s] = wv * lm[kb][r];
        }
        if (act) {
            float* lp = a.lam + (size_t)(row_hi - st) * D + 4 * g;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
                *(float4*)(lp + 16 * bi) = make_float4(lm[bi][0], lm[bi][1], lm[bi][2], lm[bi][3]);
        }
        fetch(st + 1);                          // in flight during the products (rows clamped)
#pragma unroll
        for (int sq = 0; sq < NQ; ++sq) {
            float4 av[NB];
#pragma unroll
            for (int bo = 0; bo < NB; ++bo) av[bo] = ua[(bo * NQ + sq) * 64 + l];
#pragma unroll
            for (int bo = 0; bo < NB; ++bo) {
                acc[bo] = mfma16x4(av[bo].x, bop[4 * sq + 0], acc[bo]);
                acc[bo] = mfma16x4(av[bo].y, bop[4 * sq + 1], acc[bo]);
                acc[bo] = mfma16x4(av[bo].z, bop[4 * sq + 2], acc[bo]);
                acc[bo] = mfma16x4(av[bo].w, bop[4 * sq + 3], acc[bo]);
            }
        }
        if (act) {
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int r = 0; r < 4; ++r) x[bi][r] = acc[bi][r];
        }
    }
    if (len > 0) {
        float* op = a.wout + (size_t)gi * D + 4 * g;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
            *(float4*)(op + 16 * bi) = make_float4(x[bi][0], x[bi][1], x[bi][2], x[bi][3]);
    }
}

// ---- map pass -----------------------------------------------------------------------------
// One wave per group composes M <- A_t^T M over the group's steps (latest first), M held in
// the MFMA C layout: lane (c, g) holds M[4g + r + 16 bi][c + 16 cb].  The lane builds the
// entries J[i][k] = A_t^T[i][k] = U_z[k][i] alpha_k + U_n[k][i] beta_k + U_r[k][i] gamma_k
// (+ z_k on the diagonal) for i = c + 16 bo and the rows k = 4g + r + 16 kb it holds of M,
// which is the K order of the product: at K chunk kk the lane group's slots are the rows of
// blocks 2kk and 2kk + 1 (BF16 16x16x32) or, one K step at a time, of every block (FP32
// 16x16x4), for J and M alike.
template <int D, bool BF16>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(D <= 48 ? 2 : 1)))
gru_adj_dmap_kernel(DenseAdjArgs a) {
    constexpr int NB = D / 16, NKK = (NB + 1) / 2;
    constexpr bool UREG = D <= 32;                 // U entries in registers (else from LDS)
    __shared__ __attribute__((aligned(16))) float4 uj[UREG ? 1 : 3 * NB * NB * 64];
    __shared__ __attribute__((aligned(16))) float vsh[4 * D];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
    auto uval = [&](int m, int bo, int kb) {      // U_m[4g + r + 16kb][c + 16bo], r = 0..3
        const int blk = m == 0 ? 0 : (m == 1 ? 2 : 1);
        const int i = c + 16 * bo, k0 = 4 * g + 16 * kb;
        float4 v;
        v.x = a.U[(size_t)(blk * D + k0 + 0) * D + i];
        v.y = a.U[(size_t)(blk * D + k0 + 1) * D + i];
        v.z = a.U[(size_t)(blk * D + k0 + 2) * D + i];
        v.w = a.U[(size_t)(blk * D + k0 + 3) * D + i];
        return v;
    };
    float4 ur[3][UREG ? NB : 1][UREG ? NB : 1];
    if constexpr (UREG) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int bo = 0; bo < NB; ++bo)
#pragma unroll
                for (int kb = 0; kb < NB; ++kb) ur[m][bo][kb] = uval(m, bo, kb);
    } else {
        for (int e = tid; e < 3 * NB * NB * 64; e += 256) {
            const int el = e & 63, kb = (e >> 6) % NB, bo = ((e >> 6) / NB) % NB,
                      m = (e >> 6) / (NB * NB);
            const int blk = m == 0 ? 0 : (m == 1 ? 2 : 1);
            const int i = (el & 15) + 16 * bo, k0 = 4 * (el >> 4) + 16 * kb;
            float4 v;
            v.x = a.U[(size_t)(blk * D + k0 + 0) * D + i];
            v.y = a.U[(size_t)(blk * D + k0 + 1) * D + i];
            v.z = a.U[(size_t)(blk * D + k0 + 2) * D + i];
            v.w = a.U[(size_t)(blk * D + k0 + 3) * D + i];
            uj[e] = v;
        }
        __syncthreads();
    }
    auto uget = [&](int m, int bo, int kb) -> float4 {
        if constexpr (UREG) return ur[m][bo][kb];
        else {                                   // re-read every step (kept out of registers)
            const volatile float4* p = uj + ((m * NB + bo) * NB + kb) * 64 + l;
            float4 v;
            v.x = p->x;
            v.y = p->y;
            v.z = p->z;
            v.w = p->w;
            return v;
        }
    };
    const int gi = blockIdx.x * 4 + w;
    if (gi >= a.ngroups) return;
    int64_t row_hi;
    int len, b;
    dense_group_rows(a, gi, row_hi, len, b);
    floatx4 M[NB][NB], Mn[NB][NB];
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) M[bi][cb][r] = (bi == cb && 4 * g + r == c) ? 1.f : 0.f;
    float4 ga[4][NB], gv[NB];
    auto fetch = [&](int st) {
        const float* gr = a.gates + (size_t)(row_hi - st) * 4 * D + 4 * g;
        const float* gp = a.gs + (size_t)(row_hi - st) * D + 4 * g;
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
#pragma unroll
            for (int m = 0; m < 4; ++m) ga[m][kb] = *(const float4*)(gr + m * D + 16 * kb);
            gv[kb] = *(const float4*)(gp + 16 * kb);
        }
    };
    // The affine part v of the map rides along in FP32 on the VALU: w <- A_t^T (g_t + w), w
    // held like M's rows (rows 4g + r + 16 kb); the U terms are the FP32 entries of J summed
    // over the lane's k and then over the four lane groups, handed back to the row layout
    // through LDS.
    float wv[NB][4];
#pragma unroll
    for (int kb = 0; kb < NB; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) wv[kb][r] = 0.f;
    float* vs = vsh + w * D;
    auto jrow = [&](int bo, float (&J)[NB][4]) {     // J[kb][r] = U terms of A_t^T[c + 16bo][k]
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            const float4 u0 = uget(0, bo, kb), u1 = uget(1, bo, kb), u2 = uget(2, bo, kb);
            const float4 al = ga[0][kb], be = ga[1][kb], gm = ga[2][kb];
            J[kb][0] = fmaf(u2.x, gm.x, fmaf(u1.x, be.x, u0.x * al.x));
            J[kb][1] = fmaf(u2.y, gm.y, fmaf(u1.y, be.y, u0.y * al.y));
            J[kb][2] = fmaf(u2.z, gm.z, fmaf(u1.z, be.z, u0.z * al.z));
            J[kb][3] = fmaf(u2.w, gm.w, fmaf(u1.w, be.w, u0.w * al.w));
        }
    };
    // Mo = A_t^T Mi.  The z_i M[i][.] term is the accumulator's start value (exact FP32, the
    // lane's own entries); the products carry the U terms only.
    auto step = [&](const floatx4 (&Mi)[NB][NB], floatx4 (&Mo)[NB][NB], int st) {
        float lm[NB][4], zl[NB][4], p[NB];
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            const float4 z = ga[3][kb];
            lm[kb][0] = gv[kb].x + wv[kb][0];
            lm[kb][1] = gv[kb].y + wv[kb][1];
            lm[kb][2] = gv[kb].z + wv[kb][2];
            lm[kb][3] = gv[kb].w + wv[kb][3];
            zl[kb][0] = z.x * lm[kb][0];
            zl[kb][1] = z.y * lm[kb][1];
            zl[kb][2] = z.z * lm[kb][2];
            zl[kb][3] = z.w * lm[kb][3];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                Mo[kb][cb][0] = z.x * Mi[kb][cb][0];
                Mo[kb][cb][1] = z.y * Mi[kb][cb][1];
                Mo[kb][cb][2] = z.z * Mi[kb][cb][2];
                Mo[kb][cb][3] = z.w * Mi[kb][cb][3];
            }
        }
        if constexpr (BF16) {
            bf16x8 Ab[NB][NKK], Bb[NKK][NB];
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk)
#pragma unroll
                for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int kb = 2 * kk + (j >> 2);
                        Bb[kk][cb][j] = kb < NB ? (__bf16)Mi[kb][cb][j & 3] : (__bf16)0.f;
                    }
            // one output row block at a time: its U entries, its row of J, its BF16 operands
            // (the empty asm keeps the compiler from loading every block's U entries at once)
#pragma unroll
            for (int bo = 0; bo < NB; ++bo) {
                float J[NB][4];
                jrow(bo, J);
                float pp = 0.f;
#pragma unroll
                for (int kb = 0; kb < NB; ++kb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) pp = fmaf(J[kb][r], lm[kb][r], pp);
                p[bo] = pp;
#pragma unroll
                for (int kk = 0; kk < NKK; ++kk)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int kb = 2 * kk + (j >> 2);
                        Ab[bo][kk][j] = kb < NB ? (__bf16)J[kb][j & 3] : (__bf16)0.f;
                    }
                asm volatile("" ::: "memory");
            }
            fetch(min(st + 1, len - 1));             // in flight during the products
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk)
#pragma unroll
                for (int bo = 0; bo < NB; ++bo)
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb)
                        Mo[bo][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ab[bo][kk], Bb[kk][cb],
                                                                             Mo[bo][cb], 0, 0, 0);
        } else {
#pragma unroll
            for (int bo = 0; bo < NB; ++bo) {
                float J[NB][4];
                jrow(bo, J);
                float pp = 0.f;
#pragma unroll
                for (int kb = 0; kb < NB; ++kb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) pp = fmaf(J[kb][r], lm[kb][r], pp);
                p[bo] = pp;
#pragma unroll
                for (int kb = 0; kb < NB; ++kb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int cb = 0; cb < NB; ++cb)
                            Mo[bo][cb] = mfma16x4(J[kb][r], Mi[kb][cb][r], Mo[bo][cb]);
                asm volatile("" ::: "memory");
            }
            fetch(min(st + 1, len - 1));
        }
        // U terms of row c + 16 bo summed over the four lane groups, then to the row layout
#pragma unroll
        for (int bo = 0; bo < NB; ++bo) p[bo] = sum_halves(sum_rows16(p[bo]));
        if (g == 0) {
#pragma unroll
            for (int bo = 0; bo < NB; ++bo) vs[c + 16 * bo] = p[bo];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
            const float4 q = *(const float4*)(vs + 16 * kb + 4 * g);
            wv[kb][0] = zl[kb][0] + q.x;
            wv[kb][1] = zl[kb][1] + q.y;
            wv[kb][2] = zl[kb][2] + q.z;
            wv[kb][3] = zl[kb][3] + q.w;
        }
        __builtin_amdgcn_wave_barrier();
    };
    fetch(0);
    for (int st = 0; st < len; ++st) {              // (the last step's prefetch re-reads)
        step(M, Mn, st);
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) M[bi][cb] = Mn[bi][cb];
    }
    if (c == 0) {
        float* vp = a.vbuf + (size_t)gi * D + 4 * g;
#pragma unroll
        for (int kb = 0; kb < NB; ++kb)
            *(float4*)(vp + 16 * kb) = make_float4(wv[kb][0], wv[kb][1], wv[kb][2], wv[kb][3]);
    }
    float* mp = a.mbuf + (size_t)gi * D * D;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) mp[(size_t)(4 * g + r + 16 * bi) * D + c + 16 * cb] = M[bi][cb][r];
}

// ---- carry walk and residual check (one wave per sequence) ----------------------------------
// CHECK = false: w_0 = 0, w_{q+1} = M_q w_q + v_q into wcar.
// CHECK = true:  R_q = wout_q - wcar_{q+1}; the sequence passes if max |R| <= tol max(1, max|g|)
// (NaN never passes); otherwise delta_0 = 0, delta_{q+1} = M_q delta_q + R_q, wcar += delta.
// Lane i owns row i: y_i = sum_k M_q[i][k] u_k with u broadcast from LDS.  The walk is a chain
// of dependent mat-vecs, so each lane keeps its rows of the next PF maps in flight.
template <int D, bool CHECK>
__global__ void __launch_bounds__(64) gru_adj_dcarry_kernel(DenseAdjArgs a, int pass, int last) {
    constexpr int Q = D / 4, PF = D <= 48 ? 4 : 3;
    __shared__ __attribute__((aligned(16))) float ush[D];
    const int b = blockIdx.x, i = threadIdx.x;
    const bool act = i < D;
    const int ii = act ? i : 0;
    const int g0 = a.group_start[b], G = a.group_start[b + 1] - g0;
    if (CHECK) {
        if (a.done[b]) return;
        uint32_t mr = 0;
        const float* wo = a.wout + (size_t)g0 * D;
        const float* wc = a.wcar + (size_t)(g0 + 1) * D;
        const int ne = G > 1 ? (G - 1) * D : 0;
#pragma unroll 4
        for (int e = i; e < ne; e += 64) mr = max(mr, absbits(wo[e] - wc[e]));
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mr = max(mr, (uint32_t)__shfl_xor((int)mr, off));
        const float gm = __uint_as_float(((const uint32_t*)a.gmax)[b]);
        const float lim = a.tol * fmaxf(1.f, gm);
        const bool ok = mr <= __float_as_uint(lim) && !(gm != gm);
        if (ok || last) {
            if (i == 0) {
                a.seq[b].status = ok ? kConverged : kCapped;
                a.seq[b].iters = pass;
                a.seq[b].final_resid = __uint_as_float(mr);
                if (ok) a.done[b] = 1;
            }
            return;
        }
        if (i == 0) atomicAdd(a.nopen, 1);
    } else if (G > 0 && act) {
        a.wcar[(size_t)g0 * D + i] = 0.f;
    }
    const int nq = G - 1;                          // maps applied
    if (nq <= 0) return;
    float4 ring[PF][Q];
    float radd[PF];                                // v_q (walk) or R_q (check) of the ring's maps
    auto fetch = [&](int q, int j) {
        const float* mp = a.mbuf + (size_t)(g0 + q) * D * D + (size_t)ii * D;
#pragma unroll
        for (int k = 0; k < Q; ++k) ring[j][k] = *(const float4*)(mp + 4 * k);
        radd[j] = CHECK ? a.wout[(size_t)(g0 + q) * D + ii] - a.wcar[(size_t)(g0 + q + 1) * D + ii]
                        : a.vbuf[(size_t)(g0 + q) * D + ii];
    };
    // every load unconditional (clamped to the last map) so that the waits the compiler
    // places keep PF maps in flight
#pragma unroll
    for (int j = 0; j < PF; ++j) fetch(min(j, nq - 1), j);
    float u = 0.f;                                 // w_q (walk) or delta_q (check)
    for (int q0 = 0; q0 < nq; q0 += PF) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int q = q0 + j;
            if (act) ush[i] = u;
            __builtin_amdgcn_wave_barrier();
            float y[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // short dependent chains
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const float4 uv = *(const float4*)(ush + 4 * k);
                const int h = 4 * (k & 1);
                y[h + 0] = fmaf(ring[j][k].x, uv.x, y[h + 0]);
                y[h + 1] = fmaf(ring[j][k].y, uv.y, y[h + 1]);
                y[h + 2] = fmaf(ring[j][k].z, uv.z, y[h + 2]);
                y[h + 3] = fmaf(ring[j][k].w, uv.w, y[h + 3]);
            }
            __builtin_amdgcn_wave_barrier();
            const float un = ((y[0] + y[4]) + (y[1] + y[5])) + ((y[2] + y[6]) + (y[3] + y[7])) +
                             radd[j];
            if (q < nq) {
                u = un;
                float* wn = a.wcar + (size_t)(g0 + q + 1) * D + ii;
                // check: wcar_{q+1} was read into radd before this write (only step q writes it)
                if (act) *wn = CHECK ? *wn + u : u;
            }
            fetch(min(q + PF, nq - 1), j);
        }
    }
}

template <int D>
static pn_status dense_adj_run(const DenseAdjArgs& a, int B, bool bf16, int max_passes,
                        hipStream_t stream, int* passes) {
    void (*chain)(DenseAdjArgs) = gru_adj_dchain_kernel<D>;
    void (*mprod)(DenseAdjArgs) = bf16 ? gru_adj_dmap_kernel<D, true> : gru_adj_dmap_kernel<D, false>;
    void (*walk)(DenseAdjArgs, int, int) = gru_adj_dcarry_kernel<D, false>;
    void (*check)(DenseAdjArgs, int, int) = gru_adj_dcarry_kernel<D, true>;
    const int cgrid = std::max(1, (a.ngroups + 63) / 64);    // 4 waves x 16 groups
    const int mgrid = std::max(1, (a.ngroups + 3) / 4);      // 4 waves x 1 group
    prof_launch("gru_adj_dmap", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(mprod, dim3(mgrid), dim3(256), 0, s2, a);
    });
    PN_HIP(hipGetLastError());
    prof_launch("gru_adj_dwalk", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(walk, dim3(B), dim3(64), 0, s2, a, 0, 0);
    });
    PN_HIP(hipGetLastError());
    PN_HIP(hipMemsetAsync(a.done, 0, sizeof(int) * B, stream));
    *passes = 0;
    for (int p = 1; p <= max_passes; ++p) {
        prof_launch("gru_adj_dchain", stream, [&](hipStream_t s2) {
            hipLaunchKernelGGL(chain, dim3(cgrid), dim3(256), 0, s2, a);
        });
        PN_HIP(hipGetLastError());
        PN_HIP(hipMemsetAsync(a.nopen, 0, sizeof(int), stream));
        prof_launch("gru_adj_dcheck", stream, [&](hipStream_t s2) {
            hipLaunchKernelGGL(check, dim3(B), dim3(64), 0, s2, a, p, p == max_passes ? 1 : 0);
        });
        PN_HIP(hipGetLastError());
        *passes = p;
        int open = 0;
        PN_HIP(hipMemcpyAsync(&open, a.nopen, sizeof(int), hipMemcpyDeviceToHost, stream));
        PN_HIP(hipStreamSynchronize(stream));
        if (open == 0) break;
    }
    return PN_OK;
}

size_t gru_adj_dense_bytes(int D, int ngroups, int B) {
    Carver c(nullptr);
    const size_t ng = (size_t)std::max(ngroups, 1);
    c.take<float>(ng * D * D);
    c.take<float>(ng * D);
    c.take<float>(ng * D);
    c.take<float>(ng * D);
    c.take<int>((size_t)B + 1);
    return c.bytes();
}

pn_status gru_adj_dense_solve(int D, const float* gates, const float* gs, const float* U,
                              float* lam, const IterState& st, int ngroups, int B,
                              const float* gmax, float tol, bool bf16, int max_passes,
                              void* dense_ws, hipStream_t stream) {
    Carver c(dense_ws);
    const size_t ng = (size_t)std::max(ngroups, 1);
    DenseAdjArgs a;
    a.gates = gates;
    a.gs = gs;
    a.U = U;
    a.lam = lam;
    a.tiles = st.tiles;
    a.groups = st.groups;
    a.group_start = st.group_start;
    a.ngroups = ngroups;
    a.mbuf = c.take<float>(ng * D * D);
    a.vbuf = c.take<float>(ng * D);
    a.wcar = c.take<float>(ng * D);
    a.wout = c.take<float>(ng * D);
    a.done = c.take<int>((size_t)B + 1);
    a.nopen = a.done + B;
    a.gmax = gmax;
    a.seq = st.seq;
    a.tol = tol;
    int passes = 0;
    // (with no groups at all every kernel returns at once and the check marks each sequence
    // converged with zero residual)
    switch (D) {
        case 16: return dense_adj_run<16>(a, B, bf16, max_passes, stream, &passes);
        case 32: return dense_adj_run<32>(a, B, bf16, max_passes, stream, &passes);
        case 48: return dense_adj_run<48>(a, B, bf16, max_passes, stream, &passes);
        case 64: return dense_adj_run<64>(a, B, bf16, max_passes, stream, &passes);
        default: break;
    }
    set_error("dense GRU adjoint not built for D=%d", D);
    return PN_ERR_UNSUPPORTED;
}

}  // namespace pn
