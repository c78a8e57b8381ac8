// GRU pieces shared by the quasi-DEER forward kernel and the adjoint kernels:
//   * GruGates: the gate pre-activations of 16 steps x 16 units per wave on FP32 MFMA, with
//     the recurrent and input weights held in registers as B operands;
//   * lookback(): the single-pass decoupled look-back of a scalar affine scan.
#pragma once
#include "pn_device.hpp"

namespace pn {

// Gate GEMM for one wave.  Units j = 16w + (lane % 16).  K runs over [h (D) ; x (DX)]; the K
// order inside every 16-wide block is permuted so that lane group g = lane / 16 reads one
// float4 (k = 16 kb + 4 g + i, i = 0..3) per four MFMAs; an 8-wide tail block over x uses
// float2 reads (k = 16 kb + 2 g + i, i = 0..1).  The B operands hold the same permutation.
template <int D, int DX>
struct GruGates {
    static constexpr int KH = D / 16;
    static constexpr int KX = DX / 16;
    static constexpr int KT = (DX % 16) / 8;
    float bzh[KH][4], brh[KH][4], bqh[KH][4];
    float bzx[KX + KT][4], brx[KX + KT][4], bnx[KX + KT][4];
    float b_z, b_r, b_n, b_hn;     // biases of unit j
    float dUz, dUr, dUn;           // diagonals U_z[j][j], U_r[j][j], U_n[j][j]

    PN_DEV void load(const float* params, int j, int g) {
        const float* W = params;                 // [W_z;W_r;W_n] (3D x DX)
        const float* U = W + 3 * D * DX;         // [U_z;U_r;U_n] (3D x D)
        const float* bias = U + 3 * D * D;       // [b_z;b_r;b_n]
        const float* bhn = bias + 3 * D;
#pragma unroll
        for (int kb = 0; kb < KH; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int kk = 16 * kb + 4 * g + i;
                bzh[kb][i] = U[(0 * D + j) * D + kk];
                brh[kb][i] = U[(1 * D + j) * D + kk];
                bqh[kb][i] = U[(2 * D + j) * D + kk];
            }
#pragma unroll
        for (int kb = 0; kb < KX + KT; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int kk;
                bool ok = true;
                if (kb < KX) kk = 16 * kb + 4 * g + i;
                else { kk = 16 * kb + 2 * g + i; ok = i < 2; }
                bzx[kb][i] = ok ? W[(0 * D + j) * DX + kk] : 0.f;
                brx[kb][i] = ok ? W[(1 * D + j) * DX + kk] : 0.f;
                bnx[kb][i] = ok ? W[(2 * D + j) * DX + kk] : 0.f;
            }
        b_z = bias[j];
        b_r = bias[D + j];
        b_n = bias[2 * D + j];
        b_hn = bhn[j];
        dUz = U[(0 * D + j) * D + j];
        dUr = U[(1 * D + j) * D + j];
        dUn = U[(2 * D + j) * D + j];
    }

    // Pre-activations for the 16 steps whose h rows start at `hrow` / x rows at `xrow`
    // (this lane's A row is hrow/xrow; outputs follow the MFMA D layout).
    //   az = W_z x + U_z h,  ar = W_r x + U_r h,  aq = U_n h,  an = W_n x   (no biases)
    PN_DEV void gemm(const float* hrow, const float* xrow, int g, floatx4& az, floatx4& ar,
                     floatx4& aq, floatx4& an) const {
        az = floatx4{0.f, 0.f, 0.f, 0.f};
        ar = az;
        aq = az;
        an = az;
#pragma unroll
        for (int kb = 0; kb < KH; ++kb) {
            const float4 h4 = *(const float4*)(hrow + 16 * kb + 4 * g);
            const float hv[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                az = mfma16x4(hv[i], bzh[kb][i], az);
                ar = mfma16x4(hv[i], brh[kb][i], ar);
                aq = mfma16x4(hv[i], bqh[kb][i], aq);
            }
        }
#pragma unroll
        for (int kb = 0; kb < KX; ++kb) {
            const float4 x4 = *(const float4*)(xrow + 16 * kb + 4 * g);
            const float xv[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                az = mfma16x4(xv[i], bzx[kb][i], az);
                ar = mfma16x4(xv[i], brx[kb][i], ar);
                an = mfma16x4(xv[i], bnx[kb][i], an);
            }
        }
        if (KT) {
            const float2 x2 = *(const float2*)(xrow + 16 * KX + 2 * g);
            const float xv[2] = {x2.x, x2.y};
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                az = mfma16x4(xv[i], bzx[KX][i], az);
                ar = mfma16x4(xv[i], brx[KX][i], ar);
                an = mfma16x4(xv[i], bnx[KX][i], an);
            }
        }
    }
};

// Gate values of one (step, unit) from its pre-activations.
struct GruPoint {
    float z, r, q, n;
};
PN_DEV GruPoint gru_point(float az, float ar, float aq, float an, float b_z, float b_r,
                          float b_n, float b_hn) {
    GruPoint p;
    p.z = sigmoidf_(az + b_z);
    p.r = sigmoidf_(ar + b_r);
    p.q = aq + b_hn;
    p.n = tanhf_(an + b_n + p.r * p.q);
    return p;
}

// Decoupled look-back of a scalar affine scan, one lane per (tile, unit) slot.
// The tile's own composed map is Delta_out = Ra * Delta_in + Rc.  `first` tiles have no
// predecessor (Delta_in = 0).  Predecessors are tile-1, tile-2, ... of the same chain; each
// publishes its aggregate (agg) before looking back and its inclusive value (incl) after.
// Returns Delta_in; sets ctrl->error if the spin watchdog expires.
PN_DEV float lookback(uint64_t* agg, uint32_t* incl, int tile, bool first, int stride, int j,
                      float Ra, float Rc, int* err) {
    const size_t slot = (size_t)tile * stride + j;
    if (first) {
        st_u32(&incl[slot], __float_as_uint(canon(Rc)));
        return 0.f;
    }
    st_u64(&agg[slot], pack2(Ra, Rc));
    float Aa = 1.f, Ac = 0.f;   // composed maps of the tiles between `pred` and this one
    float din = 0.f;
    int pred = tile - 1;
    int spins = 0;
    for (;;) {
        const uint32_t iv = ld_u32(&incl[(size_t)pred * stride + j]);
        if (ready32(iv)) {
            din = Aa * __uint_as_float(iv) + Ac;
            break;
        }
        const uint64_t av = ld_u64(&agg[(size_t)pred * stride + j]);
        if (ready64(av)) {
            Ac = Aa * hi_of(av) + Ac;
            Aa = Aa * lo_of(av);
            --pred;
            continue;
        }
        if (++spins > (1 << 20) || ld_i32(err)) {
            atomicExch(err, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    st_u32(&incl[slot], __float_as_uint(canon(Ra * din + Rc)));
    return din;
}

// Look-back with four predecessors per round: the four lanes g = 0..3 of unit u (lanes
// u, u+16, u+32, u+48) inspect slots base, base-1, base-2, base-3 at once.  Called by all 64
// lanes; returns Delta_in of unit j on every lane.  Slots of one sequence are consecutive,
// `first` is the sequence's first slot (it publishes only its inclusive value).
PN_DEV float lookback4(uint64_t* agg, uint32_t* incl, int slot, int first, int stride, int j,
                       int g, int u, float Ra, float Rc, int* err) {
    const size_t own = (size_t)slot * stride + j;
    if (slot == first) {
        if (g == 0) st_u32(&incl[own], __float_as_uint(canon(Rc)));
        return 0.f;
    }
    if (g == 0) st_u64(&agg[own], pack2(Ra, Rc));
    float Aa = 1.f, Ac = 0.f;     // composed maps of slots base+1 .. slot-1
    float din = 0.f;
    int base = slot - 1;
    int spins = 0;
    for (;;) {
        const int p = base - g;
        const bool valid = p >= first;
        const uint32_t iv = valid ? ld_u32(&incl[(size_t)p * stride + j]) : kSent32;
        const uint64_t av = valid ? ld_u64(&agg[(size_t)p * stride + j]) : kSent64;
        const uint64_t im = __ballot(valid && ready32(iv));
        const uint64_t am = __ballot(valid && ready64(av));
        int gs = -1;
#pragma unroll
        for (int gg = 3; gg >= 0; --gg)
            if ((im >> (16 * gg + u)) & 1ull) gs = gg;
        // aggregates needed: slots base .. base-gs+1 (all four when no inclusive value seen)
        const int need = gs >= 0 ? gs : 4;
        bool ok = gs >= 0 || base - 3 >= first;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg)
            if (gg < need && !((am >> (16 * gg + u)) & 1ull)) ok = false;
        // compose the needed aggregates, nearest first: map from Delta_end(base-need) to
        // Delta_end(base) is a_0 (a_1 (... ) + c_1) + c_0
        const float a_own = lo_of(av), c_own = hi_of(av);
        float pa = 1.f, pc = 0.f;
#pragma unroll
        for (int gg = 3; gg >= 0; --gg) {
            const float ag = __shfl(a_own, 16 * gg + u), cg = __shfl(c_own, 16 * gg + u);
            if (gg < need) { pc = ag * pc + cg; pa = ag * pa; }
        }
        const float ival = __uint_as_float(__shfl((int)iv, 16 * (gs < 0 ? 0 : gs) + u));
        if (ok) {
            if (gs >= 0) {
                din = Aa * (pa * ival + pc) + Ac;
                break;
            }
            Ac = Aa * pc + Ac;
            Aa = Aa * pa;
            base -= 4;
            continue;
        }
        if (++spins > (1 << 20) || ld_i32(err)) {
            atomicExch(err, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (g == 0) st_u32(&incl[own], __float_as_uint(canon(Ra * din + Rc)));
    return din;
}

}  // namespace pn
