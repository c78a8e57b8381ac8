// GRU pieces shared by the quasi-DEER forward kernel and the adjoint kernels:
//   * GruGates: the gate pre-activations of 16 steps x 16 units per wave on FP32 MFMA, with
//     the recurrent and input weights held in registers as B operands.
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
        gemm_impl<false>(hrow, xrow, make_float2(0.f, 0.f), g, az, ar, aq, an);
    }
    // The same, with the lane's two x values of the row tail (DX % 16 == 8) read by the
    // caller beforehand (`xtail`), so that no LDS read of x follows later copies into LDS.
    PN_DEV void gemm_xtail(const float* hrow, const float* xrow, float2 xtail, int g,
                           floatx4& az, floatx4& ar, floatx4& aq, floatx4& an) const {
        gemm_impl<true>(hrow, xrow, xtail, g, az, ar, aq, an);
    }
    // the lane's x tail values, as gemm reads them
    PN_DEV static float2 xtail_of(const float* xrow, int g) {
        return KT ? *(const float2*)(xrow + 16 * KX + 2 * g) : make_float2(0.f, 0.f);
    }

    template <bool PRE>
    PN_DEV void gemm_impl(const float* hrow, const float* xrow, float2 xtail, int g,
                          floatx4& az, floatx4& ar, floatx4& aq, floatx4& an) const {
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
            const float2 x2 = PRE ? xtail : xtail_of(xrow, g);
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
    p.z = sigmoid_rcp(az + b_z);
    p.r = sigmoid_rcp(ar + b_r);
    p.q = aq + b_hn;
    p.n = tanh_rcp(an + b_n + p.r * p.q);
    return p;
}

}  // namespace pn
