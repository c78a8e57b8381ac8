// DEER with dense Jacobians for the tanh-RNN f(h, x) = tanh(W h + U x + b), D = 32: one Newton
// iteration as a per-group pass and a carry pass, no workgroup waiting for another.
//
// Steps are cut into chunks of 32 (one MFMA row block) and the chunks of a sequence into groups
// of consecutive chunks (see IterState).  Iteration k, one single-wave workgroup per group,
// chunk by chunk in time order:
//   1. (k >= 1) apply the previous update: re-linearise at s^(k-1) (the same d_t, c_t the
//      previous iteration used) and replay Delta_t = d_t (W Delta_{t-1}) + c_t in FP32 from the
//      group's carry, giving s^(k) = s^(k-1) + Delta with the overflow reset guard; write it.
//   2. linearise at s^(k): f_t, the residual r_t = s_t - f_t (Ch. 2, eq. r_def), c_t = -r_t and
//      d_t = 1 - f_t^2, the pre-activations a [32 x (32 + Dx)] x [(32 + Dx) x 32] GEMM on FP32
//      MFMA (32x32x2).  The Jacobian A_t = diag(d_t) W (eq. lil_j) is never stored.
//   3. compose the group's affine map Delta_end = P Delta_in + q of Delta_t = A_t Delta_{t-1} +
//      c_t (eq. lin_rr, composed as eq. bin_op_affine):
//        P <- diag(d_t) (W P) on MFMA -- BF16 operands with FP32 accumulation (32x32x16, the
//        running product re-rounded to BF16 before every step) or FP32 (32x32x2);
//        q <- d_t (W q) + c_t in FP32.
//      The K order of each MFMA is the row order in which the previous MFMA leaves P in its
//      accumulator registers, so the product feeds the next step without data movement.
//   The carry pass (dense_carry_kernel) then runs Delta_in(g+1) = P_g Delta_in(g) + q_g over the
//   groups of every sequence (FP32 mat-vecs, the group maps streamed through LDS).
// Because c_t is the exact FP32 residual, c = 0 gives Delta = 0 whatever the rounding of P:
// the fixed point is the FP32 rollout and BF16 products only change the convergence rate.  (A
// group's first halo row is formed from its carry, which rounds differently from the replay
// that wrote that row; the difference scales with Delta and vanishes at the fixed point.)
#include <algorithm>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Row held by accumulator element e of lane group g in a 32x32 MFMA result.
PN_DEV int acc_row(int g, int e) { return 8 * (e >> 2) + 4 * g + (e & 3); }

constexpr int TD_ = 32;
// Stores column n of a 32x32 map held in accumulator layout (element e = row acc_row(g, e)) into
// a column-major map: rows 8k + 4g .. 8k + 4g + 3 are consecutive, four float4 stores per lane.
// Column-major maps let the carry's mat-vec read them with consecutive lanes on consecutive
// LDS banks.
PN_DEV void store_map_column(float* gm, const float* pacc, int n, int g) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
        *(float4*)(gm + n * TD_ + 8 * k + 4 * g) =
            make_float4(pacc[4 * k], pacc[4 * k + 1], pacc[4 * k + 2], pacc[4 * k + 3]);
}

constexpr int TD = TD_;                      // state size handled by this kernel
constexpr int TL = 32;                       // chunk length (one MFMA row block)
constexpr int GMAP = TD * TD + TD;           // floats per group map: P column-major, then q

struct TanhDArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];           // ping-pong iterates: s^(k) lives in sbuf[k & 1]
    const float* params;      // W (32x32) | U (32xDx) | b (32)
    float* gmap;              // [ngroups][GMAP] group maps of this iteration
    const float* gcarry;      // [ngroups][TD] carry into every group (previous iteration)
    Ctrl* ctrl;
    SeqState* seq;
    const TileInfo* tiles;    // by slot (chunks)
    const GroupInfo* groups;
    int ngroups;
    float dscale;             // scale damping: A_t <- dscale A_t (1 - k; 1 without damping)
};

template <int DX, bool BF16>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
tanh_dense_local_kernel(TanhDArgs a) {
    constexpr int SS = TD + 4, XS = DX + 4;
    constexpr int KT = TD + DX;               // linearise K
    static_assert(KT % 2 == 0, "shape");
    __shared__ __attribute__((aligned(16))) float sst[(TL + 1) * SS];
    __shared__ __attribute__((aligned(16))) float xst[TL * XS];
    __shared__ __attribute__((aligned(16))) float dsh[TL * TD];
    __shared__ __attribute__((aligned(16))) float csh[TL * TD];
    __shared__ __attribute__((aligned(16))) float vec[TD];        // q chain
    __shared__ __attribute__((aligned(16))) float dvec[2][TD];    // Delta chain of the replay
    __shared__ int badrow[TL + 1];
    constexpr int WS = KT + 4;                // row stride of [W | U] in LDS
    __shared__ __attribute__((aligned(16))) float wl[TD * WS];

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k_it = a.ctrl->iter;
    const bool fuse = k_it > 0;
    const float reset_abs = a.ctrl->reset_abs;
    const float* __restrict__ sprev = a.sbuf[(k_it + 1) & 1];   // s^(k-1)
    float* __restrict__ scur = a.sbuf[k_it & 1];                 // s^(k)
    const int l = threadIdx.x;
    const int n = l & 31, g = l >> 5;

    const float* Wm = a.params;
    const float* Um = Wm + TD * TD;
    const float* bv = Um + TD * DX;
    // [W | U] in LDS: the B operand of the linearisation and the W rows of the mat-vec chains
    for (int idx = l; idx < TD * KT; idx += 64) {
        const int r = idx / KT, c = idx % KT;
        wl[r * WS + c] = c < TD ? Wm[r * TD + c] : Um[r * DX + (c - TD)];
    }
    const float bias_n = bv[n];
    // A operand of the compose: W with its K order permuted to the accumulator row order
    bf16x8 wa_bf[2];
    float wa_f[16];
    // W[n][16 g .. 16 g + 15]: the lane's share of the mat-vecs of the replay and the q chain
    float wrow[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) wrow[i] = Wm[n * TD + 16 * g + i];
    // (W v)[n] for v in LDS: the lane's 16 products in four independent partial sums, the two
    // half-waves' halves added on the VALU (the same bits on both halves)
    auto wdot = [&](const float* v) {
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
            const float4 q = *(const float4*)(v + 16 * g + i);
            p0 += wrow[i] * q.x;
            p1 += wrow[i + 1] * q.y;
            p2 += wrow[i + 2] * q.z;
            p3 += wrow[i + 3] * q.w;
        }
        return sum_halves((p0 + p1) + (p2 + p3));
    };
    if (BF16) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) wa_bf[h][jj] = (__bf16)Wm[n * TD + acc_row(g, 8 * h + jj)];
    } else {
#pragma unroll
        for (int p = 0; p < 16; ++p) wa_f[p] = Wm[n * TD + acc_row(g, p)];
    }

    // pre-activations of the 32 staged steps (rows = steps) -> d, c in LDS; returns max |r|
    // over the valid steps
    auto linearise = [&](bool first, int len) -> uint32_t {
        floatx16 acc = {};
#pragma unroll
        for (int p = 0; p < KT / 2; ++p) {
            const int kk = 2 * p + g;
            const float av = kk < TD ? sst[n * SS + kk] : xst[n * XS + (kk - TD)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, wl[n * WS + kk], acc, 0, 0, 0);
        }
        uint32_t rm = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = acc_row(g, e);
            const float f = tanhf_(acc[e] + bias_n);
            const float res = sst[(t + 1) * SS + n] - f;
            dsh[t * TD + n] = (first && t == 0) ? 0.f : a.dscale * (1.f - f * f);
            csh[t * TD + n] = -res;
            if (t < len) rm = max(rm, absbits(res));
        }
        __syncthreads();
        return rm;
    };

    for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
        const GroupInfo gr = a.groups[gi];
        if (a.seq[gr.b].status != kActive) continue;
        const int b = gr.b;
        float pacc[16];                        // P (rows acc_row(g, e) of column n)
        uint32_t rmax = 0;
        int nreset = 0;
        if (g == 0 && fuse) dvec[0][n] = a.gcarry[(size_t)gi * TD + n];   // Delta_in of the group
        TileInfo tnext = a.tiles[gr.tile0];
        for (int kt = 0; kt < gr.ntl; ++kt) {
            const TileInfo ti = tnext;
            if (kt + 1 < gr.ntl) tnext = a.tiles[gr.tile0 + kt + 1];   // read ahead
            const int len = ti.len;
            const int64_t row0 = ti.row0;
            const bool first = (ti.flags & kTileTimeFirst) != 0;
            __syncthreads();
            // ---- stage s_{t-1}, s_t (of s^(k-1), or the guess s^(0)) and x_t: every load of
            // the chunk is issued before the first LDS write (one round trip, not one per row
            // block)
            const float* src = fuse ? sprev : scur;
            constexpr int NSI = ((TL + 1) * (TD / 4) + 63) / 64, NXI = (TL * (DX / 4) + 63) / 64;
            float4 sv[NSI], xv[NXI];
#pragma unroll
            for (int q = 0; q < NSI; ++q) {
                const int idx = l + 64 * q;
                const int r = idx / (TD / 4), c4 = idx % (TD / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (idx < (TL + 1) * (TD / 4)) {
                    if (r == 0) v = first ? *(const float4*)(a.s0 + (size_t)b * TD + 4 * c4)
                                          : *(const float4*)(src + (size_t)(row0 - 1) * TD + 4 * c4);
                    else if (r - 1 < len)
                        v = *(const float4*)(src + (size_t)(row0 + r - 1) * TD + 4 * c4);
                }
                sv[q] = v;
            }
#pragma unroll
            for (int q = 0; q < NXI; ++q) {
                const int idx = l + 64 * q;
                const int r = idx / (DX / 4), c4 = idx % (DX / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (idx < TL * (DX / 4) && r < len)
                    v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
                xv[q] = v;
            }
#pragma unroll
            for (int q = 0; q < NSI; ++q) {
                const int idx = l + 64 * q;
                if (idx < (TL + 1) * (TD / 4))
                    *(float4*)(sst + (idx / (TD / 4)) * SS + 4 * (idx % (TD / 4))) = sv[q];
            }
#pragma unroll
            for (int q = 0; q < NXI; ++q) {
                const int idx = l + 64 * q;
                if (idx < TL * (DX / 4))
                    *(float4*)(xst + (idx / (DX / 4)) * XS + 4 * (idx % (DX / 4))) = xv[q];
            }
            if (l <= TL) badrow[l] = 0;
            __syncthreads();

            if (fuse) {
                // ---- the previous iteration's update: d, c at s^(k-1), replay from Delta_in
                linearise(first, len);
                // halo row s^(k)_{t0-1} = s^(k-1)_{t0-1} + Delta_{t0-1} (whole-row reset guard)
                float hv = 0.f;
                if (!first) {
                    hv = sst[n] + dvec[0][n];
                    if (!(fabsf(hv) <= reset_abs)) badrow[0] = 1;
                }
                // one wave: the LDS exchange of Delta between lanes needs no barrier (the wave's
                // LDS operations complete in order); the wave barrier keeps the compiler from
                // moving them across steps.  Both half-waves hold the same values and both
                // write them (no divergent branch on the chain).
                for (int t = 0; t < len; ++t) {
                    const float dl = dsh[t * TD + n] * wdot(dvec[t & 1]) + csh[t * TD + n];
                    const float v = sst[(t + 1) * SS + n] + dl;
                    const bool rb = __any(!(fabsf(v) <= reset_abs));
                    dvec[(t + 1) & 1][n] = dl;
                    sst[(t + 1) * SS + n] = rb ? 0.f : v;
                    nreset += rb ? 1 : 0;
                    __builtin_amdgcn_wave_barrier();
                }
                __syncthreads();
                if (g == 0) {
                    if (!first) sst[n] = badrow[0] ? 0.f : hv;
                    dvec[0][n] = dvec[len & 1][n];      // Delta at the chunk's last step
                }
                __syncthreads();
                // s^(k) of the chunk to HBM
                for (int idx = l; idx < len * (TD / 4); idx += 64) {
                    const int r = idx / (TD / 4), c4 = idx % (TD / 4);
                    *(float4*)(scur + (size_t)(row0 + r) * TD + 4 * c4) =
                        *(const float4*)(sst + (r + 1) * SS + 4 * c4);
                }
            }

            // ---- linearise at s^(k) and compose the group's map
            rmax = max(rmax, linearise(first, len));
            int t0 = 0;
            if (kt == 0) {
                // P = A_{t0} = diag(d_{t0}) W, q = c_{t0}
#pragma unroll
                for (int e = 0; e < 16; ++e) pacc[e] = dsh[acc_row(g, e)] * wl[acc_row(g, e) * WS + n];
                if (g == 0) vec[n] = csh[n];
                t0 = 1;
                __syncthreads();
            }
            for (int t = t0; t < len; ++t) {
                const float* dt = dsh + t * TD;
                floatx16 acc = {};
                if (BF16) {
                    bf16x8 b0, b1;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        b0[jj] = (__bf16)pacc[jj];
                        b1[jj] = (__bf16)pacc[8 + jj];
                    }
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa_bf[0], b0, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa_bf[1], b1, acc, 0, 0, 0);
                } else {
#pragma unroll
                    for (int p = 0; p < 16; ++p)
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wa_f[p], pacc[p], acc, 0, 0, 0);
                }
                // q chain (LDS exchange within the wave, as in the replay)
                const float qn = dt[n] * wdot(vec) + csh[t * TD + n];
#pragma unroll
                for (int e = 0; e < 16; ++e) pacc[e] = dt[acc_row(g, e)] * acc[e];
                __builtin_amdgcn_wave_barrier();
                vec[n] = qn;
                __builtin_amdgcn_wave_barrier();
            }
        }
        // ---- the group's map: P column-major (P[r][c] at c * 32 + r), then q
        float* gm = a.gmap + (size_t)gi * GMAP;
        store_map_column(gm, pacc, n, g);
        if (g == 0) gm[TD * TD + n] = vec[n];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) {
            atomicMax(&a.seq[b].maxr, rmax);
            if (nreset) atomicAdd(&a.seq[b].resets_pending, nreset);
        }
    }
}

// ---- carry pass: Delta_in(g+1) = P_g Delta_in(g) + q_g over the groups of a sequence -------
// One workgroup of 256 threads per sequence.  The group maps are staged through LDS in batches
// of CB groups, double-buffered: waves 1-3 load the next batch while wave 0 runs the chain over
// the current one (wave 0 loads nothing, so its chain never waits on HBM).
constexpr int CB = 12;

__global__ void __launch_bounds__(256) dense_carry_kernel(const float* __restrict__ gmap,
                                                          float* __restrict__ gcarry,
                                                          const Ctrl* ctrl, const SeqState* seq,
                                                          const int32_t* group_start, int B) {
    __shared__ __attribute__((aligned(16))) float buf[2][CB * GMAP];
    __shared__ __attribute__((aligned(16))) float cv[2][TD];
    if (ld_i32(&ctrl->all_done)) return;
    const int b = blockIdx.x;
    if (b >= B || seq[b].status != kActive) return;       // same on every thread
    const int tid = threadIdx.x;
    const int g0 = group_start[b], G = group_start[b + 1] - g0;
    const int nb = (G + CB - 1) / CB;
    // batch j into buffer p by waves w0 .. w0 + nw - 1: straight from HBM into LDS
    // (global_load_lds, 16 B per lane to byte 16 * lane of a 1 KB slice), every slice of a wave
    // in flight at once, then one wait
    auto load = [&](int j, int p, int w0, int nw) {
        const int nv = min(CB, G - j * CB) * (GMAP / 4);          // float4 in the batch
        const float4* srcv = (const float4*)(gmap + (size_t)(g0 + j * CB) * GMAP);
        const int ln = tid & 63;
        for (int c = (tid >> 6) - w0; c * 64 < nv; c += nw)
            if (c * 64 + ln < nv)
                __builtin_amdgcn_global_load_lds(
                    (const void*)(srcv + c * 64 + ln),
                    (__attribute__((address_space(3))) void*)(buf[p] + c * 256), 16, 0, 0);
        __builtin_amdgcn_s_waitcnt(0x0F70);                        // vmcnt(0)
    };
    if (nb > 0) load(0, 0, 0, 4);
    if (tid < TD) cv[0][tid] = 0.f;
    __syncthreads();
    int cur = 0;                               // wave 0 only
    for (int j = 0; j < nb; ++j) {
        if (j + 1 < nb && tid >= 64) load(j + 1, (j + 1) & 1, 1, 3);
        if (tid < 64) {
            const int n = tid & 31, g = tid >> 5;
            const int gcount = min(CB, G - j * CB);
            const float* bb = buf[j & 1];
            for (int q = 0; q < gcount; ++q) {
                const float* P = bb + q * GMAP;
                if (g == 0) gcarry[(size_t)(g0 + j * CB + q) * TD + n] = cv[cur][n];
                float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
                for (int i = 0; i < 16; i += 4) {
                    const float4 c = *(const float4*)(cv[cur] + 16 * g + i);
                    p0 += P[(16 * g + i) * TD + n] * c.x;
                    p1 += P[(16 * g + i + 1) * TD + n] * c.y;
                    p2 += P[(16 * g + i + 2) * TD + n] * c.z;
                    p3 += P[(16 * g + i + 3) * TD + n] * c.w;
                }
                cv[cur ^ 1][n] = sum_halves((p0 + p1) + (p2 + p3)) + P[TD * TD + n];
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the LDS write has landed
                __builtin_amdgcn_wave_barrier();
                cur ^= 1;
            }
        }
        __syncthreads();
    }
}

// ---- host -------------------------------------------------------------------------------------

struct TanhDLayout {
    IterState st;
    float* salt;
    float* gmap;
    float* gcarry;
    size_t bytes;
};

static TanhDLayout tanhd_layout(void* ws, const HostBatch& hb, int ntiles, int ngroups) {
    Carver c(ws);
    TanhDLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles, ngroups);
    lay.salt = c.take<float>((size_t)hb.N * TD);
    lay.gmap = c.take<float>((size_t)std::max(ngroups, 1) * GMAP);
    lay.gcarry = c.take<float>((size_t)std::max(ngroups, 1) * TD);
    lay.bytes = c.bytes();
    return lay;
}

bool tanh_dense_supported(int D, int Dx) { return D == TD && (Dx == 16 || Dx == 32); }

typedef void (*TanhDKernel)(TanhDArgs);

static TanhDKernel tanhd_kernel(int Dx, bool bf) {
    if (Dx == 16) return bf ? tanh_dense_local_kernel<16, true> : tanh_dense_local_kernel<16, false>;
    if (Dx == 32) return bf ? tanh_dense_local_kernel<32, true> : tanh_dense_local_kernel<32, false>;
    return nullptr;
}

// Chunks per group: enough groups for about two per resident single-wave workgroup, at most 8
// chunks (256 steps), which keeps the carry chain of a sequence short.
static int tanhd_group_tiles(int ntiles, int resident) {
    return std::max(1, std::min(8, ntiles / std::max(1, 2 * resident)));
}

static int tanhd_resident(TanhDKernel k) {
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k, 64, 0) != hipSuccess || occ < 1)
        occ = 1;
    return cu_count() * occ;
}

size_t tanh_dense_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    TanhDKernel k = tanhd_kernel(Dx, o.compose == PN_COMPOSE_BF16);
    if (!k || D != TD) return 0;
    const std::vector<int32_t> ts = tile_starts(hb, TL);
    const int gt = o.group > 0 ? o.group : tanhd_group_tiles(ts[hb.B], tanhd_resident(k));
    return tanhd_layout(nullptr, hb, ts[hb.B], count_groups(ts, hb.B, gt)).bytes;
}

pn_status tanh_dense_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                             const float* s0, float* s, const pn_opts& o, void* ws,
                             hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    TanhDKernel kern = tanhd_kernel(cd.Dx, o.compose == PN_COMPOSE_BF16);
    if (!kern) return PN_ERR_UNSUPPORTED;
    const std::vector<int32_t> ts = tile_starts(hb, TL);
    const int ntiles = ts[hb.B];
    const int resident = tanhd_resident(kern);
    const int gt = o.group > 0 ? o.group : tanhd_group_tiles(ntiles, resident);
    const int ngroups = count_groups(ts, hb.B, gt);
    TanhDLayout lay = tanhd_layout(ws, hb, ntiles, ngroups);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, TL, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream, gt));
    const int grid = std::max(1, std::min(ngroups, resident));
    TanhDArgs args;
    args.x = x;
    args.s0 = s0;
    args.sbuf[0] = s;
    args.sbuf[1] = lay.salt;
    args.params = (const float*)cd.params;
    args.gmap = lay.gmap;
    args.gcarry = lay.gcarry;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.tiles = lay.st.tiles;
    args.groups = lay.st.groups;
    args.ngroups = ngroups;
    args.dscale = o.damping == PN_DAMP_SCALE ? 1.f - o.damp_k : 1.f;
    auto one_iter = [&](hipStream_t st) {
        prof_launch("tanh_dense_local", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, s2, args);
        });
        prof_launch("dense_carry", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(dense_carry_kernel, dim3(std::max(1, hb.B)), dim3(256), 0, s2,
                               (const float*)lay.gmap, lay.gcarry, (const Ctrl*)lay.st.ctrl,
                               (const SeqState*)lay.st.seq, (const int32_t*)lay.st.group_start,
                               hb.B);
        });
        launch_decide(lay.st, hb.B, st, true);
    };
    std::vector<uintptr_t> key = {0x7445u, (uintptr_t)kern, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)cd.params,
                                  (uintptr_t)ws, (uintptr_t)hb.B, (uintptr_t)ntiles,
                                  (uintptr_t)ngroups, float_bits(args.dscale)};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    PN_TRY(finish_iterations(lay.st, hb, TD, sizeof(float), s, lay.salt, stream, info, all_conv));
    return PN_OK;
}

// ==== adjoint ===================================================================================
// Ch. 3, "Training and the backwards pass": lambda_t = g_t + A_{t+1}^T lambda_{t+1}, lambda_T = g_T,
// where A_{t+1}^T = W^T diag(d_{t+1}) and d_t = 1 - f(s_{t-1}, x_t)^2 at the solution (eq. lil_j).
// The reverse recurrence is solved by the forward Newton step run backwards in time, on the
// same chunks, groups and dense carry:
//   rho_t   = lambda_t - g_t - W^T (e_t * lambda_{t+1})    (exact FP32 residual, on MFMA)
//   Delta_t = W^T (e_t * Delta_{t+1}) - rho_t,  lambda <- lambda + Delta,
// with e_t = d_{t+1} (0 at the sequence end, where Delta_{T+1} = 0).  The recurrence is linear,
// so with FP32 group maps one update lands on the adjoint up to rounding and the next iteration
// only confirms the stopping test; with BF16 maps the update is approximate and the exact FP32
// residual drives further updates to the same fixed point.  Stopping rule: max |rho| <=
// tol * max(1, max |g|) over the sequence.  Then (eq. unrolled_bwds), with delta_t = d_t * lambda_t:
//   dW = sum_t delta_t s_{t-1}^T,  dU = sum_t delta_t x_t^T,  db = sum_t delta_t,
//   dx_t = U^T delta_t,  ds_0 = W^T delta_1.
// Kernels: prep (d_t at the solution and max |g|, once), local (one per iteration, per group,
// chunks taken from the sequence end), dense_carry over the reverse-ordered groups, grad
// (per-workgroup partials of dW, dU, db on MFMA, dx, ds_0), the FP64 sum of the partials.

struct TanhAdjArgs {
    const float* x;
    const float* s0;
    const float* s;
    const float* gs;
    const float* params;      // W (32x32) | U (32xDx) | b (32)
    float* dd;                // [N][TD] d_t at the solution
    float* lam[2];            // iteration k >= 1 writes lambda^(k) to lam[k & 1]; lambda^(0) = gs
    float* gmap;              // [ngroups][GMAP] group maps of this iteration
    const float* gcarry;      // [ngroups][TD] Delta at the step after every group (previous iteration)
    uint32_t* gmax;           // [B] max |g| per sequence (float bits)
    uint32_t* cmax;           // [ntiles] max |g| per chunk (float bits), by slot
    const int32_t* tile_start; // [B + 1] chunk slots of every sequence
    Ctrl* ctrl;
    SeqState* seq;
    const TileInfo* tiles;    // by slot: chunks taken from the sequence end
    const GroupInfo* groups;
    int ngroups;
    int ntiles;
    int B;
    float* part;              // [grid][P] per-workgroup partial parameter gradients
    float* gx;                // may be null
    float* gs0;               // may be null
};

// d_t = 1 - tanh(W s_{t-1} + U x_t + b)^2 of every step (pre-activations on FP32 MFMA, one chunk
// per single-wave workgroup, the B operand [W | U] read straight into registers) and max |g| of
// every sequence.
template <int DX>
__global__ void __launch_bounds__(64) tanh_adj_prep_kernel(TanhAdjArgs a) {
    constexpr int SS = TD + 4, XS = DX + 4, KT = TD + DX;
    static_assert(KT % 2 == 0, "shape");
    __shared__ __attribute__((aligned(16))) float hst[TL * SS];
    __shared__ __attribute__((aligned(16))) float xst[TL * XS];
    const int l = threadIdx.x, n = l & 31, g = l >> 5;
    const float* Wm = a.params;
    const float* Um = Wm + TD * TD;
    // B operand: [W | U][n][kk], kk = 2 p + g
    float bw[KT / 2];
#pragma unroll
    for (int p = 0; p < KT / 2; ++p) {
        const int kk = 2 * p + g;
        bw[p] = kk < TD ? Wm[n * TD + kk] : Um[n * DX + (kk - TD)];
    }
    const float bias_n = Um[TD * DX + n];
    for (int slot = blockIdx.x; slot < a.ntiles; slot += gridDim.x) {
        const TileInfo ti = a.tiles[slot];
        const int len = ti.len, b = ti.b;
        const int64_t row0 = ti.row0;
        const bool first = (ti.flags & kTileTimeFirst) != 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TL * (TD / 4) / 64; ++q) {
            const int idx = l + 64 * q;
            const int r = idx / (TD / 4), c4 = idx % (TD / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < len) v = (r == 0 && first) ? *(const float4*)(a.s0 + (size_t)b * TD + 4 * c4)
                                               : *(const float4*)(a.s + (size_t)(row0 + r - 1) * TD + 4 * c4);
            *(float4*)(hst + r * SS + 4 * c4) = v;
        }
#pragma unroll
        for (int q = 0; q < TL * (DX / 4) / 64; ++q) {
            const int idx = l + 64 * q;
            const int r = idx / (DX / 4), c4 = idx % (DX / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
            *(float4*)(xst + r * XS + 4 * c4) = v;
        }
        uint32_t gm = 0;                  // max |g| of the chunk: four float4 loads per lane in flight
#pragma unroll
        for (int q = 0; q < TL * (TD / 4) / 64; ++q) {
            const int idx = l + 64 * q;
            if (idx / (TD / 4) < len) {
                const float4 v = *(const float4*)(a.gs + (size_t)row0 * TD + 4 * idx);
                gm = max(max(gm, absbits(v.x)), max(absbits(v.y), max(absbits(v.z), absbits(v.w))));
            }
        }
        __syncthreads();
        floatx16 acc = {};
#pragma unroll
        for (int p = 0; p < KT / 2; ++p) {
            const int kk = 2 * p + g;
            const float av = kk < TD ? hst[n * SS + kk] : xst[n * XS + (kk - TD)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bw[p], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = acc_row(g, e);
            const float f = tanhf_(acc[e] + bias_n);
            if (t < len) a.dd[(size_t)(row0 + t) * TD + n] = 1.f - f * f;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) gm = max(gm, (uint32_t)__shfl_xor((int)gm, off));
        if (l == 0) a.cmax[slot] = gm;
    }
}

// max |g| of every sequence from its chunks' maxima (one workgroup per sequence)
__global__ void __launch_bounds__(256) tanh_adj_gmax_kernel(TanhAdjArgs a) {
    __shared__ uint32_t red[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    uint32_t m = 0;
    for (int k = a.tile_start[b] + tid; k < a.tile_start[b + 1]; k += 256) m = max(m, a.cmax[k]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) a.gmax[b] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// One adjoint iteration, one single-wave workgroup per group, the group's chunks from the
// latest to the earliest in time:
//   1. (k >= 1) apply the previous update: rho at lambda^(k-1) again, then the replay
//      Delta_t = W^T (e_t * Delta_{t+1}) + c_t from the group's carry, lambda^(k) = lambda^(k-1)
//      + Delta; write it;
//   2. the residual at lambda^(k): c_t = -rho_t, max |rho|;
//   3. compose the group's map Delta_first = P Delta_after + q in reverse time:
//        P <- W^T (diag(e_t) P) on MFMA (BF16 operands with FP32 accumulation, or FP32),
//        q <- W^T (e_t * q) + c_t in FP32.
template <bool BF16>
__global__ void __launch_bounds__(64) tanh_adj_local_kernel(TanhAdjArgs a) {
    constexpr int SS = TD + 4;
    __shared__ __attribute__((aligned(16))) float lst[(TL + 1) * SS];   // lambda rows 0 .. TL
    __shared__ __attribute__((aligned(16))) float gst[TL * SS];
    __shared__ __attribute__((aligned(16))) float est[TL * SS];         // e_t = d_{t+1}
    __shared__ __attribute__((aligned(16))) float csh[TL * TD];         // c_t = -rho_t
    __shared__ __attribute__((aligned(16))) float wl[TD * SS];          // W row-major
    __shared__ __attribute__((aligned(16))) float vec[TD];              // q chain
    __shared__ __attribute__((aligned(16))) float dvec[2][TD];          // Delta chain of the replay

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k_it = a.ctrl->iter;
    const bool fuse = k_it > 0;
    const float* __restrict__ lprev = k_it <= 1 ? a.gs : a.lam[(k_it + 1) & 1];   // lambda^(k-1)
    float* __restrict__ lcur = a.lam[k_it & 1];                                    // lambda^(k)
    const int l = threadIdx.x;
    const int n = l & 31, g = l >> 5;
    const float* Wm = a.params;
    for (int idx = l; idx < TD * TD; idx += 64) wl[(idx / TD) * SS + idx % TD] = Wm[idx];
    // A operand of the compose: W^T with its K order permuted to the accumulator row order
    bf16x8 wa_bf[2];
    float wa_f[16];
    // W[16 g .. 16 g + 15][n]: the lane's share of W^T v in the replay and the q chain
    float wcol[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) wcol[i] = Wm[(16 * g + i) * TD + n];
    // (W^T (e .* v))[n] for e, v in LDS: four independent partial sums, the half-waves' halves
    // added on the VALU (the same bits on both halves)
    auto wtdot = [&](const float* e, const float* v) {
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
            const float4 ee = *(const float4*)(e + 16 * g + i);
            const float4 vv = *(const float4*)(v + 16 * g + i);
            p0 += wcol[i] * (ee.x * vv.x);
            p1 += wcol[i + 1] * (ee.y * vv.y);
            p2 += wcol[i + 2] * (ee.z * vv.z);
            p3 += wcol[i + 3] * (ee.w * vv.w);
        }
        return sum_halves((p0 + p1) + (p2 + p3));
    };
    if (BF16) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) wa_bf[h][jj] = (__bf16)Wm[acc_row(g, 8 * h + jj) * TD + n];
    } else {
#pragma unroll
        for (int p = 0; p < 16; ++p) wa_f[p] = Wm[acc_row(g, p) * TD + n];
    }

    // rho_t = lambda_t - g_t - W^T (e_t * lambda_{t+1}) of the staged chunk -> c = -rho in LDS;
    // returns max |rho| over the valid steps
    auto residual = [&](int len) -> uint32_t {
        floatx16 acc = {};
#pragma unroll
        for (int p = 0; p < TD / 2; ++p) {
            const int kk = 2 * p + g;
            const float av = est[n * SS + kk] * lst[(n + 1) * SS + kk];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, wl[kk * SS + n], acc, 0, 0, 0);
        }
        uint32_t rm = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int t = acc_row(g, e);
            const float rho = lst[t * SS + n] - gst[t * SS + n] - acc[e];
            csh[t * TD + n] = -rho;
            if (t < len) rm = max(rm, absbits(rho));
        }
        __syncthreads();
        return rm;
    };

    for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
        const GroupInfo gr = a.groups[gi];
        if (a.seq[gr.b].status != kActive) continue;
        const int b = gr.b;
        const float gscale = 1.f / fmaxf(1.f, __uint_as_float(a.gmax[b]));
        float pacc[16];                        // P (rows acc_row(g, e) of column n)
        float qreg = 0.f;                      // q[n] (lanes of g = 0)
        uint32_t rmax = 0;
        if (g == 0) dvec[0][n] = fuse ? a.gcarry[(size_t)gi * TD + n] : 0.f;
        TileInfo tnext = a.tiles[gr.tile0];
        for (int kt = 0; kt < gr.ntl; ++kt) {
            const TileInfo ti = tnext;
            if (kt + 1 < gr.ntl) tnext = a.tiles[gr.tile0 + kt + 1];   // read ahead
            const int len = ti.len;
            const int64_t row0 = ti.row0;
            const bool last = (ti.flags & kTileScanFirst) != 0;        // chunk at the sequence end
            const int nl = last ? len : len + 1;                       // lambda rows with the halo
            const int ne = last ? len - 1 : len;                       // rows with a successor step
            __syncthreads();
            // ---- stage lambda^(k-1) (rows 0 .. len, row len being the first step of the next
            // chunk in time), g and e of the chunk
            for (int idx = l; idx < (TL + 1) * (TD / 4); idx += 64) {
                const int r = idx / (TD / 4), c4 = idx % (TD / 4);
                const size_t o = (size_t)(row0 + r) * TD + 4 * c4;
                const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                *(float4*)(lst + r * SS + 4 * c4) = r < nl ? *(const float4*)(lprev + o) : z;
                if (r < TL) {
                    *(float4*)(gst + r * SS + 4 * c4) = r < len ? *(const float4*)(a.gs + o) : z;
                    *(float4*)(est + r * SS + 4 * c4) = r < ne ? *(const float4*)(a.dd + o + TD) : z;
                }
            }
            __syncthreads();

            if (fuse) {
                residual(len);                 // c of the previous iteration (at lambda^(k-1))
                float hv = 0.f;                // lambda^(k) of the halo row
                if (!last) hv = lst[len * SS + n] + dvec[0][n];
                // one wave: the LDS exchange of Delta between lanes needs no barrier (the wave's
                // LDS operations complete in order); the wave barrier keeps the compiler from
                // moving them across steps
                for (int it = 0; it < len; ++it) {
                    const int t = len - 1 - it;
                    const float dl = wtdot(est + t * SS, dvec[it & 1]) + csh[t * TD + n];
                    if (g == 0) {
                        dvec[(it + 1) & 1][n] = dl;
                        lst[t * SS + n] += dl;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                __syncthreads();
                if (g == 0) {
                    if (!last) lst[len * SS + n] = hv;
                    dvec[0][n] = dvec[len & 1][n];      // Delta at the chunk's first step
                }
                __syncthreads();
                for (int idx = l; idx < len * (TD / 4); idx += 64) {
                    const int r = idx / (TD / 4), c4 = idx % (TD / 4);
                    *(float4*)(lcur + (size_t)(row0 + r) * TD + 4 * c4) =
                        *(const float4*)(lst + r * SS + 4 * c4);
                }
            }

            // ---- residual at lambda^(k) and the group's map, latest step first
            rmax = max(rmax, residual(len));
            int t0 = len - 1;
            if (kt == 0) {
                // P = W^T diag(e_{t0}), q = c_{t0}
                const float en = est[t0 * SS + n];
#pragma unroll
                for (int e = 0; e < 16; ++e) pacc[e] = wl[n * SS + acc_row(g, e)] * en;
                qreg = csh[t0 * TD + n];
                if (g == 0) vec[n] = qreg;
                t0 -= 1;
                __syncthreads();
            }
            for (int t = t0; t >= 0; --t) {
                const float* et = est + t * SS;
                floatx16 acc = {};
                if (BF16) {
                    bf16x8 b0, b1;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        b0[jj] = (__bf16)(et[acc_row(g, jj)] * pacc[jj]);
                        b1[jj] = (__bf16)(et[acc_row(g, 8 + jj)] * pacc[8 + jj]);
                    }
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa_bf[0], b0, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa_bf[1], b1, acc, 0, 0, 0);
                } else {
#pragma unroll
                    for (int p = 0; p < 16; ++p)
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wa_f[p], et[acc_row(g, p)] * pacc[p],
                                                                   acc, 0, 0, 0);
                }
                qreg = wtdot(et, vec) + csh[t * TD + n];
#pragma unroll
                for (int e = 0; e < 16; ++e) pacc[e] = acc[e];
                __builtin_amdgcn_wave_barrier();
                if (g == 0) vec[n] = qreg;
                __builtin_amdgcn_wave_barrier();
            }
        }
        float* gm = a.gmap + (size_t)gi * GMAP;
        store_map_column(gm, pacc, n, g);
        if (g == 0) gm[TD * TD + n] = qreg;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) atomicMax(&a.seq[b].maxr, absbits(__uint_as_float(rmax) * gscale));
    }
}

// Gradients from the final adjoint iterate: single-wave workgroups over the chunks; per chunk
// delta = d * lambda (LDS), dW += delta^T [s_{t-1}], dU += delta^T [x_t] (FP32 MFMA, K = steps,
// accumulated in registers over the workgroup's chunks), db, dx = delta U^T (MFMA, rows = steps),
// ds_0 = W^T delta at a sequence's first step.  Partials: [dW | dU | db] per workgroup.
template <int DX>
__global__ void __launch_bounds__(64) tanh_adj_grad_kernel(TanhAdjArgs a) {
    constexpr int SS = TD + 4, XS = DX + 4;
    constexpr int P = TD * TD + TD * DX + TD;
    __shared__ __attribute__((aligned(16))) float dst[TL * SS];
    __shared__ __attribute__((aligned(16))) float hst[TL * SS];
    __shared__ __attribute__((aligned(16))) float xst[TL * XS];
    const int l = threadIdx.x, n = l & 31, g = l >> 5;
    const float* Wm = a.params;
    const float* Um = Wm + TD * TD;
    // B operand of dx = delta U^T: U[k][n], k = 2 p + g
    float ub[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) ub[p] = n < DX ? Um[(2 * p + g) * DX + n] : 0.f;
    floatx16 aw = {}, au = {};
    float dbs = 0.f;
    for (int slot = blockIdx.x; slot < a.ntiles; slot += gridDim.x) {
        const TileInfo ti = a.tiles[slot];
        const int len = ti.len, b = ti.b;
        const int64_t row0 = ti.row0;
        const bool first = (ti.flags & kTileTimeFirst) != 0;
        const SeqState sq = a.seq[b];
        const float* lam = sq.iters == 0 ? a.gs : a.lam[sq.parity];
        __syncthreads();
        for (int idx = l; idx < TL * (TD / 4); idx += 64) {
            const int r = idx / (TD / 4), c4 = idx % (TD / 4);
            const size_t o = (size_t)(row0 + r) * TD + 4 * c4;
            float4 dv = make_float4(0.f, 0.f, 0.f, 0.f), hv = dv;
            if (r < len) {
                const float4 lv = *(const float4*)(lam + o), ev = *(const float4*)(a.dd + o);
                dv = make_float4(lv.x * ev.x, lv.y * ev.y, lv.z * ev.z, lv.w * ev.w);
                hv = (r == 0 && first) ? *(const float4*)(a.s0 + (size_t)b * TD + 4 * c4)
                                       : *(const float4*)(a.s + o - TD);
            }
            *(float4*)(dst + r * SS + 4 * c4) = dv;
            *(float4*)(hst + r * SS + 4 * c4) = hv;
        }
        for (int idx = l; idx < TL * (DX / 4); idx += 64) {
            const int r = idx / (DX / 4), c4 = idx % (DX / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
            *(float4*)(xst + r * XS + 4 * c4) = v;
        }
        __syncthreads();
        floatx16 ax = {};
#pragma unroll
        for (int p = 0; p < TL / 2; ++p) {
            const int kk = 2 * p + g;                 // step (K of the parameter GEMMs)
            const float dv = dst[kk * SS + n];        // delta_kk[n]
            dbs += dv;
            aw = __builtin_amdgcn_mfma_f32_32x32x2f32(dv, hst[kk * SS + n], aw, 0, 0, 0);
            au = __builtin_amdgcn_mfma_f32_32x32x2f32(dv, n < DX ? xst[kk * XS + n] : 0.f, au, 0, 0, 0);
            ax = __builtin_amdgcn_mfma_f32_32x32x2f32(dst[n * SS + kk], ub[p], ax, 0, 0, 0);
        }
        if (a.gx && n < DX) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int t = acc_row(g, e);
                if (t < len) a.gx[(size_t)(row0 + t) * DX + n] = ax[e];
            }
        }
        if (first && a.gs0 && g == 0) {
            float v = 0.f;
            for (int i = 0; i < TD; ++i) v += Wm[i * TD + n] * dst[i];
            a.gs0[(size_t)b * TD + n] = v;
        }
    }
    float* pp = a.part + (size_t)blockIdx.x * P;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = acc_row(g, e);
        pp[i * TD + n] = aw[e];
        if (n < DX) pp[TD * TD + i * DX + n] = au[e];
    }
    dbs += __shfl_xor(dbs, 32);
    if (g == 0) pp[TD * TD + TD * DX + n] = dbs;
}

__global__ void tanh_adj_gs0_clear_kernel(float* gs0, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) gs0[i] = 0.f;
}

// Sequential baseline of the adjoint: lambda_t = g_t + W^T (e_t * lambda_{t+1}) one step at a
// time per sequence (one single-wave workgroup per sequence, lane j holds column j of W; the
// products e_k lambda_k go through LDS without barriers), g and e of the next 4 steps
// prefetched into registers; writes lambda to lam[1] and marks it as the final iterate.
__global__ void __launch_bounds__(64) tanh_seq_adj_kernel(TanhAdjArgs a, const int64_t* offsets) {
    constexpr int PF = 4;
    __shared__ __attribute__((aligned(16))) float pb[2][TD];     // e_k lambda_k of the step
    const int b = blockIdx.x, j = threadIdx.x;
    const bool act = j < TD;
    const int jj = act ? j : 0;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    if (T == 0) return;                      // nothing to walk (and no row to prefetch)
    float w[TD];                                  // column j of W
#pragma unroll
    for (int k = 0; k < TD; ++k) w[k] = a.params[k * TD + jj];
    float* lam = a.lam[1];
    // operands of reverse step it (t = T - 1 - it): g_t and e_t = d_{t+1} (0 at the end)
    auto fetch = [&](int64_t it) {
        const int64_t t = T - 1 - it;
        return float2{a.gs[(size_t)(r0 + t) * TD + jj],
                      it > 0 ? a.dd[(size_t)(r0 + t + 1) * TD + jj] : 0.f};
    };
    float lnext = 0.f;                            // lambda_{t+1}, lane j's entry
    auto step = [&](int64_t it, float2 ge) {
        const int64_t t = T - 1 - it;
        float* pc = pb[it & 1];
        if (act) pc[j] = ge.y * lnext;
        __builtin_amdgcn_wave_barrier();
        float a0 = ge.x, a1 = 0.f;
#pragma unroll
        for (int k = 0; k < TD; k += 4) {
            const float4 p4 = *(const float4*)(pc + k);
            a0 = fmaf(w[k], p4.x, a0);
            a1 = fmaf(w[k + 1], p4.y, a1);
            a0 = fmaf(w[k + 2], p4.z, a0);
            a1 = fmaf(w[k + 3], p4.w, a1);
        }
        lnext = a0 + a1;
        if (act) lam[(size_t)(r0 + t) * TD + j] = lnext;
        __builtin_amdgcn_wave_barrier();
    };
    const int64_t Tm = T - T % PF;
    float2 ring[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i) ring[i] = fetch(i < Tm ? i : 0);
    for (int64_t it0 = 0; it0 < Tm; it0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const float2 ge = ring[i];
            const int64_t itn = it0 + i + PF < Tm ? it0 + i + PF : it0 + i;
            ring[i] = fetch(itn);
            step(it0 + i, ge);
        }
    }
    for (int64_t it = Tm; it < T; ++it) step(it, fetch(it));
    if (j == 0 && T > 0) {
        a.seq[b].iters = 1;
        a.seq[b].parity = 1;
    }
}

struct TanhALayout {
    IterState st;
    float* dd;
    float* lam[2];
    float* gmap;
    float* gcarry;
    uint32_t* gmax;
    uint32_t* cmax;
    float* part;
    size_t bytes;
};

// Two single-wave workgroups per SIMD resident at once (the grad kernel's register budget).
static int tanha_grad_grid(int ntiles) { return std::max(1, std::min(ntiles, 8 * cu_count())); }

static TanhALayout tanha_layout(void* ws, int Dx, const HostBatch& hb, int ntiles, int ngroups) {
    Carver c(ws);
    TanhALayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles, ngroups);
    lay.dd = c.take<float>((size_t)hb.N * TD);
    for (int p = 0; p < 2; ++p) lay.lam[p] = c.take<float>((size_t)hb.N * TD);
    lay.gmap = c.take<float>((size_t)std::max(ngroups, 1) * GMAP);
    lay.gcarry = c.take<float>((size_t)std::max(ngroups, 1) * TD);
    lay.gmax = c.take<uint32_t>(std::max(hb.B, 1));
    lay.cmax = c.take<uint32_t>(std::max(ntiles, 1));
    lay.part = c.take<float>((size_t)tanha_grad_grid(ntiles) * (TD * TD + TD * Dx + TD));
    lay.bytes = c.bytes();
    return lay;
}

typedef void (*TanhAKernel)(TanhAdjArgs);

static int tanha_groups(const std::vector<int32_t>& ts, int B, int group, bool bf, int* gt,
                        int* resident) {
    const TanhAKernel k = bf ? tanh_adj_local_kernel<true> : tanh_adj_local_kernel<false>;
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k, 64, 0) != hipSuccess || occ < 1)
        occ = 1;
    *resident = cu_count() * occ;
    // about one group per resident workgroup, at most 8 chunks: the adjoint's local pass runs
    // only twice, so a shorter carry chain pays more than a second round of groups
    *gt = group > 0 ? group : std::max(1, std::min(8, ts[B] / std::max(1, *resident)));
    return count_groups(ts, B, *gt);
}

size_t tanh_adjoint_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    if (!tanh_dense_supported(D, Dx)) return 0;
    const std::vector<int32_t> ts = tile_starts(hb, TL);
    int gt, resident;
    const int ngroups = tanha_groups(ts, hb.B, o.group, o.compose == PN_COMPOSE_BF16, &gt, &resident);
    return tanha_layout(nullptr, Dx, hb, ts[hb.B], ngroups).bytes;
}

pn_status tanh_adjoint(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                       const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                       float* gparams, const pn_opts& o, void* ws, hipStream_t stream,
                       pn_seq_info* info, bool* all_conv) {
    const int Dx = cd.Dx;
    if (!tanh_dense_supported(cd.D, Dx)) return PN_ERR_UNSUPPORTED;
    const bool bf = o.compose == PN_COMPOSE_BF16;
    const TanhAKernel local = bf ? tanh_adj_local_kernel<true> : tanh_adj_local_kernel<false>;
    const TanhAKernel prep = Dx == 16 ? tanh_adj_prep_kernel<16> : tanh_adj_prep_kernel<32>;
    const TanhAKernel grad = Dx == 16 ? tanh_adj_grad_kernel<16> : tanh_adj_grad_kernel<32>;
    const std::vector<int32_t> ts = tile_starts(hb, TL);
    const int ntiles = ts[hb.B];
    int gt, resident;
    const int ngroups = tanha_groups(ts, hb.B, o.group, bf, &gt, &resident);
    TanhALayout lay = tanha_layout(ws, Dx, hb, ntiles, ngroups);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, TL, true, max_iters, (float)o.tol, (float)o.reset_abs,
                           stream, gt));

    TanhAdjArgs args{};
    args.x = x;
    args.s0 = s0;
    args.s = s;
    args.gs = gs;
    args.params = (const float*)cd.params;
    args.dd = lay.dd;
    for (int p = 0; p < 2; ++p) args.lam[p] = lay.lam[p];
    args.gmap = lay.gmap;
    args.gcarry = lay.gcarry;
    args.gmax = lay.gmax;
    args.cmax = lay.cmax;
    args.tile_start = lay.st.tile_start;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.tiles = lay.st.tiles;
    args.groups = lay.st.groups;
    args.ngroups = ngroups;
    args.ntiles = ntiles;
    args.B = hb.B;
    args.part = lay.part;
    args.gx = gx;
    args.gs0 = gs0;

    if (ntiles > 0) {
        prof_launch("tanh_adj_prep", stream, [&](hipStream_t s2) {
            hipLaunchKernelGGL(prep, dim3(ntiles), dim3(64), 0, s2, args);
            hipLaunchKernelGGL(tanh_adj_gmax_kernel, dim3(hb.B), dim3(256), 0, s2, args);
        });
        PN_HIP(hipGetLastError());
    } else {
        // no steps anywhere: every sequence stops at iteration 0 with a zero residual
        hipLaunchKernelGGL(tanh_adj_gmax_kernel, dim3(hb.B), dim3(256), 0, stream, args);
    }
    const int grid = std::max(1, std::min(ngroups, resident));
    auto one_iter = [&](hipStream_t st) {
        prof_launch("tanh_adj_local", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(local, dim3(grid), dim3(64), 0, s2, args);
        });
        prof_launch("dense_carry", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(dense_carry_kernel, dim3(std::max(1, hb.B)), dim3(256), 0, s2,
                               (const float*)lay.gmap, lay.gcarry, (const Ctrl*)lay.st.ctrl,
                               (const SeqState*)lay.st.seq, (const int32_t*)lay.st.group_start,
                               hb.B);
        });
        launch_decide(lay.st, hb.B, st, true);
    };
    std::vector<uintptr_t> key = {0x7441u, (uintptr_t)local, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)gs,
                                  (uintptr_t)cd.params, (uintptr_t)ws, (uintptr_t)hb.B,
                                  (uintptr_t)ntiles, (uintptr_t)ngroups};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    PN_TRY(finish_iterations(lay.st, hb, TD, sizeof(float), nullptr, nullptr, stream, info,
                             all_conv));
    if (gs0) {
        hipLaunchKernelGGL(tanh_adj_gs0_clear_kernel, dim3(1), dim3(256), 0, stream, gs0, hb.B * TD);
        PN_HIP(hipGetLastError());
    }
    const int gg = tanha_grad_grid(ntiles);
    prof_launch("tanh_adj_grad", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(grad, dim3(gg), dim3(64), 0, s2, args);
    });
    PN_HIP(hipGetLastError());
    const int P = TD * TD + TD * Dx + TD;
    launch_partial_sum(lay.part, gg, P, gparams, stream);
    PN_HIP(hipGetLastError());
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    return PN_OK;
}

// Sequential baseline of tanh_adjoint: the same outputs, the reverse recurrence walked step by
// step (d_t and the gradient reductions are the parallel kernels above).
pn_status tanh_seq_bptt(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                        const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                        float* gparams, void* ws, hipStream_t stream) {
    const int Dx = cd.Dx;
    if (!tanh_dense_supported(cd.D, Dx)) return PN_ERR_UNSUPPORTED;
    const TanhAKernel prep = Dx == 16 ? tanh_adj_prep_kernel<16> : tanh_adj_prep_kernel<32>;
    const TanhAKernel grad = Dx == 16 ? tanh_adj_grad_kernel<16> : tanh_adj_grad_kernel<32>;
    const std::vector<int32_t> ts = tile_starts(hb, TL);
    const int ntiles = ts[hb.B];
    TanhALayout lay = tanha_layout(ws, Dx, hb, ntiles, 0);
    PN_TRY(init_iter_state(lay.st, hb, ts, TL, true, 1, 1.f, 1e4f, stream));
    TanhAdjArgs args{};
    args.x = x;
    args.s0 = s0;
    args.s = s;
    args.gs = gs;
    args.params = (const float*)cd.params;
    args.dd = lay.dd;
    for (int p = 0; p < 2; ++p) args.lam[p] = lay.lam[p];
    args.gmax = lay.gmax;
    args.cmax = lay.cmax;
    args.tile_start = lay.st.tile_start;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.tiles = lay.st.tiles;
    args.ntiles = ntiles;
    args.B = hb.B;
    args.part = lay.part;
    args.gx = gx;
    args.gs0 = gs0;
    if (ntiles > 0)
        hipLaunchKernelGGL(prep, dim3(ntiles), dim3(64), 0, stream, args);
    prof_launch("seq_adj", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(tanh_seq_adj_kernel, dim3(std::max(1, hb.B)), dim3(64), 0, s2, args,
                           (const int64_t*)lay.st.offsets);
    });
    PN_HIP(hipGetLastError());
    if (gs0) hipLaunchKernelGGL(tanh_adj_gs0_clear_kernel, dim3(1), dim3(256), 0, stream, gs0, hb.B * TD);
    const int gg = tanha_grad_grid(ntiles);
    hipLaunchKernelGGL(grad, dim3(gg), dim3(64), 0, stream, args);
    launch_partial_sum(lay.part, gg, TD * TD + TD * Dx + TD, gparams, stream);
    PN_HIP(hipGetLastError());
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    return PN_OK;
}

}  // namespace pn
