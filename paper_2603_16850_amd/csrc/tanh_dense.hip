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

constexpr int TD = 32;                       // state size handled by this kernel
constexpr int TL = 32;                       // chunk length (one MFMA row block)
constexpr int GMAP = TD * TD + TD;           // floats per group map: P row-major, then q

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
__global__ void __launch_bounds__(64) tanh_dense_local_kernel(TanhDArgs a) {
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
            // ---- stage s_{t-1}, s_t (of s^(k-1), or the guess s^(0)) and x_t
            const float* src = fuse ? sprev : scur;
            for (int idx = l; idx < (TL + 1) * (TD / 4); idx += 64) {
                const int r = idx / (TD / 4), c4 = idx % (TD / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r == 0) v = first ? *(const float4*)(a.s0 + (size_t)b * TD + 4 * c4)
                                      : *(const float4*)(src + (size_t)(row0 - 1) * TD + 4 * c4);
                else if (r - 1 < len) v = *(const float4*)(src + (size_t)(row0 + r - 1) * TD + 4 * c4);
                *(float4*)(sst + r * SS + 4 * c4) = v;
            }
            for (int idx = l; idx < TL * (DX / 4); idx += 64) {
                const int r = idx / (DX / 4), c4 = idx % (DX / 4);
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
                *(float4*)(xst + r * XS + 4 * c4) = v;
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
                // moving them across steps
                for (int t = 0; t < len; ++t) {
                    const float* prev = dvec[t & 1];
                    float part = 0.f;
#pragma unroll
                    for (int i = 0; i < 16; ++i) part += wrow[i] * prev[16 * g + i];
                    part += __shfl_xor(part, 32);
                    const float dl = dsh[t * TD + n] * part + csh[t * TD + n];
                    const float v = sst[(t + 1) * SS + n] + dl;
                    const bool rb = __any(!(fabsf(v) <= reset_abs));
                    if (g == 0) {
                        dvec[(t + 1) & 1][n] = dl;
                        sst[(t + 1) * SS + n] = rb ? 0.f : v;
                    }
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
                float part = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) part += wrow[i] * vec[16 * g + i];
                part += __shfl_xor(part, 32);
                const float qn = dt[n] * part + csh[t * TD + n];
#pragma unroll
                for (int e = 0; e < 16; ++e) pacc[e] = dt[acc_row(g, e)] * acc[e];
                __builtin_amdgcn_wave_barrier();
                if (g == 0) vec[n] = qn;
                __builtin_amdgcn_wave_barrier();
            }
        }
        // ---- the group's map: P row-major (P[r][c] at r * 32 + c), then q
        float* gm = a.gmap + (size_t)gi * GMAP;
#pragma unroll
        for (int e = 0; e < 16; ++e) gm[acc_row(g, e) * TD + n] = pacc[e];
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
// of CB groups, double-buffered: every thread loads the next batch while wave 0 runs the chain
// over the current one.
constexpr int CB = 6;

__global__ void __launch_bounds__(256) dense_carry_kernel(const float* __restrict__ gmap,
                                                          float* __restrict__ gcarry,
                                                          const Ctrl* ctrl, const SeqState* seq,
                                                          const int32_t* group_start, int B) {
    __shared__ __attribute__((aligned(16))) float buf[2][CB * GMAP];
    __shared__ float cv[2][TD];
    if (ld_i32(&ctrl->all_done)) return;
    const int b = blockIdx.x;
    if (b >= B || seq[b].status != kActive) return;       // same on every thread
    const int tid = threadIdx.x;
    const int g0 = group_start[b], G = group_start[b + 1] - g0;
    const int nb = (G + CB - 1) / CB;
    auto load = [&](int j, int p) {
        const int nv = min(CB, G - j * CB) * (GMAP / 4);
        const float4* srcv = (const float4*)(gmap + (size_t)(g0 + j * CB) * GMAP);
        for (int i = tid; i < nv; i += 256) ((float4*)buf[p])[i] = srcv[i];
    };
    if (nb > 0) load(0, 0);
    if (tid < TD) cv[0][tid] = 0.f;
    __syncthreads();
    int cur = 0;                               // wave 0 only
    for (int j = 0; j < nb; ++j) {
        if (j + 1 < nb) load(j + 1, (j + 1) & 1);
        if (tid < 64) {
            const int n = tid & 31, g = tid >> 5;
            const int gcount = min(CB, G - j * CB);
            const float* bb = buf[j & 1];
            for (int q = 0; q < gcount; ++q) {
                const float* P = bb + q * GMAP;
                if (g == 0) gcarry[(size_t)(g0 + j * CB + q) * TD + n] = cv[cur][n];
                float part = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) part += P[n * TD + 16 * g + i] * cv[cur][16 * g + i];
                part += __shfl_xor(part, 32);
                if (g == 0) cv[cur ^ 1][n] = part + P[TD * TD + n];
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
    int derr = 0;
    PN_TRY(finish_iterations(lay.st, hb, TD, sizeof(float), s, lay.salt, stream, info, all_conv,
                             &derr));
    if (derr) {
        set_error("device-side check failed in the dense tanh iteration");
        return PN_ERR_INTERNAL;
    }
    return PN_OK;
}

}  // namespace pn
