// DEER with dense Jacobians for the tanh-RNN f(h, x) = tanh(W h + U x + b), D = 32: one fused
// kernel per Newton iteration; each single-wave workgroup takes chunks of L consecutive steps
// of one sequence (dynamic chunk ids, in sequence order).
//
// Per chunk:
//   1. f_t, the residual r_t = s_t - f_t (eq. r_def) and d_t = 1 - f_t^2 for the L steps; the
//      pre-activations are a [L x (32 + Dx)] x [(32 + Dx) x 32] GEMM on FP32 MFMA (32x32x2).
//      The Jacobian A_t = diag(d_t) W (eq. lil_j) is never stored: it is rebuilt on chip.
//   2. the chunk's composed affine map Delta_end = P Delta_in + q of the recurrence
//      Delta_t = A_t Delta_{t-1} + c_t, c_t = -r_t (eq. lin_rr):
//        P <- diag(d_t) (W P) on MFMA -- BF16 operands with FP32 accumulation (32x32x16, the
//        running product re-rounded to BF16 before every step) or FP32 (32x32x2);
//        q <- d_t (W q) + c_t in FP32.
//      The K order of each MFMA is the row order in which the previous MFMA leaves P in its
//      accumulator registers, so the product feeds the next step without any data movement
//      (W's columns are permuted to match once, in registers).
//   3. decoupled look-back over the preceding chunks of the sequence for Delta_in (words
//      published with self-validating sentinels; aggregates are applied as mat-vecs);
//   4. replay Delta_t = d_t (W Delta_{t-1}) + c_t from Delta_in in FP32, write
//      s^(k+1)_t = s_t + Delta_t (overflow reset guard), publish Delta_end.
// Because c_t is the exact FP32 residual, c = 0 gives Delta = 0 whatever the rounding of P:
// the fixed point is the FP32 rollout and BF16 products only change the convergence rate.
#include <algorithm>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Row held by accumulator element e of lane group g in a 32x32 MFMA result.
PN_DEV int acc_row(int g, int e) { return 8 * (e >> 2) + 4 * g + (e & 3); }

constexpr int TD = 32;                    // state size handled by this kernel
constexpr int AGG_WORDS = TD * TD / 2 + TD / 2;   // P (pairs along a row) + q
constexpr int INCL_WORDS = TD / 2;

struct TanhDArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];
    const float* params;      // W (32x32) | U (32xDx) | b (32)
    uint64_t* agg[2];         // [ntiles][AGG_WORDS]
    uint64_t* incl[2];        // [ntiles][INCL_WORDS]
    Ctrl* ctrl;
    SeqState* seq;
    const int64_t* offsets;
    const int32_t* tile_start;
    const int32_t* order;
    int B;
    int ntiles;
    float dscale;             // scale damping: A_t <- dscale A_t (1 - k; 1 without damping)
};

template <int DX, int L, bool BF16>
__global__ void __launch_bounds__(64) tanh_dense_iter_kernel(TanhDArgs a) {
    constexpr int SS = TD + 4, XS = DX + 4;
    constexpr int KT = TD + DX;               // linearise K
    static_assert(KT % 2 == 0 && L % 32 == 0, "shape");
    __shared__ __attribute__((aligned(16))) float sst[(L + 1) * SS];
    __shared__ __attribute__((aligned(16))) float xst[L * XS];
    __shared__ __attribute__((aligned(16))) float dsh[L * TD];
    __shared__ __attribute__((aligned(16))) float csh[L * TD];
    __shared__ __attribute__((aligned(16))) float vec[2][TD];
    __shared__ int tinfo[5];

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k_it = a.ctrl->iter;
    const int par = k_it & 1;
    const float reset_abs = a.ctrl->reset_abs;
    const float* __restrict__ sin = a.sbuf[par];
    float* __restrict__ sout = a.sbuf[par ^ 1];
    const int l = threadIdx.x;
    const int n = l & 31, g = l >> 5;

    const float* Wm = a.params;
    const float* Um = Wm + TD * TD;
    const float* bv = Um + TD * DX;
    // linearise B operand: Bk[p] = Wcat[n][2p + g], Wcat = [W | U]
    float blin[KT / 2];
#pragma unroll
    for (int p = 0; p < KT / 2; ++p) {
        const int kk = 2 * p + g;
        blin[p] = kk < TD ? Wm[n * TD + kk] : Um[n * DX + (kk - TD)];
    }
    const float bias_n = bv[n];
    // W row m = n, half g, for the FP32 mat-vec chains
    float wrow[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) wrow[i] = Wm[n * TD + 16 * g + i];
    // W column n at the rows this lane's accumulator holds (for P = diag(d) W at chunk start)
    float wcol[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) wcol[e] = Wm[acc_row(g, e) * TD + n];
    // A operand of the compose: W with its K order permuted to the accumulator row order
    bf16x8 wa_bf[2];
    float wa_f[16];
    if (BF16) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) wa_bf[h][jj] = (__bf16)Wm[n * TD + acc_row(g, 8 * h + jj)];
    } else {
#pragma unroll
        for (int p = 0; p < 16; ++p) wa_f[p] = Wm[n * TD + acc_row(g, p)];
    }

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
        for (int w = l; w < AGG_WORDS; w += 64) st_u64(&a.agg[par ^ 1][(size_t)tile * AGG_WORDS + w], kSent64);
        if (l < INCL_WORDS) st_u64(&a.incl[par ^ 1][(size_t)tile * INCL_WORDS + l], kSent64);

        // ---- stage s_{t-1}, s_t and x_t
        for (int idx = l; idx < (L + 1) * (TD / 4); idx += 64) {
            const int r = idx / (TD / 4), c4 = idx % (TD / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r == 0) v = first ? *(const float4*)(a.s0 + (size_t)b * TD + 4 * c4)
                                  : *(const float4*)(sin + (size_t)(row0 - 1) * TD + 4 * c4);
            else if (r - 1 < len) v = *(const float4*)(sin + (size_t)(row0 + r - 1) * TD + 4 * c4);
            *(float4*)(sst + r * SS + 4 * c4) = v;
        }
        for (int idx = l; idx < L * (DX / 4); idx += 64) {
            const int r = idx / (DX / 4), c4 = idx % (DX / 4);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
            *(float4*)(xst + r * XS + 4 * c4) = v;
        }
        __syncthreads();

        // ---- linearise: pre = [s_{t-1}, x_t] Wcat^T on MFMA, rows = steps
        uint32_t rmax = 0;
#pragma unroll
        for (int mb = 0; mb < L / 32; ++mb) {
            floatx16 acc = {};
            const int tr = mb * 32 + n;       // A row of this lane = step tr
#pragma unroll
            for (int p = 0; p < KT / 2; ++p) {
                const int kk = 2 * p + g;
                const float av = kk < TD ? sst[tr * SS + kk] : xst[tr * XS + (kk - TD)];
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, blin[p], acc, 0, 0, 0);
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int t = mb * 32 + acc_row(g, e);
                const float f = tanhf_(acc[e] + bias_n);
                const float sc = sst[(t + 1) * SS + n];
                const float res = sc - f;
                const bool valid = t < len;
                dsh[t * TD + n] = (first && t == 0) ? 0.f : a.dscale * (1.f - f * f);
                csh[t * TD + n] = -res;
                if (valid) rmax = max(rmax, absbits(res));
            }
        }
        __syncthreads();

        // ---- compose the chunk: P (MFMA) and q (FP32 mat-vec)
        float pacc[16];
        {
            const float* d0 = dsh;
#pragma unroll
            for (int e = 0; e < 16; ++e) pacc[e] = d0[acc_row(g, e)] * wcol[e];
        }
        if (g == 0) vec[0][n] = csh[n];
        __syncthreads();
        for (int t = 1; t < len; ++t) {
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
            // q chain (previous q in vec[(t-1)&1])
            const float* qv = vec[(t - 1) & 1];
            float part = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) part += wrow[i] * qv[16 * g + i];
            part += __shfl_xor(part, 32);
            if (g == 0) vec[t & 1][n] = dt[n] * part + csh[t * TD + n];
#pragma unroll
            for (int e = 0; e < 16; ++e) pacc[e] = dt[acc_row(g, e)] * acc[e];
            __syncthreads();
        }
        const float qend = vec[(len - 1) & 1][n];   // q[n] (all lanes)

        // ---- look-back for Delta_in
        float din = 0.f;   // lane n (both halves): Delta_in[n]
        if (!first) {
            uint64_t* ag = a.agg[par] + (size_t)tile * AGG_WORDS;
            // P as row pairs: word k*16 + n/2 holds (P[k][n], P[k][n+1]); lane (n, g) holds
            // rows acc_row(g, e) of column n
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float other = __shfl_down(pacc[e], 1);
                if ((n & 1) == 0) st_u64(&ag[acc_row(g, e) * 16 + (n >> 1)], pack2(pacc[e], other));
            }
            const float qo = __shfl_down(qend, 1);     // all lanes take part in the shuffle
            if (g == 0 && (n & 1) == 0) st_u64(&ag[TD * 16 + (n >> 1)], pack2(qend, qo));
            // walk back until an inclusive value is found
            int pred = tile - 1, spins = 0;
            for (;;) {
                const uint64_t iv = l < INCL_WORDS ? ld_u64(&a.incl[par][(size_t)pred * INCL_WORDS + l]) : 0ull;
                const bool iready = __all(l >= INCL_WORDS || ready64(iv));
                if (iready) break;
                bool aready = true;
                for (int w = l; w < AGG_WORDS; w += 64)
                    aready = aready && ready64(ld_u64(&a.agg[par][(size_t)pred * AGG_WORDS + w]));
                if (__all(aready)) { --pred; continue; }
                if (++spins > (1 << 20) || ld_i32(&a.ctrl->error)) { if (l == 0) atomicExch(&a.ctrl->error, 1); break; }
                __builtin_amdgcn_s_sleep(1);
            }
            // Delta_end of `pred`, then forward through the aggregates of pred+1 .. tile-1
            {
                const uint64_t iv = ld_u64(&a.incl[par][(size_t)pred * INCL_WORDS + (n >> 1)]);
                din = (n & 1) ? hi_of(iv) : lo_of(iv);
            }
            for (int p2 = pred + 1; p2 < tile; ++p2) {
                const uint64_t* pa = a.agg[par] + (size_t)p2 * AGG_WORDS;
                // lane (k = n, half g): sum over columns 16g .. 16g+15 of P[k][c] * din[c]
                float part = 0.f;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint64_t wv = ld_u64(&pa[n * 16 + 8 * g + i]);
                    const float d0 = __shfl(din, 16 * g + 2 * i), d1 = __shfl(din, 16 * g + 2 * i + 1);
                    part += lo_of(wv) * d0 + hi_of(wv) * d1;
                }
                part += __shfl_xor(part, 32);
                const uint64_t qw = ld_u64(&pa[TD * 16 + (n >> 1)]);
                din = part + ((n & 1) ? hi_of(qw) : lo_of(qw));
            }
        }

        // ---- replay from Delta_in, write s^(k+1), publish Delta_end
        if (g == 0) vec[0][n] = din;
        __syncthreads();
        int nreset = 0;
        float dlast = din;
        for (int t = 0; t < len; ++t) {
            const float* prev = vec[t & 1];
            float part = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) part += wrow[i] * prev[16 * g + i];
            part += __shfl_xor(part, 32);
            const float dl = dsh[t * TD + n] * part + csh[t * TD + n];
            const float v = sst[(t + 1) * SS + n] + dl;
            const bool bad = !(fabsf(v) <= reset_abs);
            const bool rowbad = __any(bad);
            if (g == 0) {
                vec[(t + 1) & 1][n] = dl;
                sout[(size_t)(row0 + t) * TD + n] = rowbad ? 0.f : v;
            }
            nreset += rowbad ? 1 : 0;
            dlast = dl;
            __syncthreads();
        }
        {
            const float other = __shfl_down(dlast, 1);
            if (g == 0 && (n & 1) == 0)
                st_u64(&a.incl[par][(size_t)tile * INCL_WORDS + (n >> 1)], pack2(dlast, other));
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) {
            atomicMax(&a.seq[b].maxr, rmax);
            if (nreset) atomicAdd(&a.seq[b].resets_pending, nreset);
        }
    }
}

// ---- host -------------------------------------------------------------------------------------

struct TanhDLayout {
    IterState st;
    float* salt;
    uint64_t* agg[2];
    uint64_t* incl[2];
    size_t bytes;
};

static TanhDLayout tanhd_layout(void* ws, const HostBatch& hb, int ntiles) {
    Carver c(ws);
    TanhDLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles);
    lay.salt = c.take<float>((size_t)hb.N * TD);
    for (int p = 0; p < 2; ++p) lay.agg[p] = c.take<uint64_t>((size_t)ntiles * AGG_WORDS);
    for (int p = 0; p < 2; ++p) lay.incl[p] = c.take<uint64_t>((size_t)ntiles * INCL_WORDS);
    lay.bytes = c.bytes();
    return lay;
}

constexpr int kTanhL = 32;

bool tanh_dense_supported(int D, int Dx) { return D == TD && (Dx == 16 || Dx == 32); }

size_t tanh_dense_workspace(int, int, const HostBatch& hb, const pn_opts&) {
    return tanhd_layout(nullptr, hb, tile_starts(hb, kTanhL)[hb.B]).bytes;
}

__global__ void fill_u64_kernel(uint64_t* p, size_t n, uint64_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

pn_status tanh_dense_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                             const float* s0, float* s, const pn_opts& o, void* ws,
                             hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    void (*kern)(TanhDArgs) = nullptr;
    const bool bf = o.compose == PN_COMPOSE_BF16;
    if (cd.Dx == 16) kern = bf ? tanh_dense_iter_kernel<16, kTanhL, true> : tanh_dense_iter_kernel<16, kTanhL, false>;
    else if (cd.Dx == 32) kern = bf ? tanh_dense_iter_kernel<32, kTanhL, true> : tanh_dense_iter_kernel<32, kTanhL, false>;
    else return PN_ERR_UNSUPPORTED;
    const std::vector<int32_t> ts = tile_starts(hb, kTanhL);
    const int ntiles = ts[hb.B];
    TanhDLayout lay = tanhd_layout(ws, hb, ntiles);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, kTanhL, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream));
    if (ntiles > 0) {
        const size_t na = (size_t)ntiles * AGG_WORDS, ni = (size_t)ntiles * INCL_WORDS;
        hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)std::min<size_t>(4096, (na + 255) / 256)),
                           dim3(256), 0, stream, lay.agg[0], na, kSent64);
        hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)std::min<size_t>(4096, (ni + 255) / 256)),
                           dim3(256), 0, stream, lay.incl[0], ni, kSent64);
        PN_HIP(hipGetLastError());
    }
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, 64, 0) != hipSuccess || occ < 1)
        occ = 1;
    const int grid = std::max(1, std::min(ntiles, cu_count() * occ));
    TanhDArgs args;
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
    args.dscale = o.damping == PN_DAMP_SCALE ? 1.f - o.damp_k : 1.f;
    auto one_iter = [&](hipStream_t st) {
        prof_launch("tanh_dense_iter", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, s2, args);
        });
        launch_decide(lay.st, hb.B, st);
    };
    std::vector<uintptr_t> key = {0x7444u, (uintptr_t)kern, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)cd.params,
                                  (uintptr_t)ws, (uintptr_t)hb.B, (uintptr_t)ntiles,
                                  float_bits(args.dscale)};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    int derr = 0;
    PN_TRY(finish_iterations(lay.st, hb, TD, sizeof(float), s, lay.salt, stream, info, all_conv,
                             &derr));
    if (derr) {
        set_error("look-back watchdog expired in the dense tanh scan");
        return PN_ERR_INTERNAL;
    }
    return PN_OK;
}

}  // namespace pn
