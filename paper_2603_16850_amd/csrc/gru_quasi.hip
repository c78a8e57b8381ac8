// quasi-DEER for the GRU cell: one fused kernel per Newton iteration.
//
// For iterate s^(k) each workgroup takes tiles of L consecutive steps of one sequence (dynamic
// tile ids, in sequence order) and, in one pass over HBM:
//   1. stages s_{t-1}, s_t (L+1 rows) and x_t (L rows) in LDS;
//   2. evaluates the three gate pre-activations of f(s_{t-1}, x_t) for the L steps as a
//      small GEMM [L x (D+Dx)] x [(D+Dx) x 4 gate blocks] on FP32 MFMA (16x16x4), the
//      weights held in registers for the whole kernel;
//   3. forms the residual r_t = s_t - f_t(s_{t-1}) (Ch. 2, eq. r_def), the scan leaf
//      (a_t, c_t) = (diag A_t, -r_t) with the closed-form GRU diagonal (quasi-DEER,
//      eq. quasi_lds), and the per-sequence max |r| that the stopping test reads;
//   4. scans Delta_t = a_t Delta_{t-1} + c_t (eq. lin_rr with a diagonal transition) over
//      the tile: in registers, across lane groups by shuffles, across 16-step blocks serially;
//   5. publishes the tile aggregate, looks back over preceding tiles of the same sequence
//      for the carry-in Delta_{t0-1} (single-pass decoupled look-back), publishes its own
//      inclusive prefix, and
//   6. writes s^(k+1)_t = s_t + Delta_t with the overflow reset guard.
// At a sequence head a_t = 0, so the carry-in is Delta_0 = 0 (s_0 is fixed).
#include <algorithm>

#include "gru_common.hpp"
#include "pn_host.hpp"

namespace pn {

template <int D, int DX, int L>
struct GruQ {
    static_assert(D % 16 == 0 && D >= 16 && D <= 64, "D must be 16, 32, 48 or 64");
    static_assert(DX % 8 == 0 && DX >= 8 && DX <= 64, "Dx must be a multiple of 8");
    static_assert(L % 16 == 0 && L >= 16 && L <= 128, "tile length");
    static constexpr int NW = D / 16;       // waves; wave w owns units [16w, 16w+16)
    static constexpr int NT = 64 * NW;
    static constexpr int KH = D / 16;       // 16-wide K blocks over h
    static constexpr int KX = DX / 16;      // 16-wide K blocks over x
    static constexpr int KT = (DX % 16) / 8;// one 8-wide tail block over x (0/1)
    static constexpr int HS = D + 4;        // LDS row strides (floats), padded against
    static constexpr int XS = DX + 4;       // bank conflicts of the 16-row float4 reads
    static constexpr int MB = L / 16;       // 16-step blocks per tile
};

struct GruQArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];          // ping-pong iterates; iteration k reads sbuf[k&1]
    const float* params;
    uint64_t* agg[2];        // tile aggregates (a, c) per unit, by iteration parity
    uint32_t* incl[2];       // tile inclusive prefixes Delta_end per unit
    Ctrl* ctrl;
    SeqState* seq;
    const int64_t* offsets;
    const int32_t* tile_start;
    const int32_t* order;
    const TileInfo* tiles;   // processing order with geometry
    int B;
    int ntiles;
};

template <int D, int DX, int L>
__global__ void __launch_bounds__(64 * (D / 16)) __attribute__((amdgpu_waves_per_eu(2, 2)))
gru_quasi_iter_kernel(GruQArgs a) {
    using C = GruQ<D, DX, L>;
    __shared__ __attribute__((aligned(16))) float hs[(L + 1) * C::HS];
    __shared__ __attribute__((aligned(16))) float xs[L * C::XS];
    __shared__ int rowbad[L];
    __shared__ int tnext[2][8];   // next tile, double-buffered by loop parity

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k = a.ctrl->iter;
    const int par = k & 1;
    const float reset_abs = a.ctrl->reset_abs;
    const float* __restrict__ sin = a.sbuf[par];
    float* __restrict__ sout = a.sbuf[par ^ 1];
    uint64_t* aggc = a.agg[par];
    uint32_t* inclc = a.incl[par];
    uint64_t* aggn = a.agg[par ^ 1];
    uint32_t* incln = a.incl[par ^ 1];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int g = l >> 4;          // lane group (k-slot of A/B, row quad of D)
    const int u = l & 15;          // unit within the wave / row of A
    const int j = 16 * w + u;      // state unit this lane owns in the outputs

    GruGates<D, DX> wg;   // this wave's weights (units j) as MFMA B operands
    wg.load(a.params, j, g);

    for (int t = tid; t < L; t += C::NT) rowbad[t] = 0;
    if (tid == 0) fetch_tile(a.ctrl, a.tiles, a.seq, a.ntiles,
                             (int)atomicAdd(&a.ctrl->tile_counter, 1u), tnext[0]);

    for (int it = 0;; ++it) {
        __syncthreads();   // previous tile fully consumed (LDS reuse); tnext[it&1] published
        const int* tn = tnext[it & 1];
        if (tn[0] >= a.ntiles) break;
        const int tile = tn[1];         // scan slot of this tile
        const int b = tn[2];
        const int lt = tn[3];
        const int len = tn[4];
        const int64_t row0 = ((int64_t)tn[6] << 32) | (uint32_t)tn[5];
        if (tn[7] != kActive) {
            if (tid == 0)
                fetch_tile(a.ctrl, a.tiles, a.seq, a.ntiles,
                           (int)atomicAdd(&a.ctrl->tile_counter, 1u), tnext[(it + 1) & 1]);
            continue;
        }
        const bool first = lt == 0;

        // this tile's slots of the next iteration start unpublished
        if (g == 0) {
            st_u64(&aggn[(size_t)tile * D + j], kSent64);
            st_u32(&incln[(size_t)tile * D + j], kSent32);
        }

        // ---- stage s rows row0-1 .. row0+L-1 (stage row r <-> s_{t0-1+r}) and x rows ----
        {
            constexpr int Q = D / 4;
            for (int idx = tid; idx < (L + 1) * Q; idx += C::NT) {
                const int r = idx / Q, c4 = idx % Q;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r == 0) {
                    v = first ? *(const float4*)(a.s0 + (size_t)b * D + 4 * c4)
                              : *(const float4*)(sin + (size_t)(row0 - 1) * D + 4 * c4);
                } else if (r - 1 < len) {
                    v = *(const float4*)(sin + (size_t)(row0 + r - 1) * D + 4 * c4);
                }
                *(float4*)(hs + r * C::HS + 4 * c4) = v;
            }
            constexpr int QX = DX / 4;
            for (int idx = tid; idx < L * QX; idx += C::NT) {
                const int r = idx / QX, c4 = idx % QX;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < len) v = *(const float4*)(a.x + (size_t)(row0 + r) * DX + 4 * c4);
                *(float4*)(xs + r * C::XS + 4 * c4) = v;
            }
        }
        __syncthreads();

        // ---- gates by MFMA, then residual and leaves, per 16-step block ----
        float la[C::MB][4], lc[C::MB][4];
        uint32_t rmax = 0;
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            floatx4 az, ar, aq, an;
            wg.gemm(hs + (mb * 16 + u) * C::HS, xs + (mb * 16 + u) * C::XS, g, az, ar, aq, an);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tl = mb * 16 + 4 * g + i;      // step index within the tile
                const float h = hs[tl * C::HS + j];      // s_{t-1}
                const float sc = hs[(tl + 1) * C::HS + j];   // s_t (current iterate)
                const GruPoint p = gru_point(az[i], ar[i], aq[i], an[i], wg.b_z, wg.b_r,
                                             wg.b_n, wg.b_hn);
                const float f = (1.f - p.z) * p.n + p.z * h;
                const float res = sc - f;
                const float e = (1.f - p.z) * (1.f - p.n * p.n);
                float dg = p.z + (h - p.n) * p.z * (1.f - p.z) * wg.dUz + e * p.r * wg.dUn
                         + e * p.q * p.r * (1.f - p.r) * wg.dUr;
                const bool valid = tl < len;
                if (first && tl == 0) dg = 0.f;
                la[mb][i] = valid ? dg : 1.f;
                lc[mb][i] = valid ? -res : 0.f;

                if (valid) rmax = max(rmax, absbits(res));
            }
        }

        // ---- scan inside the tile ----
        // lane-local over the 4 steps of each block
        float Ra = 1.f, Rc = 0.f;      // composed map of all blocks before the current one
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            float pa = 1.f, pc = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                pa = la[mb][i] * pa;
                pc = la[mb][i] * pc + lc[mb][i];
                la[mb][i] = pa;
                lc[mb][i] = pc;
            }
            // inclusive scan of lane aggregates over the 4 lane groups of a unit
            float Ia = pa, Ic = pc;
            {
                const float qa = __shfl_up(Ia, 16), qc = __shfl_up(Ic, 16);
                if (g >= 1) { Ic = Ia * qc + Ic; Ia = Ia * qa; }
            }
            {
                const float qa = __shfl_up(Ia, 32), qc = __shfl_up(Ic, 32);
                if (g >= 2) { Ic = Ia * qc + Ic; Ia = Ia * qa; }
            }
            float Ea = __shfl_up(Ia, 16), Ec = __shfl_up(Ic, 16);
            if (g == 0) { Ea = 1.f; Ec = 0.f; }
            const float Ta = __shfl(Ia, 48 + u), Tc = __shfl(Ic, 48 + u);
            // prefix of this lane group's start = E o R
            const float Xa = Ea * Ra, Xc = Ea * Rc + Ec;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                lc[mb][i] = la[mb][i] * Xc + lc[mb][i];
                la[mb][i] = la[mb][i] * Xa;
            }
            Rc = Ta * Rc + Tc;
            Ra = Ta * Ra;
        }

        // ---- decoupled look-back for the carry-in Delta_{t0-1} of unit j ----
        const float din = lookback4(aggc, inclc, tile, tile - lt, D, j, g, u, Ra, Rc,
                                    &a.ctrl->error);

        // The next tile is claimed only now.  A claim made earlier would hand a tile to a
        // workgroup that is still blocked in this look-back, and every later tile of that
        // sequence would wait on it; claimed this late, its geometry is read while the new
        // iterate is written.
        if (tid == 0)
            fetch_tile(a.ctrl, a.tiles, a.seq, a.ntiles,
                       (int)atomicAdd(&a.ctrl->tile_counter, 1u), tnext[(it + 1) & 1]);

        // ---- new iterate (kept in lc), overflow guard ----
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = hs[(mb * 16 + 4 * g + i + 1) * C::HS + j] + (la[mb][i] * din + lc[mb][i]);
                lc[mb][i] = v;
                const int tl = mb * 16 + 4 * g + i;
                const bool bad = (tl < len) && !(fabsf(v) <= reset_abs);
                const uint64_t m = __ballot(bad);
                if (u == 0 && ((m >> (16 * g)) & 0xFFFFull)) rowbad[tl] = 1;
            }
        // residual max of the current iterate, one atomic per wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) atomicMax(&a.seq[b].maxr, rmax);
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tl = mb * 16 + 4 * g + i;
                if (tl < len) sout[(size_t)(row0 + tl) * D + j] = rowbad[tl] ? 0.f : lc[mb][i];
            }
        if (w == 0) {
            int nb = 0;
#pragma unroll
            for (int base = 0; base < L; base += 64) {
                const int t = base + l;
                const bool bad = (t < L) && rowbad[t];
                nb += __popcll(__ballot(bad));
            }
            if (l == 0 && nb) atomicAdd(&a.seq[b].resets_pending, nb);
        }
        __syncthreads();
        for (int t = tid; t < L; t += C::NT) rowbad[t] = 0;
    }
}

// ---- host driver ------------------------------------------------------------------------

struct GruQLayout {
    IterState st;
    float* salt;
    uint64_t* agg[2];
    uint32_t* incl[2];
    size_t bytes;
};

static GruQLayout gruq_layout(void* ws, int D, const HostBatch& hb, int ntiles) {
    Carver c(ws);
    GruQLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles);
    lay.salt = c.take<float>((size_t)hb.N * D);
    for (int p = 0; p < 2; ++p) lay.agg[p] = c.take<uint64_t>((size_t)ntiles * D);
    for (int p = 0; p < 2; ++p) lay.incl[p] = c.take<uint32_t>((size_t)ntiles * D);
    lay.bytes = c.bytes();
    return lay;
}

__global__ void fill_sentinels_kernel(uint64_t* agg, uint32_t* incl, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        agg[i] = kSent64;
        incl[i] = kSent32;
    }
}

typedef void (*GruQKernel)(GruQArgs);

template <int D, int DX, int L>
static void gruq_get(GruQKernel* k, int* nt) {
    *k = gru_quasi_iter_kernel<D, DX, L>;
    *nt = GruQ<D, DX, L>::NT;
}

static bool gruq_lookup(int D, int Dx, int L, GruQKernel* k, int* nt) {
#define PN_GQ(d, dx, ll) if (D == d && Dx == dx && L == ll) { gruq_get<d, dx, ll>(k, nt); return true; }
#define PN_GQL(d, dx) PN_GQ(d, dx, 32) PN_GQ(d, dx, 64) PN_GQ(d, dx, 128)
    PN_GQL(64, 32) PN_GQL(48, 24) PN_GQL(32, 16) PN_GQL(16, 8) PN_GQL(16, 16) PN_GQL(64, 64)
    PN_GQL(32, 32) PN_GQL(48, 48) PN_GQL(64, 16) PN_GQL(32, 8)
#undef PN_GQL
#undef PN_GQ
    return false;
}

bool gru_quasi_supported(int D, int Dx) {
    GruQKernel k;
    int nt;
    return gruq_lookup(D, Dx, 64, &k, &nt);
}

int gru_quasi_tile(int D, int Dx, const pn_opts& o) {
    if (o.tile == 32 || o.tile == 64 || o.tile == 128) return o.tile;
    return 64;
}

size_t gru_quasi_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    const int L = gru_quasi_tile(D, Dx, o);
    const int ntiles = tile_starts(hb, L)[hb.B];
    return gruq_layout(nullptr, D, hb, ntiles).bytes;
}

pn_status gru_quasi_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                            const float* s0, float* s, const pn_opts& o, void* ws,
                            hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    const int D = cd.D, Dx = cd.Dx;
    const int L = gru_quasi_tile(D, Dx, o);
    GruQKernel kern;
    int nt;
    if (!gruq_lookup(D, Dx, L, &kern, &nt)) {
        set_error("GRU quasi-DEER not built for D=%d Dx=%d tile=%d", D, Dx, L);
        return PN_ERR_UNSUPPORTED;
    }
    const std::vector<int32_t> ts = tile_starts(hb, L);
    const int ntiles = ts[hb.B];
    GruQLayout lay = gruq_layout(ws, D, hb, ntiles);
    const int max_iters = o.max_iters > 0 ? o.max_iters : (int)std::max<int64_t>(1, hb.Tmax);
    PN_TRY(init_iter_state(lay.st, hb, ts, L, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream));
    if (ntiles > 0) {
        const size_t n = (size_t)ntiles * D;
        hipLaunchKernelGGL(fill_sentinels_kernel, dim3((unsigned)std::min<size_t>(4096, (n + 255) / 256)),
                           dim3(256), 0, stream, lay.agg[0], lay.incl[0], n);
        PN_HIP(hipGetLastError());
    }
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, nt, 0) != hipSuccess || occ < 1)
        occ = 1;
    const int grid = std::max(1, std::min(ntiles, cu_count() * occ));

    GruQArgs args;
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
    args.tiles = lay.st.tiles;
    args.B = hb.B;
    args.ntiles = ntiles;

    auto one_iter = [&](hipStream_t st) {
        prof_launch("gru_quasi_iter", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), 0, s2, args);
        });
        launch_decide(lay.st, hb.B, st);
    };
    std::vector<uintptr_t> key = {0x6751u, (uintptr_t)kern, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)cd.params,
                                  (uintptr_t)ws, (uintptr_t)hb.B, (uintptr_t)ntiles};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    int derr = 0;
    PN_TRY(finish_iterations(lay.st, hb, D, sizeof(float), s, lay.salt, stream, info, all_conv,
                             &derr));
    if (derr) {
        set_error("look-back watchdog expired in the GRU quasi-DEER scan");
        return PN_ERR_INTERNAL;
    }
    return PN_OK;
}

}  // namespace pn
