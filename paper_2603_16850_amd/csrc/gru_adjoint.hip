// Exact adjoint of the GRU recurrence by iterated reverse quasi-Newton scans, then the
// parameter, input and initial-state gradients.
//
// Ch. 3 ("Training and the backwards pass"): backpropagation through s_t = f(s_{t-1}, x_t) is
// the reverse-time linear recurrence lambda_t = g_t + A_{t+1}^T lambda_{t+1} (lambda_T = g_T),
// and the thesis recommends an exact backward pass for quasi-DEER obtained by iterating
// reverse scans whose transition is diag(A_t) while the true A_{t+1}^T lambda_{t+1} enters
// through a vector-Jacobian product.  Written like the forward Newton step (eq. lin_rr):
//   rho_t   = lambda_t - g_t - A_{t+1}^T lambda_{t+1}             (exact VJP residual)
//   Delta_t = diag(A_{t+1}) Delta_{t+1} - rho_t,  Delta_{T+1} = 0  (reverse diagonal scan)
//   lambda <- lambda + Delta,
// repeated until max |rho| <= tol * max(1, max |g|) for the sequence.  Since the recurrence is
// linear in lambda, the same global-convergence argument as Prop. global_convergence bounds it
// by T iterations.  Then (eq. unrolled_bwds)
//   dL/dtheta = sum_t (df_t/dtheta)^T lambda_t,  dL/dx_t = (df_t/dx_t)^T lambda_t,
//   dL/ds_0 = A_1^T lambda_1.
//
// Kernels: prep (gate values at the solution, once), local pass (one per adjoint iteration:
// VJP on FP32 MFMA + reverse diagonal scan over groups of tiles taken from the sequence end)
// with the carry pass over the group maps, grad (per-workgroup partial parameter gradients
// on MFMA, dx), reduce, gs0.
#include <algorithm>
#include <cmath>

#include "carry.hpp"
#include "gru_common.hpp"
#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

template <int D, int DX, int L>
struct GruA {
    static constexpr int NW = D / 16;
    static constexpr int NT = 64 * NW;
    static constexpr int HS = D + 4;
    static constexpr int XS = DX + 4;
    static constexpr int PS = 3 * D + 4;    // row stride of the VJP operand tile
    static constexpr int MB = L / 16;
    static constexpr int DXP = (DX + 15) / 16 * 16;
};

struct GruAdjArgs {
    const float* x;
    const float* s0;
    const float* s;
    const float* gs;
    const float* params;
    float* gates;            // [N][4][D]: alpha, beta, gamma, z at the solution (the VJP
                             // operands of every adjoint iteration)
    float* eps;              // [N][D]: (1 - z)(1 - n^2) at the solution (parameter gradients)
    float* lam;              // [N][D] adjoint iterate: iteration k writes lambda^(k) on the rows
                             // of the sequences it updates, so it ends holding each
                             // sequence's final iterate
    float* mu[2];            // ping-pong [N][D]: mu^(k) = lambda^(k-1) + lc^(k-1), the previous
                             // iterate plus the carry-free part of its update; iteration k reads
                             // mu[k & 1] (mu^(0) = g is read from gs) and writes mu[(k + 1) & 1]
    float* gprod;            // [ngroups][D] product of the scan transitions over each group
                             // (written by iteration 0: the transitions diag(A_{t+1}) are those
                             // of the solution and do not change between iterations)
    float2* gagg;            // [ngroups][D] group maps
    const float* gcarry;     // [ngroups][D] carry into every group (previous iteration)
    float* gmax;             // [B] max |g| per sequence (as float bits)
    uint32_t* cmax;          // [ntiles][D / 16] max |g| per tile and wave (float bits)
    Ctrl* ctrl;
    SeqState* seq;
    const int64_t* offsets;
    const int32_t* tile_start;
    const TileInfo* tiles;   // by slot (reverse scan: slots from the sequence end)
    const GroupInfo* groups;
    int ngroups;
    int B;
    int ntiles;
    uint32_t* grmax;         // [ngroups][D / 16] scaled residual max of each group's waves
    int freeze;              // converged-prefix skipping (in scan order, from the sequence end)
    float dscale;            // damping of the reverse scan's transition (as the forward)
    int clip;
    float clo, chi;
    float* part;             // [grid][P] per-workgroup parameter-gradient partials
    float* gx;
    float* gs0;
    float* gparams;
};

// ---- prep: gate values at the solution, max |g| -------------------------------------------
// Tiles are processed with their inputs double-buffered in LDS: the s rows (h of every step),
// the x rows and the g rows of the next tile are copied from HBM straight into LDS
// (global_load_lds, 16 B per lane) while the current tile is computed.
template <int D, int DX, int L>
__global__ void __launch_bounds__(64 * (D / 16))
__attribute__((amdgpu_waves_per_eu(L <= 32 && D + DX <= 72 ? 3 : 2,
                                   L <= 32 && D + DX <= 72 ? 3 : 2)))
gru_adj_prep_kernel(GruAdjArgs a) {
    using C = GruA<D, DX, L>;
    constexpr int BUF = L * (2 * D + DX);        // [h rows | x rows | g rows], unpadded
    __shared__ __attribute__((aligned(16))) float stg0[BUF];
    __shared__ __attribute__((aligned(16))) float stg1[BUF];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, u = l & 15;
    const int j = 16 * w + u;
    GruGates<D, DX> wg;
    wg.load(a.params, j, g);
    // nbytes (a multiple of 16) from src to LDS dst, 1 KB per wave instruction
    auto bulk = [&](float* dst, const float* src, int nbytes) {
        for (int c = w; c * 1024 < nbytes; c += C::NW) {
            const int off = c * 1024 + 16 * l;
            if (off < nbytes)
                __builtin_amdgcn_global_load_lds(
                    (const void*)((const char*)src + off),
                    (__attribute__((address_space(3))) void*)((char*)dst + c * 1024), 16, 0, 0);
        }
    };
    // row r of the h block is s_{t0 + r - 1}; a sequence's first step takes s0
    auto issue = [&](const TileInfo& ti, float* buf) {
        const int hr = (ti.flags & kTileTimeFirst) ? 1 : 0;
        if (hr) bulk(buf, a.s0 + (size_t)ti.b * D, D * 4);
        bulk(buf + hr * D, a.s + (size_t)(ti.row0 - 1 + hr) * D, (ti.len - hr) * D * 4);
        bulk(buf + L * D, a.x + (size_t)ti.row0 * DX, ti.len * DX * 4);
        bulk(buf + L * (D + DX), a.gs + (size_t)ti.row0 * D, ti.len * D * 4);
    };
    // the tile table is not written while the kernel runs: read it through the scalar cache
    // (s_load), whose counter is not the one the copies into LDS advance
    using CTile = const __attribute__((address_space(4))) TileInfo;
    CTile* ctiles = (CTile*)a.tiles;
    auto tiles = [&](int i) {
        TileInfo r;
        r.slot = ctiles[i].slot;
        r.b = ctiles[i].b;
        r.len = ctiles[i].len;
        r.flags = ctiles[i].flags;
        r.row0 = ctiles[i].row0;
        r.gslot = ctiles[i].gslot;
        r.hgslot = ctiles[i].hgslot;
        return r;
    };
    int tile = blockIdx.x;
    if (tile >= a.ntiles) return;
    TileInfo ti = tiles(tile);
    issue(ti, stg0);
    TileInfo tn{};
    if (tile + (int)gridDim.x < a.ntiles) tn = tiles(tile + gridDim.x);
    // one tile: its inputs are in `hs`, the next tile's go to `nb` meanwhile.  The two buffers
    // are distinct LDS objects and every use names one of them statically, so that the
    // compiler can tell the reads of one from the copies into the other.
    auto one = [&](const float* hs, float* nb) {
        const float* xs = hs + L * D;
        const float* gsl = xs + L * DX;
        __builtin_amdgcn_s_waitcnt(0x0F70);       // vmcnt(0): this wave's copies have landed
        __syncthreads();                          // every wave's; the other buffer is free
        float2 xt[C::MB];                         // x row tails, read before the next copies
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) xt[mb] = wg.xtail_of(xs + (mb * 16 + u) * DX, g);
        if (tile + (int)gridDim.x < a.ntiles) issue(tn, nb);
        const int len = ti.len;
        const int64_t row0 = ti.row0;
        int o_a = u * D, o_x = u * DX, o_own = 4 * g * D + j;
        asm volatile("" : "+v"(o_a), "+v"(o_x), "+v"(o_own));
        uint32_t gm = 0;
#pragma unroll
        for (int mb = 0; mb < C::MB; ++mb) {
            floatx4 az, ar, aq, an;
            wg.gemm_xtail(hs + mb * 16 * D + o_a, xs + mb * 16 * DX + o_x, xt[mb], g, az, ar, aq,
                          an);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int tl = mb * 16 + 4 * g + i;
                if (tl >= len) continue;
                const GruPoint p = gru_point(az[i], ar[i], aq[i], an[i], wg.b_z, wg.b_r, wg.b_n,
                                             wg.b_hn);
                const float h = hs[mb * 16 * D + i * D + o_own];
                const float gv = gsl[mb * 16 * D + i * D + o_own];
                const float e = (1.f - p.z) * (1.f - p.n * p.n);
                const size_t row = (size_t)(row0 + tl);
                float* gr = a.gates + row * 4 * D;
                const float al = (h - p.n) * p.z * (1.f - p.z);
                const float be = e * p.r;
                const float ga = e * p.q * p.r * (1.f - p.r);
                gr[0 * D + j] = al;
                gr[1 * D + j] = be;
                gr[2 * D + j] = ga;
                gr[3 * D + j] = p.z;
                a.eps[row * D + j] = e;
                gm = max(gm, absbits(gv));
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) gm = max(gm, (uint32_t)__shfl_xor((int)gm, off));
        if (l == 0) a.cmax[(size_t)tile * C::NW + w] = gm;
        ti = tn;
        if (tile + 2 * (int)gridDim.x < a.ntiles) tn = tiles(tile + 2 * gridDim.x);
        tile += gridDim.x;
    };
    while (true) {
        one(stg0, stg1);
        if (tile >= a.ntiles) break;
        one(stg1, stg0);
        if (tile >= a.ntiles) break;
    }
}

// max |g| of every sequence from the maxima of its tiles (one workgroup per sequence)
template <int NW>
__global__ void __launch_bounds__(256) gru_adj_gmax_kernel(GruAdjArgs a) {
    __shared__ uint32_t red[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    uint32_t m = 0;
    for (int k = a.tile_start[b] * NW + tid; k < a.tile_start[b + 1] * NW; k += 256)
        m = max(m, a.cmax[k]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) ((uint32_t*)a.gmax)[b] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// ---- one adjoint iteration ------------------------------------------------------------------
// Reverse scan of one tile's steps held in the MFMA output layout (lane (u, g) of a wave holds
// rows 16 mb + 4 g + i of its column), later steps first, composed with the map (Ra, Rc) of the
// group's steps scanned before the tile.  On entry sa, sc hold every step's own map
// Delta_t = sa Delta_{t+1} + sc; on return they hold the map from the Delta entering the group
// to Delta_t, and (Ra, Rc) the map of the group's steps scanned so far, this tile included.
// With WC false only the multiplicative parts are formed (sc and Rc are left alone).
template <int MB, bool WC>
PN_DEV void adj_tile_scan(float (&sa)[MB][4], float (&sc)[MB][4], float& Ra, float& Rc, int g,
                          int u) {
#pragma unroll
    for (int mb = MB - 1; mb >= 0; --mb) {
        float pa = 1.f, pc = 0.f;
#pragma unroll
        for (int i = 3; i >= 0; --i) {
            if (WC) {
                pc = sa[mb][i] * pc + sc[mb][i];
                sc[mb][i] = pc;
            }
            pa = sa[mb][i] * pa;
            sa[mb][i] = pa;
        }
        float Ia = pa, Ic = pc;
        {
            const float qa = __shfl_down(Ia, 16);
            const float qc = WC ? __shfl_down(Ic, 16) : 0.f;
            if (g <= 2) {
                if (WC) Ic = Ia * qc + Ic;
                Ia = Ia * qa;
            }
        }
        {
            const float qa = __shfl_down(Ia, 32);
            const float qc = WC ? __shfl_down(Ic, 32) : 0.f;
            if (g <= 1) {
                if (WC) Ic = Ia * qc + Ic;
                Ia = Ia * qa;
            }
        }
        float Ea = __shfl_down(Ia, 16), Ec = WC ? __shfl_down(Ic, 16) : 0.f;
        if (g == 3) { Ea = 1.f; Ec = 0.f; }
        const float Ta = __shfl(Ia, u), Tc = WC ? __shfl(Ic, u) : 0.f;
        const float Xa = Ea * Ra, Xc = Ea * Rc + Ec;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (WC) sc[mb][i] = sa[mb][i] * Xc + sc[mb][i];
            sa[mb][i] = sa[mb][i] * Xa;
        }
        if (WC) Rc = Ta * Rc + Tc;
        Ra = Ta * Ra;
    }
}

// One Newton iteration of the adjoint over groups of tiles.  With la_t the product of the
// scan's transitions from step t to the group's first scanned step and lc^(k)_t the scan of
// -rho^(k) inside the group (the update for a zero carry), iteration k forms
//   lambda^(k)_t = mu^(k)_t + la_t carry_g     (carry_g: the carry into the group, from the
//                                               previous carry pass; reset guard per row)
//   mu^(k+1)_t  = lambda^(k)_t + lc^(k)_t
// and writes lambda^(k) and mu^(k+1).  la is recomputed in every iteration from the gate rows
// that the VJP reads anyway (diag(A_{t+1})_j = z + alpha U_z[j][j] + beta U_n[j][j]
// + gamma U_r[j][j]), so per step an iteration reads mu, the gate row of the successor step and
// g, and writes lambda and mu.
template <int D, int DX, int L>
__global__ void __launch_bounds__(64 * (D / 16))
__attribute__((amdgpu_waves_per_eu(L <= 32 ? 3 : 2, L <= 32 ? 3 : 2)))
gru_adj_local_kernel(GruAdjArgs a) {
    using C = GruA<D, DX, L>;
    constexpr int MB = C::MB;
    __shared__ __attribute__((aligned(16))) float ps[L * C::PS];
    __shared__ __attribute__((aligned(16))) float lst[(L + 1) * C::HS];   // lambda rows t0 .. t0+L
    __shared__ int rowbad[L + 1];

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k = a.ctrl->iter;
    const bool fuse = k > 0;
    const float reset_abs = a.ctrl->reset_abs;
    const float* __restrict__ mu_in = fuse ? a.mu[k & 1] : a.gs;     // mu^(k) (mu^(0) = g)
    float* __restrict__ mu_out = a.mu[(k + 1) & 1];                   // mu^(k+1)
    float* __restrict__ lam = a.lam;

    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, u = l & 15;
    const int j = 16 * w + u;

    // B operands of [U_z; U_n; U_r] (3D x D), column j, same K permutation as GruGates
    const float* U = a.params + 3 * D * DX;
    float bu[3 * D / 16][4];
#pragma unroll
    for (int kb = 0; kb < 3 * D / 16; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = 16 * kb + 4 * g + i;     // 0..3D-1 over (z | n | r) blocks
            const int mat = kk / D, ii = kk % D;
            const int base = (mat == 0 ? 0 : (mat == 1 ? 2 : 1)) * D;   // U_z, U_n, U_r rows
            bu[kb][i] = U[(base + ii) * D + j];
        }
    const float dUz = U[(0 * D + j) * D + j], dUr = U[(1 * D + j) * D + j],
                dUn = U[(2 * D + j) * D + j];

    for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
        const GroupInfo gr = a.groups[gi];
        if (a.seq[gr.b].status != kActive) continue;     // same on every thread
        const int b = gr.b;
        // converged-prefix skipping in scan order (the sequence's last groups in time first):
        // the carry into a group frozen by the last carry pass is zero, so its iterate is
        // mu^(k); it goes into lambda and into both mu buffers once, and the group is skipped
        // from then on
        bool halo_frozen = false;
        if (a.freeze) {
            const int li = gi - gr.gfirst, nf = a.seq[b].frozen;
            if (li < nf) {
                if (li >= a.seq[b].frozen_prev) {
                    const TileInfo t0 = a.tiles[gr.tile0 + gr.ntl - 1], t1 = a.tiles[gr.tile0];
                    const int64_t e0 = t0.row0 * (D / 4), e1 = (t1.row0 + t1.len) * (D / 4);
                    for (int64_t e = e0 + tid; e < e1; e += C::NT) {
                        const float4 v = ((const float4*)mu_in)[e];
                        ((float4*)lam)[e] = v;
                        ((float4*)mu_out)[e] = v;
                    }
                }
                continue;
            }
            halo_frozen = li == nf && nf > 0;    // the row after the group does not move
        }
        const float gscale = 1.f / fmaxf(1.f, a.gmax[b]);
        float Pa = 1.f, Pc = 0.f;        // map of the group's tiles before the current one
        uint32_t rmax = 0;
        TileInfo tnext = a.tiles[gr.tile0];
        for (int kt = 0; kt < gr.ntl; ++kt) {
            const TileInfo ti = tnext;                     // scan order: later tiles first
            if (kt + 1 < gr.ntl) tnext = a.tiles[gr.tile0 + kt + 1];   // read ahead
            const int len = ti.len;
            const int64_t row0 = ti.row0;
            const bool first = (ti.flags & kTileScanFirst) != 0;   // tile at the sequence end
            // one past the last row that has a successor step inside the sequence
            const int64_t rend = first ? row0 + len : row0 + L + 1;
            const bool halo_moves = fuse && !first && !(kt == 0 && halo_frozen);
            // carry terms of column j: into the own group, into the halo row's group, and the
            // transition product from the halo row to its group's first scanned step (the
            // group's earlier tiles for kt > 0: Pa; the whole previous group for kt = 0)
            float cown = 0.f, chalo = 0.f, lah = 0.f;
            if (fuse) {      // in flight together with the staging loads below
                cown = a.gcarry[(size_t)ti.gslot * D + j];
                if (halo_moves) {
                    chalo = a.gcarry[(size_t)ti.hgslot * D + j];
                    lah = kt == 0 ? a.gprod[(size_t)ti.hgslot * D + j] : Pa;
                }
            }
            __syncthreads();                 // LDS of the previous tile consumed
            for (int r = tid; r <= L; r += C::NT) rowbad[r] = 0;
            constexpr int Q = D / 4;
            static_assert(C::NT % Q == 0, "column per thread");
            // Lane offsets into the LDS tiles and the step rows, formed anew for every tile
            // (hidden from the optimiser): hoisted out of the loops, one precomputed address
            // per (row, operand) would stay live across the whole group loop.
            int o_own = 4 * g * C::HS + j;           // lst: own row 4 g, column j
            int o_gate = 4 * g * C::PS + j;          // ps: gate row of the step after row 4 g
            int o_arow = u * C::PS + 4 * g;          // ps: VJP operand row u
            int o_lrow = (u + 1) * C::HS + 4 * g;    // lst: lambda row u + 1
            int o_row = 4 * g * D + j;               // [N][D] arrays: own row 4 g, column j
            int o_grow = 16 * g * D + j;             // [N][4][D] gate rows: row 4 g, column j
            int o_st = (tid / Q) * C::HS + 4 * (tid % Q);   // staging item 0 in lst
            int o_sg = (tid / Q) * D + 4 * (tid % Q);       // staging item 0 in [N][D]
            asm volatile("" : "+v"(o_own), "+v"(o_gate), "+v"(o_arow), "+v"(o_lrow), "+v"(o_row),
                              "+v"(o_grow), "+v"(o_st), "+v"(o_sg));
            // The gate planes (alpha, beta, gamma) of rows row0 + 1 .. row0 + L go straight
            // from HBM into ps (row r - 1 for row row0 + r), one 3D-float row per instruction of
            // 3D / 4 lanes (16 B each, lane i to byte 16 i of the row), issued before the other
            // loads so that all are in flight together and no register holds them.  Rows past
            // the sequence's last row with a successor read that row instead: their lambda row
            // is zero, so the products formed from them vanish.
            {
                const int64_t last = rend - 1;
                for (int r = w + 1; r <= L; r += C::NW) {
                    const int64_t nr = min(row0 + r, last);
                    if (l < 3 * D / 4)
                        __builtin_amdgcn_global_load_lds(
                            (const void*)(a.gates + (size_t)nr * 4 * D + 4 * l),
                            (__attribute__((address_space(3))) void*)(ps + (r - 1) * C::PS), 16,
                            0, 0);
                }
            }
            // mu rows row0 .. row0 + L (item (r, c4): mu_{t0+r}[4 c4 .. 4 c4 + 3]; row L, when
            // the tile is not the sequence's last, belongs to the next tile in time); item q of
            // a thread is row tid / Q + q NT / Q
            constexpr int NI = ((L + 1) * Q + C::NT - 1) / C::NT;
            constexpr int RQ = C::NT / Q;
            const float* mrow = mu_in + (size_t)row0 * D + o_sg;
            float4 vl[NI];
#pragma unroll
            for (int q = 0; q < NI; ++q) {
                const int idx = tid + q * C::NT;
                vl[q] = (idx < (L + 1) * Q && row0 + idx / Q < rend)
                            ? *(const float4*)(mrow + q * RQ * D)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
            }
            // z of the successor step of every own row (g_t is loaded later, a block ahead)
            float zv[MB][4];
            const float* zrow = a.gates + (size_t)(row0 + 1) * 4 * D + 3 * D + o_grow;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;
                    zv[mb][i] = tl < len && row0 + tl + 1 < rend
                                    ? zrow[(mb * 16 + i) * 4 * D] : 0.f;
                }
#pragma unroll
            for (int q = 0; q < NI; ++q) {
                const int idx = tid + q * C::NT;
                if (idx < (L + 1) * Q) *(float4*)(lst + o_st + q * RQ * C::HS) = vl[q];
            }
            // the gate rows were issued before the other loads, so they have landed once those
            // have; the explicit wait also covers them for the barrier
            __builtin_amdgcn_s_waitcnt(0x0F70);              // vmcnt(0)
            __syncthreads();

            // transitions dg_t = diag(A_{t+1}) of the own rows (damped or clipped as in the
            // forward; a row without a successor has A = 0, an invalid row the identity), from
            // the gate rows in ps; formed twice (for the update and for the scan) rather than
            // kept in registers
            auto transitions = [&](float (&dg)[MB][4]) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int tl = mb * 16 + 4 * g + i;
                        const float* pr = ps + o_gate + (mb * 16 + i) * C::PS;   // step t + 1
                        const bool has_next = tl < len && row0 + tl + 1 < rend;
                        float d = has_next ? zv[mb][i] + pr[0] * dUz + pr[D] * dUn +
                                                 pr[2 * D] * dUr
                                           : 0.f;
                        d *= a.dscale;
                        if (a.clip) d = fminf(fmaxf(d, a.clo), a.chi);
                        dg[mb][i] = tl < len ? d : 1.f;
                    }
            };
            float la[MB][4], lc[MB][4];

            if (fuse) {
                // ---- lambda^(k) = mu^(k) + la carry, with the reset guard ----
                float ra = Pa, rc = 0.f;
                transitions(la);
                adj_tile_scan<MB, false>(la, lc, ra, rc, g, u);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int tl = mb * 16 + 4 * g + i;
                        if (tl < len) {
                            float* lp = lst + o_own + (mb * 16 + i) * C::HS;
                            const float v = *lp + la[mb][i] * cown;
                            *lp = v;
                            if (!(fabsf(v) <= reset_abs)) rowbad[tl] = 1;
                        }
                    }
                if (g == 0 && halo_moves) {
                    float* lp = lst + L * C::HS + j;
                    const float v = *lp + lah * chalo;
                    *lp = v;
                    if (!(fabsf(v) <= reset_abs)) rowbad[L] = 1;
                }
                __syncthreads();
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int tl = mb * 16 + 4 * g + i;
                        if (tl < len && rowbad[tl]) lst[o_own + (mb * 16 + i) * C::HS] = 0.f;
                    }
                if (g == 0 && halo_moves && rowbad[L]) lst[L * C::HS + j] = 0.f;
                if (tid < 64) {
                    int nb = 0;
                    for (int base = 0; base < L; base += 64) {
                        const int r = base + tid;
                        nb += __popcll(__ballot(r < len && rowbad[r]));
                    }
                    if (tid == 0 && nb) atomicAdd(&a.seq[b].resets_pending, nb);
                }
                __syncthreads();
            }

            // ---- VJP, residual rho^(k) and its scan inside the tile ----
            // g_t of a 16-step block, loaded one block ahead so that its latency hides behind
            // the previous block's MFMAs
            float gtc[4], gtn[4];
            const float* grow = a.gs + (size_t)row0 * D + o_row;
            auto load_g = [&](int mb, float* gt) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;
                    gt[i] = tl < len ? grow[(mb * 16 + i) * D] : 0.f;
                }
            };
            load_g(0, gtc);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                if (mb + 1 < MB) load_g(mb + 1, gtn);
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                // VJP operand row (alpha, beta, gamma)_{t+1} * lambda_{t+1} of step t = row
                // mb * 16 + u, formed from the gate rows in ps and the lambda row in lst
                const float* prow = ps + o_arow + mb * 16 * C::PS;
                const float* lrow = lst + o_lrow + mb * 16 * C::HS;
#pragma unroll
                for (int kb = 0; kb < 3 * D / 16; ++kb) {
                    const float4 g4 = *(const float4*)(prow + 16 * kb);
                    const float4 l4 = *(const float4*)(lrow + 16 * (kb % (D / 16)));
                    acc = mfma16x4(g4.x * l4.x, bu[kb][0], acc);
                    acc = mfma16x4(g4.y * l4.y, bu[kb][1], acc);
                    acc = mfma16x4(g4.z * l4.z, bu[kb][2], acc);
                    acc = mfma16x4(g4.w * l4.w, bu[kb][3], acc);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;
                    const bool valid = tl < len;
                    const float* lp = lst + o_own + (mb * 16 + i) * C::HS;
                    const float lam_t = lp[0];
                    // (A_{t+1}^T lambda_{t+1})_j = z_j lambda_j + [U_z; U_n; U_r]^T part (MFMA)
                    const float vjp = zv[mb][i] * lp[C::HS] + acc[i];
                    const float rho = lam_t - gtc[i] - vjp;
                    lc[mb][i] = valid ? -rho : 0.f;
                    if (valid) rmax = max(rmax, absbits(rho * gscale));
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) gtc[i] = gtn[i];
            }
            transitions(la);
            adj_tile_scan<MB, true>(la, lc, Pa, Pc, g, u);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;
                    if (tl < len) {
                        const size_t e = (size_t)row0 * D + o_row + (mb * 16 + i) * D;
                        const float lam_t = lst[o_own + (mb * 16 + i) * C::HS];
                        lam[e] = lam_t;
                        mu_out[e] = lam_t + lc[mb][i];
                    }
                }
        }
        if (g == 0) {
            a.gagg[(size_t)gi * D + j] = make_float2(Pa, Pc);
            if (!fuse) a.gprod[(size_t)gi * D + j] = Pa;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) {
            atomicMax(&a.seq[b].maxr, rmax);
            if (a.freeze) a.grmax[(size_t)gi * C::NW + w] = rmax;
        }
    }
}

// ---- gradients: per-workgroup partials of dW, dU, db on MFMA; dx rows --------------------
// Output tiles of the parameter GEMMs (16 x 16 each): for each gate block G in {z, r, n}
// and unit block ib:  dU_G[ib] x (h blocks)  and  dW_G[ib] x (x blocks).  dU_n pairs with
// delta_q = beta * lambda, dW_n with delta_n = eps * lambda.  Wave w owns unit block ib = w
// (D / 16 waves, D / 16 blocks): per 4-step K slice it reads its four delta operands and the
// h / x operands once and issues all 3 (HB + XB) MFMAs of its tiles.
template <int D, int DX>
struct GradTiles {
    static constexpr int IB = D / 16;
    static constexpr int HB = D / 16;
    static constexpr int XB = (DX + 15) / 16;
    static constexpr int PER_GATE = IB * (HB + XB);
    static constexpr int TOTAL = 3 * PER_GATE;
};

// L: steps per pass; the tile table has tiles of LT = SUB * L steps, each done in SUB passes.
template <int D, int DX, int L, int SUB>
__global__ void __launch_bounds__(64 * (D / 16)) __attribute__((amdgpu_waves_per_eu(2, 2)))
gru_adj_grad_kernel(GruAdjArgs a) {
    using C = GruA<D, DX, L>;
    using TT = GradTiles<D, DX>;
    constexpr int NW = C::NW;
    constexpr int DS = 4 * D + 4;        // delta tile stride: [dz | dr | dq | dn]
    constexpr int XSP = C::DXP + 4;
    constexpr int WT = 3 * D + 4;        // row stride of [W_z;W_r;W_n]^T in LDS
    __shared__ __attribute__((aligned(16))) float dl[L * DS];
    __shared__ __attribute__((aligned(16))) float hsm[L * C::HS];
    __shared__ __attribute__((aligned(16))) float xsm[L * XSP];
    __shared__ __attribute__((aligned(16))) float wst[C::DXP * WT];  // [W_z;W_r;W_n]^T, for dx

    static_assert(TT::IB == NW, "one unit block per wave");
    constexpr int HB = TT::HB, XB = TT::XB;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, u = l & 15;
    floatx4 acc[3][HB + XB];                // [gate][h blocks | x blocks] of unit block w
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int c = 0; c < HB + XB; ++c) acc[q][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    // bias partial of (delta column bcol, unit bu): threads cover the 4 D bias entries
    // [z | r | n | q-part of n]: entry e = tid, tid + NT, ... reads delta column {0, D, 3D, 2D}
    constexpr int NBE = (4 * D + C::NT - 1) / C::NT;
    float bsum[NBE];
#pragma unroll
    for (int i = 0; i < NBE; ++i) bsum[i] = 0.f;
    const float* W = a.params;              // [W_z;W_r;W_n] (3D x DX)
    for (int idx = tid; idx < 3 * D * C::DXP; idx += C::NT) {
        const int r = idx / C::DXP, c = idx % C::DXP;
        wst[c * WT + r] = c < DX ? W[r * DX + c] : 0.f;
    }

    TileInfo tnext{};
    if ((int)blockIdx.x < a.ntiles) tnext = a.tiles[blockIdx.x];
    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
      const TileInfo ti = tnext;
      if (tile + (int)gridDim.x < a.ntiles) tnext = a.tiles[tile + gridDim.x];   // read ahead
      const int b = ti.b;
      const float* lam = a.lam;
      for (int sub = 0; sub < SUB; ++sub) {
        const int len = min(L, ti.len - sub * L);
        if (len <= 0) break;
        const int64_t row0 = ti.row0 + (int64_t)sub * L;
        const bool first = sub == 0 && (ti.flags & kTileTimeFirst) != 0;
        __syncthreads();
        // stage the delta rows [dz | dr | dq | dn] = (alpha, gamma, beta, eps) * lambda, the
        // h_{t-1} rows and the x rows; every load is issued before the LDS writes
        constexpr int Q = D / 4, QX = C::DXP / 4;
        constexpr int NS = (L * Q + C::NT - 1) / C::NT;
        constexpr int NX = (L * QX + C::NT - 1) / C::NT;
        float4 vl[NS], va[NS], vb[NS], vg[NS], ve[NS], vh[NS], vx[NX];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int idx = tid + i * C::NT;
            const int tl = idx / Q, c4 = idx % Q;
            const bool ok = idx < L * Q && tl < len;
            const size_t row = (size_t)(row0 + tl);
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            const float* gr = a.gates + row * 4 * D + 4 * c4;
            vl[i] = ok ? *(const float4*)(lam + row * D + 4 * c4) : z4;
            va[i] = ok ? *(const float4*)(gr + 0 * D) : z4;
            vb[i] = ok ? *(const float4*)(gr + 1 * D) : z4;
            vg[i] = ok ? *(const float4*)(gr + 2 * D) : z4;
            ve[i] = ok ? *(const float4*)(a.eps + row * D + 4 * c4) : z4;
            vh[i] = !ok ? z4
                        : (tl == 0 && first) ? *(const float4*)(a.s0 + (size_t)b * D + 4 * c4)
                                             : *(const float4*)(a.s + (row - 1) * D + 4 * c4);
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int idx = tid + i * C::NT;
            const int tl = idx / QX, c4 = idx % QX;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (idx < L * QX && tl < len) {
                const float* xr = a.x + (size_t)(row0 + tl) * DX;
                // DX is a multiple of 8; the padded columns past DX stay zero
                if (4 * c4 < DX) v = *(const float4*)(xr + 4 * c4);
            }
            vx[i] = v;
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const int idx = tid + i * C::NT;
            if (idx >= L * Q) continue;
            const int tl = idx / Q, c4 = idx % Q;
            const float4 lv = vl[i];
            float* dr_ = dl + tl * DS + 4 * c4;
            *(float4*)(dr_) = make_float4(va[i].x * lv.x, va[i].y * lv.y, va[i].z * lv.z,
                                          va[i].w * lv.w);                         // dz
            *(float4*)(dr_ + D) = make_float4(vg[i].x * lv.x, vg[i].y * lv.y, vg[i].z * lv.z,
                                              vg[i].w * lv.w);                     // dr
            *(float4*)(dr_ + 2 * D) = make_float4(vb[i].x * lv.x, vb[i].y * lv.y,
                                                  vb[i].z * lv.z, vb[i].w * lv.w);  // dq
            *(float4*)(dr_ + 3 * D) = make_float4(ve[i].x * lv.x, ve[i].y * lv.y,
                                                  ve[i].z * lv.z, ve[i].w * lv.w);  // dn
            *(float4*)(hsm + tl * C::HS + 4 * c4) = vh[i];
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            const int idx = tid + i * C::NT;
            if (idx < L * QX) *(float4*)(xsm + (idx / QX) * XSP + 4 * (idx % QX)) = vx[i];
        }
        __syncthreads();
        // bias partials (every thread, its NBE entries)
#pragma unroll
        for (int i = 0; i < NBE; ++i) {
            const int e = tid + i * C::NT;
            if (e < 4 * D) {
                const int k4 = e / D, bu = e % D;
                const int bcol = k4 == 0 ? 0 : (k4 == 1 ? D : (k4 == 2 ? 3 * D : 2 * D));
                float sacc = 0.f;
#pragma unroll 8
                for (int tl = 0; tl < L; ++tl) sacc += dl[tl * DS + bcol + bu];
                bsum[i] += sacc;
            }
        }
        // parameter GEMM of unit block w: K = steps, 4 per MFMA
        const float* dlw = dl + 16 * w + u;
#pragma unroll 2
        for (int kq = 0; kq < L / 4; ++kq) {
            const int tstep = 4 * kq + g;       // step of this lane's K slot
            const float* dr_ = dlw + tstep * DS;
            const float az = dr_[0], ar = dr_[D], aq = dr_[2 * D], an = dr_[3 * D];
            float bh[HB], bx[XB];
#pragma unroll
            for (int c = 0; c < HB; ++c) bh[c] = hsm[tstep * C::HS + 16 * c + u];
#pragma unroll
            for (int c = 0; c < XB; ++c) bx[c] = xsm[tstep * XSP + 16 * c + u];
#pragma unroll
            for (int c = 0; c < HB; ++c) {
                acc[0][c] = mfma16x4(az, bh[c], acc[0][c]);
                acc[1][c] = mfma16x4(ar, bh[c], acc[1][c]);
                acc[2][c] = mfma16x4(aq, bh[c], acc[2][c]);
            }
#pragma unroll
            for (int c = 0; c < XB; ++c) {
                acc[0][HB + c] = mfma16x4(az, bx[c], acc[0][HB + c]);
                acc[1][HB + c] = mfma16x4(ar, bx[c], acc[1][HB + c]);
                acc[2][HB + c] = mfma16x4(an, bx[c], acc[2][HB + c]);
            }
        }
        // dx rows: dx_t = W_z^T dz + W_r^T dr + W_n^T dn  (K = 3D, N = DX); one 16 x 16 output
        // tile (step block mb, column block nb) per wave.  Lane group g takes the K indices
        // g KQ .. g KQ + KQ - 1 of every gate, so that its A (delta row) and B (W^T row)
        // operands are contiguous float4 runs in LDS.
        if (a.gx) {
            constexpr int NBX = C::DXP / 16;
            constexpr int KQ = D / 4;
            for (int ot = w; ot < C::MB * NBX; ot += NW) {
                const int mb = ot / NBX, nb = ot % NBX;
                floatx4 o4 = {0.f, 0.f, 0.f, 0.f};
                const int n = 16 * nb + u;
                const float* arow = dl + (mb * 16 + u) * DS + g * KQ;
                const float* brow = wst + n * WT + g * KQ;
#pragma unroll
                for (int gate = 0; gate < 3; ++gate) {
                    const float* ag = arow + (gate == 0 ? 0 : (gate == 1 ? D : 3 * D));
                    const float* bg = brow + gate * D;
#pragma unroll
                    for (int k4 = 0; k4 < KQ; k4 += 4) {
                        const float4 av = *(const float4*)(ag + k4);
                        const float4 bv = *(const float4*)(bg + k4);
                        o4 = mfma16x4(av.x, bv.x, o4);
                        o4 = mfma16x4(av.y, bv.y, o4);
                        o4 = mfma16x4(av.z, bv.z, o4);
                        o4 = mfma16x4(av.w, bv.w, o4);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;
                    if (tl < len && n < DX) a.gx[(size_t)(row0 + tl) * DX + n] = o4[i];
                }
            }
        }
      }
    }
    // write this workgroup's partials in the packed gradient layout
    constexpr int P = 3 * D * DX + 3 * D * D + 4 * D;
    float* part = a.part + (size_t)blockIdx.x * P;
#pragma unroll
    for (int gate = 0; gate < 3; ++gate)
#pragma unroll
        for (int cb = 0; cb < HB + XB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * w + 4 * g + i;      // unit
                if (cb < HB) {
                    part[3 * D * DX + (gate * D + row) * D + 16 * cb + u] = acc[gate][cb][i];
                } else {
                    const int col = 16 * (cb - HB) + u;
                    if (col < DX) part[(gate * D + row) * DX + col] = acc[gate][cb][i];
                }
            }
    float* pb = part + 3 * D * DX + 3 * D * D;
#pragma unroll
    for (int i = 0; i < NBE; ++i) {
        const int e = tid + i * C::NT;
        if (e < 4 * D) pb[e] = bsum[i];
    }
}

// dL/ds_0 = A_1^T lambda_1 for every sequence (one workgroup per sequence).
template <int D, int DX>
__global__ void gru_adj_gs0_kernel(GruAdjArgs a) {
    const int b = blockIdx.x;
    const int j = threadIdx.x;
    if (j >= D) return;
    const int64_t r0 = a.offsets[b];
    if (a.offsets[b + 1] == r0) { a.gs0[(size_t)b * D + j] = 0.f; return; }
    const float* lam = a.lam + (size_t)r0 * D;
    const float* gr = a.gates + (size_t)r0 * 4 * D;
    const float* U = a.params + 3 * D * DX;
    float v = gr[3 * D + j] * lam[j];
    for (int i = 0; i < D; ++i) {
        const float li = lam[i];
        v += U[(0 * D + i) * D + j] * gr[i] * li          // U_z^T (alpha * lambda)
           + U[(2 * D + i) * D + j] * gr[D + i] * li      // U_n^T (beta * lambda)
           + U[(1 * D + i) * D + j] * gr[2 * D + i] * li; // U_r^T (gamma * lambda)
    }
    a.gs0[(size_t)b * D + j] = v;
}

// ---- sequential adjoint (baseline): lambda_t = g_t + A_{t+1}^T lambda_{t+1}, one step at a
// time per sequence, one wave per sequence.  Lane j owns unit j and holds the columns j of
// U_z, U_n and U_r in registers; per step it writes its three VJP operands alpha_j lambda_j,
// beta_j lambda_j, gamma_j lambda_j to LDS, reads all 3 D of them back (a single wave's LDS
// operations complete in order: no barrier) and forms
//   (A_t^T lambda_t)_j = z_j lambda_j + sum_i (U_z[i][j] alpha_i + U_n[i][j] beta_i
//                                               + U_r[i][j] gamma_i) lambda_i.
// The per-step operands (g, alpha, beta, gamma, z) of the next PF steps are prefetched.
template <int D>
__global__ void __launch_bounds__(64) gru_seq_adj_kernel(const float* __restrict__ gates,
                                                         const float* __restrict__ gs,
                                                         const float* __restrict__ U,
                                                         float* __restrict__ lam,
                                                         const int64_t* __restrict__ offsets) {
    static_assert(D % 4 == 0 && D <= 64, "one lane per unit");
    constexpr int PF = 4;
    __shared__ __attribute__((aligned(16))) float prod[2][3][D];
    const int b = blockIdx.x;
    const int j = threadIdx.x;
    const bool act = j < D;
    const int jj = act ? j : 0;
    const int64_t r0 = offsets[b], T = offsets[b + 1] - r0;
    if (T == 0) return;                      // nothing to walk (and no row to prefetch)
    float wz[D], wn[D], wr[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        wz[i] = U[(size_t)i * D + jj];               // U_z[i][j]
        wr[i] = U[(size_t)(D + i) * D + jj];         // U_r[i][j]
        wn[i] = U[(size_t)(2 * D + i) * D + jj];     // U_n[i][j]
    }
    struct Ops { float g, al, be, ga, z; };          // g, alpha, beta, gamma, z of one step
    auto fetch = [&](int64_t it) {
        const int64_t row = r0 + (T - 1 - it);
        const float* gr = gates + (size_t)row * 4 * D;
        return Ops{gs[(size_t)row * D + jj], gr[jj], gr[D + jj], gr[2 * D + jj], gr[3 * D + jj]};
    };
    float v = 0.f;                                   // A_{t+1}^T lambda_{t+1}
    // reverse step it (t = T - 1 - it): lambda_t = g_t + v, then v <- A_t^T lambda_t
    auto step = [&](int64_t it, const Ops& o) {
        const int64_t t = T - 1 - it;
        const float lt = o.g + v;
        float* pb = &prod[it & 1][0][0];
        if (act) {
            lam[(size_t)(r0 + t) * D + j] = lt;
            pb[j] = o.al * lt;
            pb[D + j] = o.be * lt;
            pb[2 * D + j] = o.ga * lt;
        }
        __builtin_amdgcn_wave_barrier();
        float a0 = o.z * lt, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int k = 0; k < D; k += 4) {
            const float4 pz4 = *(const float4*)(pb + k);
            const float4 pn4 = *(const float4*)(pb + D + k);
            const float4 pr4 = *(const float4*)(pb + 2 * D + k);
            a0 = fmaf(wz[k], pz4.x, a0);
            a1 = fmaf(wn[k], pn4.x, a1);
            a2 = fmaf(wr[k], pr4.x, a2);
            a0 = fmaf(wz[k + 1], pz4.y, a0);
            a1 = fmaf(wn[k + 1], pn4.y, a1);
            a2 = fmaf(wr[k + 1], pr4.y, a2);
            a0 = fmaf(wz[k + 2], pz4.z, a0);
            a1 = fmaf(wn[k + 2], pn4.z, a1);
            a2 = fmaf(wr[k + 2], pr4.z, a2);
            a0 = fmaf(wz[k + 3], pz4.w, a0);
            a1 = fmaf(wn[k + 3], pn4.w, a1);
            a2 = fmaf(wr[k + 3], pr4.w, a2);
        }
        v = a0 + a1 + a2;
        __builtin_amdgcn_wave_barrier();
    };
    const int64_t Tm = T - T % PF;
    Ops ring[PF];
#pragma unroll
    for (int i = 0; i < PF; ++i) ring[i] = fetch(i < Tm ? i : 0);
    for (int64_t it0 = 0; it0 < Tm; it0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const Ops o = ring[i];
            const int64_t itn = it0 + i + PF < Tm ? it0 + i + PF : it0 + i;
            ring[i] = fetch(itn);
            step(it0 + i, o);
        }
    }
    for (int64_t it = Tm; it < T; ++it) step(it, fetch(it));
}

// ---- host driver ------------------------------------------------------------------------------

struct GruALayout {
    IterState st;
    float *gates, *eps, *lam, *mu[2], *gprod, *gmax, *part, *gcarry;
    uint32_t *cmax, *grmax;
    float2* gagg;
    void* dense;             // the dense scan's maps and carries (PN_JAC_DENSE only)
    size_t bytes;
};

constexpr int kAdjL = 32;
constexpr int kGradL = 32;

static int grad_grid() { return 2 * cu_count(); }
// The prep pass takes tiles in a grid-stride loop; a grid of several times the resident
// workgroups lets the hardware refill a CU as soon as one finishes (measured: 8 per CU at three
// waves per SIMD 2.50 ms against 2.85 ms for 2 per CU on the ragged D = 48 batch).
static int prep_grid() { return 8 * cu_count(); }

static GruALayout gruA_layout(void* ws, int D, int Dx, const HostBatch& hb, int ntiles,
                              int ngroups, bool freeze = false, bool dense = false) {
    Carver c(ws);
    GruALayout lay{};
    carve_iter_state(c, lay.st, hb.B, ntiles, ngroups);
    lay.gates = c.take<float>((size_t)hb.N * 4 * D);
    lay.eps = c.take<float>((size_t)hb.N * D);
    lay.lam = c.take<float>((size_t)hb.N * D);
    if (dense) {
        lay.dense = c.take<char>(gru_adj_dense_bytes(D, ngroups, hb.B));
    } else {
        for (int p = 0; p < 2; ++p) lay.mu[p] = c.take<float>((size_t)hb.N * D);
        lay.gagg = c.take<float2>((size_t)std::max(ngroups, 1) * D);
        lay.gcarry = c.take<float>((size_t)std::max(ngroups, 1) * D);
        lay.gprod = c.take<float>((size_t)std::max(ngroups, 1) * D);
    }
    lay.gmax = c.take<float>(hb.B);
    lay.cmax = c.take<uint32_t>((size_t)std::max(ntiles, 1) * (D / 16));
    const size_t P = 3 * (size_t)D * Dx + 3 * (size_t)D * D + 4 * (size_t)D;
    lay.part = c.take<float>((size_t)grad_grid() * P);
    lay.grmax = freeze ? c.take<uint32_t>((size_t)std::max(ngroups, 1) * (D / 16)) : nullptr;
    lay.bytes = c.bytes();
    return lay;
}

struct GruAKernels {
    void (*prep)(GruAdjArgs);
    void (*iter)(GruAdjArgs);
    void (*grad)(GruAdjArgs);
    void (*gs0)(GruAdjArgs);
    void (*gmax)(GruAdjArgs);
    int nt;
};

template <int D, int DX>
static GruAKernels gruA_get() {
    GruAKernels k;
    k.prep = gru_adj_prep_kernel<D, DX, kAdjL>;
    k.iter = gru_adj_local_kernel<D, DX, kAdjL>;
    k.grad = gru_adj_grad_kernel<D, DX, kGradL, kAdjL / kGradL>;
    k.gs0 = gru_adj_gs0_kernel<D, DX>;
    k.gmax = gru_adj_gmax_kernel<D / 16>;
    k.nt = 64 * (D / 16);
    return k;
}

static bool gruA_lookup(int D, int Dx, GruAKernels* k) {
#define PN_GA(d, dx) if (D == d && Dx == dx) { *k = gruA_get<d, dx>(); return true; }
    PN_GA(64, 32) PN_GA(48, 24) PN_GA(32, 16) PN_GA(16, 8) PN_GA(16, 16) PN_GA(64, 64)
    PN_GA(32, 32) PN_GA(48, 48) PN_GA(64, 16) PN_GA(32, 8)
#undef PN_GA
    return false;
}

// Tile groups of the adjoint iteration for this batch.
//
// The dense scan's default group length balances its two sequential parts (measured on the
// device): the chain pass walks 16 groups per wave and streams at a flat rate while every
// SIMD holds as many of its waves as fit (two at D <= 48, one at D = 64: 32 K or 16 K
// groups), slowing about as the square root of the shortfall below; the carry walk takes
// about 0.5 us per group of the longest sequence.
static int dense_group_tiles(const std::vector<int32_t>& ts, int B, int D, int64_t N) {
    int tmax = 0;
    for (int b = 0; b < B; ++b) tmax = std::max(tmax, ts[b + 1] - ts[b]);
    const double chain_ms = (double)N * 24.0 * D / 3.8e9;       // bytes / (3.8 TB/s), in ms
    const double full = D <= 48 ? 32768.0 : 16384.0;
    int best = 1;
    double best_ms = 1e30;
    for (int gt = 1; gt <= 64; gt *= 2) {
        const int ng = count_groups(ts, B, gt);
        const double ms = chain_ms * std::sqrt(std::max(1.0, full / std::max(ng, 1))) +
                          0.5e-3 * ((tmax + gt - 1) / gt);
        if (ms < best_ms) best_ms = ms, best = gt;
    }
    return best;
}

static int gruA_groups(const GruAKernels& kk, const std::vector<int32_t>& ts, int B, int group,
                       int* gt, int* resident, bool dense = false, int64_t N = 0, int D = 0) {
    *resident = gru_resident((const void*)kk.iter, kk.nt);
    if (group > 0)
        *gt = group;
    else if (dense)
        *gt = dense_group_tiles(ts, B, D, N);
    else
        *gt = gru_group_tiles(ts[B], *resident);
    return count_groups(ts, B, *gt);
}

size_t gru_adjoint_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    GruAKernels kk;
    if (!gruA_lookup(D, Dx, &kk)) return 0;
    const bool dense = o.jac == PN_JAC_DENSE;
    const std::vector<int32_t> ts = tile_starts(hb, kAdjL);
    int gt, resident;
    const int ngroups = gruA_groups(kk, ts, hb.B, o.group, &gt, &resident, dense, hb.N, D);
    return gruA_layout(nullptr, D, Dx, hb, ts[hb.B], ngroups, o.freeze_prefix != 0, dense).bytes;
}

static pn_status gru_adj_gradients(const GruAKernels& kk, const GruAdjArgs& args,
                                   const HostBatch& hb, int D, int Dx, const GruALayout& lay,
                                   hipStream_t stream, pn_seq_info* info, bool* all_conv,
                                   float* gs0);

pn_status gru_adjoint(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                      const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                      float* gparams, const pn_opts& o, void* ws, hipStream_t stream,
                      pn_seq_info* info, bool* all_conv) {
    const int D = cd.D, Dx = cd.Dx;
    GruAKernels kk;
    if (!gruA_lookup(D, Dx, &kk)) {
        set_error("GRU adjoint not built for D=%d Dx=%d", D, Dx);
        return PN_ERR_UNSUPPORTED;
    }
    const bool dense = o.jac == PN_JAC_DENSE;
    if (dense && (o.freeze_prefix || o.damping != PN_DAMP_NONE)) {
        set_error("the dense GRU adjoint takes no damping and no converged-prefix skipping");
        return PN_ERR_UNSUPPORTED;
    }
    const std::vector<int32_t> ts = tile_starts(hb, kAdjL);
    const int ntiles = ts[hb.B];
    int gt, resident;
    const int ngroups = gruA_groups(kk, ts, hb.B, o.group, &gt, &resident, dense, hb.N, D);
    GruALayout lay = gruA_layout(ws, D, Dx, hb, ntiles, ngroups, o.freeze_prefix != 0, dense);
    const int max_iters = o.max_iters > 0 ? o.max_iters
                                          : (dense ? 8 : (int)std::max<int64_t>(1, hb.Tmax));
    PN_TRY(init_iter_state(lay.st, hb, ts, kAdjL, true, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream, gt));

    GruAdjArgs args;
    args.x = x;
    args.s0 = s0;
    args.s = s;
    args.gs = gs;
    args.params = (const float*)cd.params;
    args.gates = lay.gates;
    args.eps = lay.eps;
    args.lam = lay.lam;
    for (int p = 0; p < 2; ++p) args.mu[p] = lay.mu[p];
    args.gprod = lay.gprod;
    args.gagg = lay.gagg;
    args.gcarry = lay.gcarry;
    args.gmax = lay.gmax;
    args.cmax = lay.cmax;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.offsets = lay.st.offsets;
    args.tile_start = lay.st.tile_start;
    args.tiles = lay.st.tiles;
    args.groups = lay.st.groups;
    args.ngroups = ngroups;
    args.grmax = lay.grmax;
    args.freeze = o.freeze_prefix ? 1 : 0;
    args.dscale = o.damping == PN_DAMP_SCALE ? 1.f - o.damp_k : 1.f;
    args.clip = o.damping == PN_DAMP_CLIP ? 1 : 0;
    args.clo = o.clip_lo;
    args.chi = o.clip_hi;
    args.B = hb.B;
    args.ntiles = ntiles;
    args.part = lay.part;
    args.gx = gx;
    args.gs0 = gs0;
    args.gparams = gparams;

    if (ntiles > 0) {
        prof_launch("gru_adj_prep", stream, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kk.prep, dim3(std::max(1, std::min(ntiles, prep_grid()))),
                               dim3(kk.nt), 0, s2, args);
        });
        PN_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(kk.gmax, dim3(hb.B), dim3(256), 0, stream, args);
    PN_HIP(hipGetLastError());
    if (dense) {
        PN_TRY(gru_adj_dense_solve(D, lay.gates, gs, (const float*)cd.params + 3 * D * Dx,
                                   lay.lam, lay.st, ngroups, hb.B, lay.gmax, (float)o.tol,
                                   o.compose == PN_COMPOSE_BF16, max_iters, lay.dense, stream));
        return gru_adj_gradients(kk, args, hb, D, Dx, lay, stream, info, all_conv, gs0);
    }
    const int grid = std::max(1, std::min(ngroups, resident));
    // iteration k (k from the control block) forms lambda^(k) from mu[k & 1] and the carries
    // of iteration k - 1, writes lambda^(k) and mu[(k + 1) & 1], then the carries
    auto one_iter = [&](hipStream_t st) {
        prof_launch("gru_adj_local", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kk.iter, dim3(grid), dim3(kk.nt), 0, s2, args);
        });
        prof_launch("carry_scan", st, [&](hipStream_t s2) {
            launch_carry_scan(lay.gagg, lay.gcarry, lay.st, hb.B, D, s2, lay.grmax, D / 16);
        });
        launch_decide(lay.st, hb.B, st, true);
    };
    std::vector<uintptr_t> key = {0x4145u, (uintptr_t)args.freeze, (uintptr_t)hb.N, lay.bytes, (uintptr_t)kk.iter, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)gs,
                                  (uintptr_t)cd.params, (uintptr_t)ws, (uintptr_t)hb.B,
                                  (uintptr_t)ntiles, (uintptr_t)ngroups,
                                  (uintptr_t)o.damping, float_bits(args.dscale),
                                  float_bits(args.clo), float_bits(args.chi)};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    return gru_adj_gradients(kk, args, hb, D, Dx, lay, stream, info, all_conv, gs0);
}

// Per-sequence results, then the gradients from the final adjoint iterate (the same tile
// table, two passes per tile).
static pn_status gru_adj_gradients(const GruAKernels& kk, const GruAdjArgs& args,
                                   const HostBatch& hb, int D, int Dx, const GruALayout& lay,
                                   hipStream_t stream, pn_seq_info* info, bool* all_conv,
                                   float* gs0) {
    PN_TRY(finish_iterations(lay.st, hb, D, sizeof(float), nullptr, nullptr, stream, info,
                             all_conv));
    const int gg = grad_grid();
    prof_launch("gru_adj_grad", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(kk.grad, dim3(gg), dim3(kk.nt), 0, s2, args);
    });
    PN_HIP(hipGetLastError());
    const int P = 3 * D * Dx + 3 * D * D + 4 * D;
    launch_partial_sum(lay.part, gg, P, args.gparams, stream);
    PN_HIP(hipGetLastError());
    if (gs0) {
        hipLaunchKernelGGL(kk.gs0, dim3(hb.B), dim3(std::max(64, D)), 0, stream, args);
        PN_HIP(hipGetLastError());
    }
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    return PN_OK;
}

// Sequential baseline of deer_adjoint: the same outputs, the reverse recurrence walked step by
// step (the gate values and the gradient reductions are parallel kernels).
pn_status seq_bptt_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                       const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                       float* gparams, void* ws, hipStream_t stream) {
    const int D = cd.D, Dx = cd.Dx;
    GruAKernels kk;
    if (!gruA_lookup(D, Dx, &kk)) return PN_ERR_UNSUPPORTED;
    void (*seqk)(const float*, const float*, const float*, float*, const int64_t*) = nullptr;
    switch (D) {
        case 16: seqk = gru_seq_adj_kernel<16>; break;
        case 32: seqk = gru_seq_adj_kernel<32>; break;
        case 48: seqk = gru_seq_adj_kernel<48>; break;
        case 64: seqk = gru_seq_adj_kernel<64>; break;
        default: return PN_ERR_UNSUPPORTED;
    }
    const std::vector<int32_t> ts = tile_starts(hb, kAdjL);
    const int ntiles = ts[hb.B];
    GruALayout lay = gruA_layout(ws, D, Dx, hb, ntiles, 0);
    PN_TRY(init_iter_state(lay.st, hb, ts, kAdjL, true, 1, 1.f, 1e4f, stream));
    GruAdjArgs args{};
    args.x = x;
    args.s0 = s0;
    args.s = s;
    args.gs = gs;
    args.params = (const float*)cd.params;
    args.gates = lay.gates;
    args.eps = lay.eps;
    args.lam = lay.lam;
    args.gmax = lay.gmax;
    args.cmax = lay.cmax;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.offsets = lay.st.offsets;
    args.tile_start = lay.st.tile_start;
    args.tiles = lay.st.tiles;
    args.B = hb.B;
    args.ntiles = ntiles;
    args.part = lay.part;
    args.gx = gx;
    args.gs0 = gs0;
    args.gparams = gparams;
    if (ntiles > 0)
        hipLaunchKernelGGL(kk.prep, dim3(std::max(1, std::min(ntiles, prep_grid()))),
                           dim3(kk.nt), 0, stream, args);
    const float* U = (const float*)cd.params + 3 * D * Dx;
    prof_launch("seq_adj", stream, [&](hipStream_t s2) {
        hipLaunchKernelGGL(seqk, dim3(hb.B), dim3(64), 0, s2, (const float*)lay.gates, gs, U,
                           lay.lam, (const int64_t*)lay.st.offsets);
    });
    PN_HIP(hipGetLastError());
    const int gg = grad_grid();
    hipLaunchKernelGGL(kk.grad, dim3(gg), dim3(kk.nt), 0, stream, args);
    const int P = 3 * D * Dx + 3 * D * D + 4 * D;
    launch_partial_sum(lay.part, gg, P, gparams, stream);
    if (gs0) hipLaunchKernelGGL(kk.gs0, dim3(hb.B), dim3(std::max(64, D)), 0, stream, args);
    PN_HIP(hipGetLastError());
    PN_HIP(hipStreamSynchronize(stream));
    prof_collect();
    return PN_OK;
}

}  // namespace pn
