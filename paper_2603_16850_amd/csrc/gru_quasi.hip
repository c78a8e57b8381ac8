// quasi-DEER for the GRU cell: one Newton iteration as two passes over HBM.
//
// Tiles are L consecutive steps; groups are runs of consecutive tiles of one sequence (see
// IterState).  Iteration k:
//   local pass (gru_quasi_local_kernel), one workgroup per group of tiles, tile by tile:
//     1. stages s_{t-1}, s_t (L+1 rows) and x_t (L rows) in LDS (the tile's rows of s, of
//        the previous maps and of x are contiguous blocks, copied straight from HBM into
//        LDS).  For k >= 1 the rows of s^(k) are formed from s^(k-1) and the previous
//        iteration's maps, s^(k)_t = s^(k-1)_t + la_t carry + lc_t, the reset guard applied (a
//        row with a non-finite entry or one above reset_abs becomes 0), and written back;
//     2. evaluates the gate pre-activations of f(s_{t-1}, x_t) for the L steps as a small
//        GEMM [L x (D+Dx)] x [(D+Dx) x 4 gate blocks] on FP32 MFMA (16x16x4), the weights
//        held in registers for the whole kernel;
//     3. forms the residual r_t = s_t - f_t(s_{t-1}) (Ch. 2, eq. r_def), the scan leaf
//        (a_t, c_t) = (diag A_t, -r_t) with the closed-form GRU diagonal (quasi-DEER,
//        eq. quasi_lds), and the per-sequence max |r| that the stopping test reads;
//     4. scans Delta_t = a_t Delta_{t-1} + c_t (eq. lin_rr with a diagonal transition) over
//        the tile (in registers, across lane groups by shuffles, across 16-step blocks
//        serially) and composes the result with the map of the group's earlier tiles, so
//        that (la_t, lc_t) gives Delta_t = la_t Delta_in(group) + lc_t;
//     5. writes (la, lc) for the tile's steps and, after the last tile, the group's map;
//   carry pass (carry_scan.hip): the carry Delta_in of every group from the group maps.
// The update s^(k+1) = s^(k) + Delta is thus applied by the next iteration's local pass,
// which is also where its residual is tested.  At a sequence head a_t = 0, so the carry into
// a sequence is Delta_0 = 0 (s_0 is fixed).  No workgroup waits for another: the passes are
// ordered by the stream.
#include <algorithm>

#include "carry.hpp"
#include "gru_common.hpp"
#include "pn_host.hpp"
#include "pn_solvers.hpp"

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

// The transition matrix A~_t of the linear recurrence solved each iteration (the fixed-point
// methods of Ch. "Convergence Rates of quasi-Newton methods", Table fxd_pt_sum):
//   kTransDiag      diag(df/ds) in closed form: quasi-DEER (eq. quasi_lds)
//   kTransIdentity  I: Picard iteration (Prop. picard); the scan is a prefix sum of -r
//   kTransZero      0: Jacobi iteration; s_t <- f(s_{t-1}) for every t at once, no scan
enum GruTrans : int { kTransDiag = 0, kTransIdentity = 1, kTransZero = 2 };

struct GruQArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];          // ping-pong iterates: s^(k) lives in sbuf[k & 1]
    const float* params;
    float2* lac[2];          // [N][D] (la, lc) of every step relative to its group's start,
                             // iteration k writes lac[k & 1]
    float2* gagg;            // [ngroups][D] map of every group
    const float* gcarry;     // [ngroups][D] carry into every group (previous iteration)
    Ctrl* ctrl;
    SeqState* seq;
    const TileInfo* tiles;   // by slot
    const GroupInfo* groups; // by group slot
    int ngroups;
    uint32_t* grmax;         // [ngroups][D / 16] residual max of each group's waves (bits),
                             // written with converged-prefix skipping
    int freeze;              // converged-prefix skipping on
    int mode;                // transition matrix: kTransDiag, kTransIdentity or kTransZero
    float dscale;            // scale damping: A~ <- dscale A~ (1 - k; 1 without damping)
    int clip;                // clip damping on: A~ <- min(max(A~, clo), chi)
    float clo, chi;
};

template <int D, int DX, int L>
__global__ void __launch_bounds__(64 * (D / 16))
__attribute__((amdgpu_waves_per_eu(L <= 32 ? 3 : 2, L <= 32 ? 3 : 2)))
gru_quasi_local_kernel(GruQArgs a) {
    using C = GruQ<D, DX, L>;
    __shared__ __attribute__((aligned(16))) float hs[(L + 1) * C::HS];
    __shared__ __attribute__((aligned(16))) float xs[L * DX];           // x rows, unpadded
    __shared__ __attribute__((aligned(16))) float sraw[(L + 1) * D];    // s rows as copied
    __shared__ __attribute__((aligned(16))) float lraw[(L + 1) * 2 * D];// (la, lc) rows as copied

    __shared__ int rowbad[L + 1];
    __shared__ int anybad[2];      // some row of the tile was reset (by tile parity)
    // With 32-step tiles the next tile's rows are copied while the current one is computed
    // (PF): the staging buffers above then take the next tile's copies as soon as the update
    // has read them, and the GEMM reads the tile's x rows from a copy of their own.
    constexpr bool PF = L == 32;
    __shared__ __attribute__((aligned(16))) float xcur[PF ? L * DX : 4];
    __shared__ __attribute__((aligned(16))) float cgs[2 * D];          // carries: own, halo

    if (ld_i32(&a.ctrl->all_done)) return;
    // Iteration k first forms s^(k) = s^(k-1) + la carry + lc from the previous iteration's
    // maps (k >= 1; s^(0) is the caller's guess) with the reset guard, then linearises there.
    const int k = a.ctrl->iter;
    const bool fuse = k > 0;
    const float reset_abs = a.ctrl->reset_abs;
    const bool bydelta = a.ctrl->stop_delta != 0;
    const float* __restrict__ sprev = a.sbuf[(k + 1) & 1];   // s^(k-1)
    float* __restrict__ scur = a.sbuf[k & 1];                 // s^(k)
    const float2* __restrict__ lacp = a.lac[(k + 1) & 1];
    float2* __restrict__ lacn = a.lac[k & 1];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int g = l >> 4;          // lane group (k-slot of A/B, row quad of D)
    const int u = l & 15;          // unit within the wave / row of A
    const int j = 16 * w + u;      // state unit this lane owns in the outputs

    GruGates<D, DX> wg;   // this wave's weights (units j) as MFMA B operands
    wg.load(a.params, j, g);
    for (int r = tid; r <= L; r += C::NT) rowbad[r] = 0;
    if (tid < 2) anybad[tid] = 0;
    int tcount = 0;                // tiles done by this workgroup (parity of anybad)

    // The group and tile tables and the sequences' status are not written while the kernel
    // runs: they are read through the scalar cache (s_load), whose short round trip is not
    // added to every tile and whose counter is not the one the copies into LDS advance.
    using CGroup = const __attribute__((address_space(4))) GroupInfo;
    using CTile = const __attribute__((address_space(4))) TileInfo;
    using CSeq = const __attribute__((address_space(4))) SeqState;
    auto tile_at = [&](int i) {
        CTile* ct = (CTile*)a.tiles + i;
        TileInfo t;
        t.slot = ct->slot;
        t.b = ct->b;
        t.len = ct->len;
        t.flags = ct->flags;
        t.row0 = ct->row0;
        t.gslot = ct->gslot;
        t.hgslot = ct->hgslot;
        return t;
    };

    for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
        GroupInfo gr;
        {
            CGroup* cg = (CGroup*)a.groups + gi;
            gr.b = cg->b;
            gr.tile0 = cg->tile0;
            gr.ntl = cg->ntl;
            gr.gfirst = cg->gfirst;
        }
        if (((CSeq*)a.seq)[gr.b].status != kActive) continue;     // same on every thread
        const int b = gr.b;
        // converged-prefix skipping: the sequence's leading groups [0, frozen) take no more
        // updates; one frozen by the last carry pass gets s^(k) = s^(k-1) on its rows once
        // (both iterate buffers then hold them) and is skipped from then on
        bool halo_frozen = false;
        if (a.freeze) {
            const int li = gi - gr.gfirst, nf = a.seq[b].frozen;
            if (li < nf) {
                if (li >= a.seq[b].frozen_prev) {
                    const TileInfo t0 = a.tiles[gr.tile0], t1 = a.tiles[gr.tile0 + gr.ntl - 1];
                    const int64_t e0 = t0.row0 * (D / 4), e1 = (t1.row0 + t1.len) * (D / 4);
                    for (int64_t e = e0 + tid; e < e1; e += C::NT)
                        ((float4*)scur)[e] = ((const float4*)sprev)[e];
                }
                continue;
            }
            halo_frozen = li == nf && nf > 0;    // the row before the group does not move
        }
        float Pa = 1.f, Pc = 0.f;        // map of the group's tiles before the current one
        uint32_t rmax = 0;
        // nbytes (a multiple of 16) from src to LDS dst, 1 KB per wave instruction (lane i's
        // 16 B to byte 16 i of the slice)
        auto bulk = [&](float* dst, const float* src, int nbytes) {
            for (int c = w; c * 1024 < nbytes; c += C::NW) {
                const int off = c * 1024 + 16 * l;
                if (off < nbytes)
                    __builtin_amdgcn_global_load_lds(
                        (const void*)((const char*)src + off),
                        (__attribute__((address_space(3))) void*)((char*)dst + c * 1024), 16, 0, 0);
            }
        };
        // a tile's s rows row0-1 .. row0+len-1 (staged row 0 is the halo s_{t0-1}: s0 at a
        // sequence's first tile), its (la, lc) rows and x rows, and the carries into its group
        // and into the one before
        auto issue = [&](const TileInfo& t) {
            const bool tf = (t.flags & kTileTimeFirst) != 0;
            const int hr = tf ? 1 : 0;
            const int64_t srow = t.row0 - 1 + hr;
            const int nrow = t.len + 1 - hr;
            if (tf) bulk(sraw, a.s0 + (size_t)b * D, D * 4);
            bulk(sraw + hr * D, (fuse ? sprev : scur) + (size_t)srow * D, nrow * D * 4);
            if (fuse) {
                bulk(lraw + hr * 2 * D, (const float*)(lacp + (size_t)srow * D), nrow * 2 * D * 4);
                bulk(cgs, a.gcarry + (size_t)t.gslot * D, D * 4);
                if (!tf) bulk(cgs + D, a.gcarry + (size_t)t.hgslot * D, D * 4);
            }
            bulk(xs, a.x + (size_t)t.row0 * DX, t.len * DX * 4);
        };
        TileInfo tnext = tile_at(gr.tile0);
        for (int kt = 0; kt < gr.ntl; ++kt) {
            const TileInfo ti = tnext;
            if (kt + 1 < gr.ntl) tnext = tile_at(gr.tile0 + kt + 1);   // read ahead
            const int len = ti.len;
            const int64_t row0 = ti.row0;
            const bool first = (ti.flags & kTileTimeFirst) != 0;

            // ---- stage s rows row0-1 .. row0+L-1 (stage row r <-> s_{t0-1+r}) and x rows.
            // The tile's rows of s, of the previous maps (la, lc) and of x are contiguous in
            // HBM and go straight into LDS as whole blocks (global_load_lds), all in flight
            // together; the update to s^(k) then runs LDS to LDS.  A thread's float4 column c4
            // is the same for all its s items (NT is a multiple of D / 4).
            constexpr int Q = D / 4;
            static_assert(C::NT % Q == 0, "column per thread");
            constexpr int NSV = ((L + 1) * Q + C::NT - 1) / C::NT;
            const int c4 = tid % Q;
            // Lane offsets into the LDS tiles and the [N][D] rows, formed anew for every tile
            // (hidden from the optimiser): hoisted out of the loops, one precomputed address
            // per (row, operand) would stay live across the whole group loop.
            int o_arow = u * C::HS;                  // hs / xs: GEMM operand row u (x: o_xrow)
            int o_xrow = u * DX;
            int o_own = 4 * g * C::HS + j;           // hs: row 4 g, column j
            int o_row = 4 * g * D + j;               // [N][D] arrays: own row 4 g, column j
            int o_st = (tid / Q) * C::HS + 4 * c4;   // staging: s item 0 in hs
            asm volatile("" : "+v"(o_arow), "+v"(o_xrow), "+v"(o_own), "+v"(o_row), "+v"(o_st));
            constexpr int RQ = C::NT / Q;            // s item i of a thread is row tid / Q + i RQ
            // with PF only a group's first tile is copied here, every later one while the
            // previous tile was computed; without, every tile once the previous one is done
            if (!PF) __syncthreads();
            if (!PF || kt == 0) issue(ti);
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies have landed
            __syncthreads();                      // every wave's; the previous tile is done
            const int par = tcount++ & 1;
            if (tid == 0) anybad[par ^ 1] = 0;    // the previous tile's flag, read by all
#pragma unroll
            for (int i = 0; i < NSV; ++i) {
                const int idx = tid + i * C::NT;
                if (idx >= (L + 1) * Q) continue;
                const int r = idx / Q;
                float4 w4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r == 0 || r - 1 < len) {
                    w4 = *(const float4*)(sraw + r * D + 4 * c4);
                    if (fuse && !(r == 0 && (first || (kt == 0 && halo_frozen)))) {
                        const float4 cv = *(const float4*)(cgs + (r == 0 ? D : 0) + 4 * c4);
                        const float4 p0 = *(const float4*)(lraw + r * 2 * D + 8 * c4);
                        const float4 p1 = *(const float4*)(lraw + r * 2 * D + 8 * c4 + 4);
                        const float d0 = p0.x * cv.x + p0.y;
                        const float d1 = p0.z * cv.y + p0.w;
                        const float d2 = p1.x * cv.z + p1.y;
                        const float d3 = p1.z * cv.w + p1.w;
                        w4.x += d0;
                        w4.y += d1;
                        w4.z += d2;
                        w4.w += d3;
                        // update norm of the group's own rows (row 0 is the halo)
                        if (bydelta && r > 0)
                            rmax = max(rmax, max(max(absbits(d0), absbits(d1)),
                                                 max(absbits(d2), absbits(d3))));
                        // s^(k) of the tile's own rows to HBM; a row the reset guard
                        // takes back is written again below
                        if (r >= 1) *(float4*)(scur + (size_t)(row0 + r - 1) * D + 4 * c4) = w4;
                        if (!(fabsf(w4.x) <= reset_abs) || !(fabsf(w4.y) <= reset_abs) ||
                            !(fabsf(w4.z) <= reset_abs) || !(fabsf(w4.w) <= reset_abs)) {
                            rowbad[r] = 1;
                            anybad[par] = 1;
                        }
                    }
                }
                *(float4*)(hs + o_st + i * RQ * C::HS) = w4;
            }
            if (PF)
                for (int e = tid; e < L * DX / 4; e += C::NT)
                    ((float4*)xcur)[e] = ((const float4*)xs)[e];
            __syncthreads();
            if (fuse && anybad[par]) {
                // reset guard: the rows with a non-finite or too large entry restart from 0
#pragma unroll
                for (int i = 0; i < NSV; ++i) {
                    const int idx = tid + i * C::NT;
                    const int r = idx / Q;
                    if (idx < (L + 1) * Q && (r == 0 || r - 1 < len) && rowbad[r]) {
                        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
                        *(float4*)(hs + r * C::HS + 4 * c4) = z4;
                        if (r >= 1) *(float4*)(scur + (size_t)(row0 + r - 1) * D + 4 * c4) = z4;
                    }
                }
                if (tid < 64) {
                    int nb = 0;
                    for (int base = 1; base <= L; base += 64) {
                        const int r = base + tid;
                        nb += __popcll(__ballot(r <= len && rowbad[r]));
                    }
                    if (tid == 0 && nb) atomicAdd(&a.seq[b].resets_pending, nb);
                }
                __syncthreads();
                for (int r = tid; r <= L; r += C::NT) rowbad[r] = 0;
            }

            // every wave is past its last read of the staging buffers: with PF the next tile's
            // copies go in now and overlap the rest of this one (no fenced barrier follows
            // before the next tile, which would wait for them)
            if (PF && kt + 1 < gr.ntl) issue(tnext);

            // ---- gates by MFMA, then residual and leaves, per 16-step block ----
            float la[C::MB][4], lc[C::MB][4];
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb) {
                floatx4 az, ar, aq, an;
                wg.gemm(hs + o_arow + mb * 16 * C::HS, (PF ? xcur : xs) + o_xrow + mb * 16 * DX, g,
                        az, ar, aq, an);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;      // step index within the tile
                    const float* hp = hs + o_own + (mb * 16 + i) * C::HS;
                    const float h = hp[0];                   // s_{t-1}
                    const float sc = hp[C::HS];              // s_t (current iterate)
                    const GruPoint p = gru_point(az[i], ar[i], aq[i], an[i], wg.b_z, wg.b_r,
                                                 wg.b_n, wg.b_hn);
                    const float f = (1.f - p.z) * p.n + p.z * h;
                    const float res = sc - f;
                    const float e = (1.f - p.z) * (1.f - p.n * p.n);
                    float dg = p.z + (h - p.n) * p.z * (1.f - p.z) * wg.dUz + e * p.r * wg.dUn
                             + e * p.q * p.r * (1.f - p.r) * wg.dUr;
                    const bool valid = tl < len;
                    if (a.mode != kTransDiag) dg = (a.mode == kTransIdentity) ? 1.f : 0.f;
                    dg *= a.dscale;                              // scale-ELK
                    if (a.clip) dg = fminf(fmaxf(dg, a.clo), a.chi);   // clip-ELK
                    if (first && tl == 0) dg = 0.f;
                    la[mb][i] = valid ? dg : 1.f;
                    lc[mb][i] = valid ? -res : 0.f;
                    if (valid && !bydelta) rmax = max(rmax, absbits(res));
                }
            }

            // ---- scan inside the tile ----
            // lane-local over the 4 steps of each block
            float Ra = Pa, Rc = Pc;    // map from the group start to the current block's start
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
            Pa = Ra;
            Pc = Rc;

            // ---- (la, lc) of every step of the tile ----
#pragma unroll
            for (int mb = 0; mb < C::MB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int tl = mb * 16 + 4 * g + i;
                    if (tl < len)
                        lacn[(size_t)row0 * D + o_row + (mb * 16 + i) * D] =
                            make_float2(la[mb][i], lc[mb][i]);
                }
        }
        if (g == 0) a.gagg[(size_t)gi * D + j] = make_float2(Pa, Pc);
        // residual max of the current iterate over the group (with the update-norm rule the
        // max of the update that formed it), one atomic per wave
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rmax = max(rmax, (uint32_t)__shfl_xor((int)rmax, off));
        if (l == 0) {
            atomicMax(bydelta ? &a.seq[b].maxd : &a.seq[b].maxr, rmax);
            if (a.freeze) a.grmax[(size_t)gi * C::NW + w] = rmax;
        }
    }
}

// ---- host driver ------------------------------------------------------------------------

struct GruQLayout {
    IterState st;
    float* salt;
    float2* lac[2];
    float2* gagg;
    float* gcarry;
    uint32_t* grmax;    // converged-prefix skipping: [ngroups][D / 16]
    void* r64;          // update-norm rule: the FP64 residual of the result
    size_t bytes;
};

static GruQLayout gruq_layout(void* ws, int D, int Dx, const HostBatch& hb, int ntiles,
                              int ngroups, const pn_opts& o) {
    Carver c(ws);
    GruQLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles, ngroups);
    lay.salt = c.take<float>((size_t)hb.N * D);
    for (int p = 0; p < 2; ++p) lay.lac[p] = c.take<float2>((size_t)hb.N * D);
    lay.gagg = c.take<float2>((size_t)std::max(ngroups, 1) * D);
    lay.gcarry = c.take<float>((size_t)std::max(ngroups, 1) * D);
    lay.grmax = o.freeze_prefix ? c.take<uint32_t>((size_t)std::max(ngroups, 1) * (D / 16))
                                : nullptr;
    lay.r64 = o.stop == PN_STOP_DELTA_INF
                  ? c.take<char>(residual64_workspace(PN_CELL_GRU, D, Dx, hb)) : nullptr;
    lay.bytes = c.bytes();
    return lay;
}

typedef void (*GruQKernel)(GruQArgs);

template <int D, int DX, int L>
static void gruq_get(GruQKernel* k, int* nt) {
    *k = gru_quasi_local_kernel<D, DX, L>;
    *nt = GruQ<D, DX, L>::NT;
}

static bool gruq_lookup(int D, int Dx, int L, GruQKernel* k, int* nt) {
#define PN_GQ(d, dx, ll) if (D == d && Dx == dx && L == ll) { gruq_get<d, dx, ll>(k, nt); return true; }
#define PN_GQL(d, dx) PN_GQ(d, dx, 32) PN_GQ(d, dx, 64) PN_GQ(d, dx, 128)
    // (64, 64) has no 128-step tiles: their staging would exceed the 160 KB of LDS
    PN_GQL(64, 32) PN_GQL(48, 24) PN_GQL(32, 16) PN_GQL(16, 8) PN_GQL(16, 16)
    PN_GQ(64, 64, 32) PN_GQ(64, 64, 64)
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
    (void)D; (void)Dx;
    if (o.tile == 32 || o.tile == 64 || o.tile == 128) return o.tile;
    return 64;
}

// Tiles per group: enough groups to give every resident workgroup about two of them, at most
// 16 tiles (a longer group only shortens the carry scan, which is already cheap).
int gru_group_tiles(int ntiles, int resident) {
    return std::max(1, std::min(16, ntiles / std::max(1, 2 * resident)));
}

int gru_resident(const void* kern, int nt) {
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, nt, 0) != hipSuccess || occ < 1)
        occ = 1;
    return cu_count() * occ;
}

size_t gru_quasi_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    const int L = gru_quasi_tile(D, Dx, o);
    GruQKernel kern;
    int nt;
    if (!gruq_lookup(D, Dx, L, &kern, &nt)) return 0;
    const std::vector<int32_t> ts = tile_starts(hb, L);
    const int ntiles = ts[hb.B];
    const int gt = o.group > 0 ? o.group : gru_group_tiles(ntiles, gru_resident((const void*)kern, nt));
    return gruq_layout(nullptr, D, Dx, hb, ntiles, count_groups(ts, hb.B, gt), o).bytes;
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
    const int resident = gru_resident((const void*)kern, nt);
    const int gt = o.group > 0 ? o.group : gru_group_tiles(ntiles, resident);
    const int ngroups = count_groups(ts, hb.B, gt);
    GruQLayout lay = gruq_layout(ws, D, Dx, hb, ntiles, ngroups, o);
    const bool bydelta = o.stop == PN_STOP_DELTA_INF;
    // the update-norm rule sees convergence one update later: cap T + 1 (Alg. alg:deer)
    const int max_iters = o.max_iters > 0 ? o.max_iters
                                          : (int)std::max<int64_t>(1, hb.Tmax) + (bydelta ? 1 : 0);
    PN_TRY(init_iter_state(lay.st, hb, ts, L, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream, gt, o.stop));
    const int grid = std::max(1, std::min(ngroups, resident));

    GruQArgs args;
    args.x = x;
    args.s0 = s0;
    args.params = (const float*)cd.params;
    for (int p = 0; p < 2; ++p) args.lac[p] = lay.lac[p];
    args.gagg = lay.gagg;
    args.gcarry = lay.gcarry;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.tiles = lay.st.tiles;
    args.groups = lay.st.groups;
    args.ngroups = ngroups;
    args.grmax = lay.grmax;
    args.freeze = o.freeze_prefix ? 1 : 0;
    args.mode = o.jac == PN_JAC_PICARD ? kTransIdentity
              : o.jac == PN_JAC_JACOBI ? kTransZero : kTransDiag;
    args.sbuf[0] = s;
    args.sbuf[1] = lay.salt;
    args.dscale = o.damping == PN_DAMP_SCALE ? 1.f - o.damp_k : 1.f;
    args.clip = o.damping == PN_DAMP_CLIP ? 1 : 0;
    args.clo = o.clip_lo;
    args.chi = o.clip_hi;

    // iteration k forms s^(k) in sbuf[k & 1] from sbuf[(k + 1) & 1] (k from the control
    // block, so a captured graph of iterations replays from any k), then the carries
    auto one_iter = [&](hipStream_t st) {
        prof_launch("gru_quasi_local", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), 0, s2, args);
        });
        prof_launch("carry_scan", st, [&](hipStream_t s2) {
            launch_carry_scan(lay.gagg, lay.gcarry, lay.st, hb.B, D, s2, lay.grmax, D / 16);
        });
        launch_decide(lay.st, hb.B, st, true);
    };
    std::vector<uintptr_t> key = {0x6752u, (uintptr_t)kern, (uintptr_t)grid, (uintptr_t)x,
                                  (uintptr_t)s0, (uintptr_t)s, (uintptr_t)cd.params,
                                  (uintptr_t)ws, (uintptr_t)hb.B, (uintptr_t)ntiles,
                                  (uintptr_t)ngroups, (uintptr_t)args.mode,
                                  (uintptr_t)o.damping, float_bits(args.dscale),
                                  float_bits(args.clo), float_bits(args.chi),
                                  (uintptr_t)args.freeze, (uintptr_t)hb.N, lay.bytes};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key,
                          one_iter, stream));
    PN_TRY(finish_iterations(lay.st, hb, D, sizeof(float), s, lay.salt, stream, info, all_conv));
    if (bydelta && info) {
        // the loop tested update norms; the reported residual is the FP64 one of the result
        std::vector<double> r64(hb.B);
        PN_TRY(residual64_run(cd, hb, x, s0, s, lay.r64, stream, r64.data()));
        for (int b = 0; b < hb.B; ++b) info[b].max_resid = r64[b];
    }
    return PN_OK;
}

}  // namespace pn
