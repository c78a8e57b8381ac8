// Parallel Newton methods on the affine test cells (D <= 16, FP32):
//   PN_CELL_AFFINE        f_t(h) = M h + N x_t + c
//   PN_CELL_AFFINE_STEPS  f_t(h) = M_t h + N x_t + c   (one matrix per step)
// A linear dynamical system (Ch. 2, eq. lds) has the constant Jacobian A_t = M (or M_t), so
// one DEER update lands on the trajectory; with a diagonal M one quasi-DEER update does
// (eq. quasi_lds), and the input-dependent permutation LDS of the group word problem (Ch. 6,
// Prop. cayley) is solved by one Newton update while the diagonal, Picard and Jacobi
// transitions need about T.  These cells put those facts through the GPU scan.
//
// Structure as the dense paths: steps are cut into chunks of 64, one single-wave workgroup per
// chunk.  Iteration k:
//   local pass: (k >= 1) replay the previous update over the chunk from the carry entering it,
//     Delta_t = A~_t Delta_{t-1} - r^(k-1)_t, s^(k) = s^(k-1) + Delta with the reset guard;
//     then linearise at s^(k) (residual r_t, its maximum, the update norm) and compose the
//     chunk's map Delta_end = P Delta_in + q, P = A~_end ... A~_first, from the leaves
//     (A~_t, -r_t) (eq. bin_op_affine);
//   carry pass: one wave per sequence walks its chunk maps from Delta = 0.
// A~_t is M_t (dense), diag(M_t) (quasi), I (Picard) or 0 (Jacobi); A~ = 0 at a sequence head.
// State vectors are padded to 16 entries; the padding stays zero.
#include <algorithm>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

constexpr int AD = 16;          // padded state size
constexpr int AL = 64;          // chunk length
constexpr int AB = 16;          // steps whose transitions are staged at once
constexpr int AMS = AD + 1;     // LDS row stride of a 16x16 matrix
constexpr int AMAP = AD * AD + AD;   // chunk map: P (row-major), q

struct AffArgs {
    const float* x;
    const float* s0;
    float* sbuf[2];          // ping-pong iterates: s^(k) lives in sbuf[k & 1]
    const float* M;          // constant M (D x D), or NULL
    const float* Mt;         // per-step M_t ([N][D][D]), or NULL
    const float* Nx;         // N (D x Dx)
    const float* c;          // c (D)
    float* gmap;             // [ntiles][AMAP] chunk maps of this iteration
    const float* gcarry;     // [ntiles][AD] Delta entering every chunk (previous iteration)
    Ctrl* ctrl;
    SeqState* seq;
    const TileInfo* tiles;
    int ntiles;
    int D, Dx;
    int mode;                // 0 dense, 1 diagonal, 2 identity (Picard), 3 zero (Jacobi)
};

// Transitions of steps [tb, tb + AB) of the chunk into Ab (A~_t, padded, by `mode`), rows
// row0 + tb.. of the batch; A~ = 0 at the sequence head.
PN_DEV void aff_stage_transitions(float* Ab, const AffArgs& a, int64_t row0, int tb, int len,
                                  bool first) {
    const int l = threadIdx.x & 63;
    for (int idx = l; idx < AB * AD * AD; idx += 64) {
        const int q = idx / (AD * AD), i = (idx / AD) % AD, j = idx % AD;
        const int t = tb + q;
        float v = 0.f;
        if (t < len && i < a.D && j < a.D && !(first && t == 0)) {
            if (a.mode == 2) {
                v = i == j ? 1.f : 0.f;
            } else if (a.mode != 3 && (a.mode == 0 || i == j)) {
                v = a.Mt ? a.Mt[((size_t)(row0 + t) * a.D + i) * a.D + j] : a.M[i * a.D + j];
            }
        }
        Ab[(q * AD + i) * AMS + j] = v;
    }
}

// r_t = s_t - (M_t s_{t-1} + N x_t + c) for the chunk's steps, sl rows 0..len (row 0 = s_{t0-1});
// returns this lane's max |r| over valid entries (float bits)
PN_DEV uint32_t aff_residual(float* rl, const float* sl, const AffArgs& a, int64_t row0, int len) {
    const int l = threadIdx.x & 63;
    uint32_t rm = 0;
    for (int idx = l; idx < AL * AD; idx += 64) {
        const int t = idx / AD, i = idx % AD;
        float r = 0.f;
        if (t < len && i < a.D) {
            const float* h = sl + t * AD;
            const float* Mrow = a.Mt ? a.Mt + ((size_t)(row0 + t) * a.D + i) * a.D : a.M + i * a.D;
            float f = a.c[i];
            for (int j = 0; j < a.D; ++j) f = fmaf(Mrow[j], h[j], f);
            const float* xr = a.x + (size_t)(row0 + t) * a.Dx;
            const float* Nr = a.Nx + (size_t)i * a.Dx;
            for (int j = 0; j < a.Dx; ++j) f = fmaf(Nr[j], xr[j], f);
            r = sl[(t + 1) * AD + i] - f;
            rm = max(rm, absbits(r));
        }
        rl[idx] = r;
    }
    __syncthreads();
    return rm;
}

__global__ void __launch_bounds__(64) affine_local_kernel(AffArgs a) {
    __shared__ float sl[(AL + 1) * AD];      // rows s_{t0-1}, s_{t0}, .., s_{t0+len-1}
    __shared__ float rl[AL * AD];            // residuals
    __shared__ float Ab[AB * AD * AMS];      // staged transitions
    __shared__ float P[AD * AMS];            // running chunk map
    __shared__ float q[AD];
    __shared__ float dv[AD];                 // replayed Delta
    __shared__ int rowbad[AL + 1];

    if (ld_i32(&a.ctrl->all_done)) return;
    const int k = a.ctrl->iter;
    const bool fuse = k > 0;
    const float reset_abs = a.ctrl->reset_abs;
    const bool bydelta = a.ctrl->stop_delta != 0;
    const float* sprev = a.sbuf[(k + 1) & 1];
    float* scur = a.sbuf[k & 1];
    const int l = threadIdx.x & 63;

    for (int ti = blockIdx.x; ti < a.ntiles; ti += gridDim.x) {
        const TileInfo tinfo = a.tiles[ti];
        const int b = tinfo.b;
        if (a.seq[b].status != kActive) continue;
        const int len = tinfo.len;
        const int64_t row0 = tinfo.row0;
        const bool first = (tinfo.flags & kTileTimeFirst) != 0;
        const float* src = fuse ? sprev : scur;

        // ---- stage s^(k-1) (or the guess s^(0)): halo row and the chunk's rows
        for (int idx = l; idx < (AL + 1) * AD; idx += 64) {
            const int r = idx / AD, i = idx % AD;
            float v = 0.f;
            if (i < a.D) {
                if (r == 0) v = first ? a.s0[(size_t)b * a.D + i] : src[(size_t)(row0 - 1) * a.D + i];
                else if (r - 1 < len) v = src[(size_t)(row0 + r - 1) * a.D + i];
            }
            sl[idx] = v;
        }
        for (int r = l; r <= AL; r += 64) rowbad[r] = 0;
        __syncthreads();

        uint32_t dmax = 0;
        if (fuse) {
            // ---- replay the previous update: Delta_t = A~_t Delta_{t-1} - r^(k-1)_t
            aff_residual(rl, sl, a, row0, len);
            if (l < AD) dv[l] = a.gcarry[(size_t)ti * AD + l];    // Delta_{t0-1}
            __syncthreads();
            if (!first && l < a.D) {                               // halo row s^(k)_{t0-1}
                const float v = sl[l] + dv[l];
                sl[l] = v;
                if (!(fabsf(v) <= reset_abs)) rowbad[0] = 1;
            }
            for (int tb = 0; tb < len; tb += AB) {
                aff_stage_transitions(Ab, a, row0, tb, len, first);
                __syncthreads();
                for (int t = tb; t < min(len, tb + AB); ++t) {
                    float d = 0.f;
                    if (l < AD) {
                        const float* Ar = Ab + ((t - tb) * AD + l) * AMS;
                        for (int j = 0; j < AD; ++j) d = fmaf(Ar[j], dv[j], d);
                        d -= rl[t * AD + l];
                    }
                    __syncthreads();
                    if (l < AD) {
                        dv[l] = d;
                        if (l < a.D) {
                            const float v = sl[(t + 1) * AD + l] + d;
                            sl[(t + 1) * AD + l] = v;
                            dmax = max(dmax, absbits(d));
                            if (!(fabsf(v) <= reset_abs)) rowbad[t + 1] = 1;
                        }
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
            // reset guard, then s^(k) of the chunk's rows to HBM
            for (int idx = l; idx < (AL + 1) * AD; idx += 64) {
                const int r = idx / AD, i = idx % AD;
                if (r > 0 && r - 1 >= len) continue;
                if (r == 0 && first) continue;
                if (rowbad[r]) sl[idx] = 0.f;
                if (r > 0 && i < a.D) scur[(size_t)(row0 + r - 1) * a.D + i] = sl[idx];
            }
            int nb = 0;
            for (int r = 1 + l; r <= AL; r += 64) nb += (r - 1 < len && rowbad[r]) ? 1 : 0;
            for (int off = 32; off >= 1; off >>= 1) nb += __shfl_xor(nb, off);
            if (l == 0 && nb) atomicAdd(&a.seq[b].resets_pending, nb);
            __syncthreads();
        }

        // ---- linearise at s^(k) and compose the chunk map from the leaves (A~_t, -r_t)
        const uint32_t rmax = aff_residual(rl, sl, a, row0, len);
        for (int idx = l; idx < AD * AD; idx += 64) {
            const int i = idx / AD, j = idx % AD;
            P[i * AMS + j] = (i == j && i < a.D) ? 1.f : 0.f;
        }
        if (l < AD) q[l] = 0.f;
        __syncthreads();
        const int i = l & 15, cb = 4 * (l >> 4);
        for (int tb = 0; tb < len; tb += AB) {
            aff_stage_transitions(Ab, a, row0, tb, len, first);
            __syncthreads();
            for (int t = tb; t < min(len, tb + AB); ++t) {
                const float* Ar = Ab + ((t - tb) * AD + i) * AMS;
                float p4[4] = {0.f, 0.f, 0.f, 0.f};
                float qv = 0.f;
                for (int j = 0; j < AD; ++j) {
                    const float av = Ar[j];
#pragma unroll
                    for (int e = 0; e < 4; ++e) p4[e] = fmaf(av, P[j * AMS + cb + e], p4[e]);
                    qv = fmaf(av, q[j], qv);
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < 4; ++e) P[i * AMS + cb + e] = p4[e];
                if (l < AD) q[l] = qv - rl[t * AD + l];
                __syncthreads();
            }
        }
        float* gm = a.gmap + (size_t)ti * AMAP;
        for (int idx = l; idx < AD * AD; idx += 64) gm[idx] = P[(idx / AD) * AMS + idx % AD];
        if (l < AD) gm[AD * AD + l] = q[l];

        uint32_t m = bydelta ? dmax : rmax;
        for (int off = 32; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
        uint32_t mr = rmax;
        for (int off = 32; off >= 1; off >>= 1) mr = max(mr, (uint32_t)__shfl_xor((int)mr, off));
        if (l == 0) {
            atomicMax(&a.seq[b].maxr, mr);
            if (bydelta) atomicMax(&a.seq[b].maxd, m);
        }
        __syncthreads();
    }
}

// One wave per sequence: Delta entering each chunk, from Delta = 0 at the sequence start.
__global__ void __launch_bounds__(64) affine_carry_kernel(const float* __restrict__ gmap,
                                                          float* __restrict__ gcarry,
                                                          const Ctrl* ctrl, const SeqState* seq,
                                                          const int32_t* tile_start, int B) {
    if (ld_i32(&ctrl->all_done)) return;
    const int b = blockIdx.x;
    if (b >= B || seq[b].status != kActive) return;
    const int l = threadIdx.x & 63;
    float cur = 0.f;                       // lane i < 16 holds entry i
    for (int c = tile_start[b]; c < tile_start[b + 1]; ++c) {
        if (l < AD) gcarry[(size_t)c * AD + l] = cur;
        const float* gm = gmap + (size_t)c * AMAP;
        float nv = l < AD ? gm[AD * AD + l] : 0.f;
        for (int j = 0; j < AD; ++j) {
            const float cj = __shfl(cur, j);
            if (l < AD) nv = fmaf(gm[l * AD + j], cj, nv);
        }
        cur = nv;
    }
}

// ---- host ---------------------------------------------------------------------------------

bool affine_supported(int D, int Dx) { return D >= 1 && D <= AD && Dx >= 1 && Dx <= 64; }

struct AffLayout {
    IterState st;
    float* salt;
    float* gmap;
    float* gcarry;
    size_t bytes;
};

static AffLayout aff_layout(void* ws, const HostBatch& hb, int D, int ntiles) {
    Carver c(ws);
    AffLayout lay;
    carve_iter_state(c, lay.st, hb.B, ntiles, 0);
    lay.salt = c.take<float>((size_t)hb.N * D);
    lay.gmap = c.take<float>((size_t)std::max(ntiles, 1) * AMAP);
    lay.gcarry = c.take<float>((size_t)std::max(ntiles, 1) * AD);
    lay.bytes = c.bytes();
    return lay;
}

size_t affine_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o) {
    (void)Dx;
    (void)o;
    const std::vector<int32_t> ts = tile_starts(hb, AL);
    return aff_layout(nullptr, hb, D, ts[hb.B]).bytes;
}

pn_status affine_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                         const float* s0, float* s, const pn_opts& o, void* ws,
                         hipStream_t stream, pn_seq_info* info, bool* all_conv) {
    const int D = cd.D, Dx = cd.Dx;
    const std::vector<int32_t> ts = tile_starts(hb, AL);
    const int ntiles = ts[hb.B];
    AffLayout lay = aff_layout(ws, hb, D, ntiles);
    const bool bydelta = o.stop == PN_STOP_DELTA_INF;
    const int max_iters = o.max_iters > 0 ? o.max_iters
                                          : (int)std::max<int64_t>(1, hb.Tmax) + (bydelta ? 1 : 0);
    PN_TRY(init_iter_state(lay.st, hb, ts, AL, false, max_iters, (float)o.tol,
                           (float)o.reset_abs, stream, 0, o.stop));
    const float* p = (const float*)cd.params;
    AffArgs args{};
    args.x = x;
    args.s0 = s0;
    args.sbuf[0] = s;
    args.sbuf[1] = lay.salt;
    const bool steps = cd.cell == PN_CELL_AFFINE_STEPS;
    const size_t mcount = steps ? (size_t)hb.N * D * D : (size_t)D * D;
    args.M = steps ? nullptr : p;
    args.Mt = steps ? p : nullptr;
    args.Nx = p + mcount;
    args.c = p + mcount + (size_t)D * Dx;
    args.gmap = lay.gmap;
    args.gcarry = lay.gcarry;
    args.ctrl = lay.st.ctrl;
    args.seq = lay.st.seq;
    args.tiles = lay.st.tiles;
    args.ntiles = ntiles;
    args.D = D;
    args.Dx = Dx;
    args.mode = o.jac == PN_JAC_DENSE ? 0 : o.jac == PN_JAC_DIAG ? 1 : o.jac == PN_JAC_PICARD ? 2 : 3;
    const int grid = std::max(1, std::min(ntiles, 4 * cu_count()));
    auto one_iter = [&](hipStream_t st) {
        prof_launch("affine_local", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(affine_local_kernel, dim3(grid), dim3(64), 0, s2, args);
        });
        prof_launch("affine_carry", st, [&](hipStream_t s2) {
            hipLaunchKernelGGL(affine_carry_kernel, dim3(std::max(1, hb.B)), dim3(64), 0, s2,
                               (const float*)lay.gmap, lay.gcarry, (const Ctrl*)lay.st.ctrl,
                               (const SeqState*)lay.st.seq, (const int32_t*)lay.st.tile_start,
                               hb.B);
        });
        launch_decide(lay.st, hb.B, st, true);
    };
    std::vector<uintptr_t> key = {0x4166u, (uintptr_t)grid, (uintptr_t)x, (uintptr_t)s0,
                                  (uintptr_t)s, (uintptr_t)cd.params, (uintptr_t)ws,
                                  (uintptr_t)hb.B, (uintptr_t)hb.N, (uintptr_t)ntiles,
                                  (uintptr_t)D, (uintptr_t)Dx, (uintptr_t)args.mode,
                                  (uintptr_t)steps, lay.bytes};
    PN_TRY(run_iterations(lay.st, max_iters + 1, o.graph_iters, o.use_graph != 0, key, one_iter,
                          stream));
    PN_TRY(finish_iterations(lay.st, hb, D, sizeof(float), s, lay.salt, stream, info, all_conv));
    return PN_OK;
}

}  // namespace pn
