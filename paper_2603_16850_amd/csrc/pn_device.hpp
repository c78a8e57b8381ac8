// Device-side building blocks shared by the gfx950 kernels: the solver state records, the
// MFMA wrapper and the gate nonlinearities.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PN_DEV __device__ __forceinline__

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace pn {

// ---- per-sequence solver state (device) ---------------------------------------------------
enum SeqStatus : int { kActive = 0, kConverged = 1, kCapped = 2 };

struct SeqState {
    int status;         // SeqStatus
    int iters;          // updates applied to the final iterate
    int resets;         // resets in kept iterates
    int resets_pending; // resets in the iterate being produced this iteration
    int parity;         // which ping-pong buffer holds the final iterate
    uint32_t maxr;      // running max |r| of the current iterate (float bits, >= 0)
    float final_resid;  // max |r| of the final iterate
    int frozen;         // converged-prefix skipping: groups of the sequence frozen so far
    int frozen_prev;    // ... and before the latest update of `frozen`
    uint32_t maxd;      // running max |s^(k) - s^(k-1)| of the update that formed the current
                        // iterate (float bits; the update-norm stopping rule)
};

// One entry per tile, indexed by scan slot (see IterState::tiles).
constexpr int kTileScanFirst = 1;   // the sequence's first scanned tile
constexpr int kTileTimeFirst = 2;   // the sequence's first tile in time (rows from its start)
struct TileInfo {
    int32_t slot;       // scan slot of the tile (consecutive within a sequence, scan order)
    int32_t b;          // sequence
    int32_t len;        // valid steps (rows row0 .. row0+len-1)
    int32_t flags;      // kTileScanFirst | kTileTimeFirst
    int64_t row0;       // first row
    int32_t gslot;      // group of the tile (see GroupInfo)
    int32_t hgslot;     // group of the tile scanned just before it in its sequence, -1 if none
};

// A group is a run of consecutive tiles of one sequence, in scan order, that one workgroup
// scans one after the other (IterState::groups, indexed by group slot).
struct GroupInfo {
    int32_t b;          // sequence
    int32_t tile0;      // slot of the group's first tile
    int32_t ntl;        // tiles in the group
    int32_t gfirst;     // group slot of the sequence's first group
};

struct Ctrl {
    int iter;           // index k of the iterate the next main kernel linearises
    int all_done;       // 1 when no sequence is active
    int max_iters;
    float tol;
    float reset_abs;
    int done_iter;      // the iteration whose decision stopped the last sequence (-1 before)
    int stop_delta;     // 1: the stopping test reads maxd (update norm) instead of maxr
};

// ---- control-block reads ------------------------------------------------------------------
// The stop flag is written by the previous kernel of the stream; a relaxed agent-scope load
// reads it past the non-coherent per-XCD L2.
PN_DEV int ld_i32(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// |v| as orderable bits; NaN counts as +inf so it never passes a stopping test.
PN_DEV uint32_t absbits(float v) {
    float a = fabsf(v);
    return (a <= 3.402823466e38f) ? __float_as_uint(a) : 0x7F800000u;
}

// ---- MFMA (gfx950 matrix cores) ---------------------------------------------------------------
// v_mfma_f32_16x16x4_f32: D(16x16) += A(16x4) * B(4x16).
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, element i holds D[4 * (l / 16) + i][l % 16].
PN_DEV floatx4 mfma16x4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---- math ---------------------------------------------------------------------------------------
PN_DEV float sigmoidf_(float a) { return 1.0f / (1.0f + __expf(-a)); }
PN_DEV float tanhf_(float a) {
    // tanh a = 1 - 2 / (exp(2a) + 1); saturates correctly for large |a|
    return 1.0f - 2.0f / (__expf(2.0f * a) + 1.0f);
}
// The same with the hardware reciprocal v_rcp_f32 (error at most 1 ulp) instead of an IEEE
// division (about ten instructions), for the GRU gates: a few ulp of error in f, far below the
// tolerances of the (contracting) GRU solves, at a third of the instruction count.  The tanh
// cells keep the divisions: their unstable dense recurrences amplify evaluation error.
PN_DEV float sigmoid_rcp(float a) { return __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }
PN_DEV float tanh_rcp(float a) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * a) + 1.0f);   // rcp(inf) = 0
}

PN_DEV int lane_id() { return __lane_id(); }

// ---- cross-lane sums on the VALU ---------------------------------------------------------------
// x + x of lane l ^ 32 (sum_halves) or lane l ^ 16 (sum_rows16), the same bits on both lanes
// of a pair.  v_permlane32_swap / v_permlane16_swap exchange the two halves of the wave (the odd
// and even 16-lane rows) between two registers; swapping x with itself leaves x of one lane of
// the pair in each result register, and their sum does not depend on which.  Unlike a shuffle
// (ds_bpermute) this does not go through the LDS unit.
PN_DEV float sum_halves(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
PN_DEV float sum_rows16(float x) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

}  // namespace pn
