// Device-side building blocks shared by the gfx950 kernels.
//
// Cross-workgroup communication (the decoupled look-back of the scans) uses only relaxed
// 32/64-bit atomic loads and stores at agent scope.  On gfx950 those bypass the per-XCD
// L2 (which is not coherent between XCDs) without the L2 write-back / invalidate that an
// agent-scope release/acquire fence costs.  No ordering between different words is needed
// because every published word validates itself: a slot holds a signalling-NaN sentinel
// until it is written, and no arithmetic result can equal that pattern (arithmetic NaNs are
// quiet).  Payloads that could carry a NaN are canonicalised to the quiet NaN first.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PN_DEV __device__ __forceinline__

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace pn {

constexpr uint32_t kSent32 = 0x7FA5A5A5u;                  // signalling NaN: "not published"
constexpr uint64_t kSent64 = 0x7FA5A5A57FA5A5A5ull;        // both halves the same pattern
constexpr uint32_t kQNaN = 0x7FC00000u;

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
    int pad_;
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
    uint32_t tile_counter;
    int error;          // nonzero: device-side check failed (look-back watchdog)
    int max_iters;
    float tol;
    float reset_abs;
    int done_iter;      // the iteration whose decision stopped the last sequence (-1 before)
};

// ---- atomics ------------------------------------------------------------------------------
PN_DEV uint64_t ld_u64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
PN_DEV void st_u64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
PN_DEV uint32_t ld_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
PN_DEV void st_u32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
PN_DEV int ld_i32(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

PN_DEV float canon(float v) { return (v != v) ? __uint_as_float(kQNaN) : v; }

PN_DEV uint64_t pack2(float lo, float hi) {
    return (uint64_t)__float_as_uint(canon(lo)) | ((uint64_t)__float_as_uint(canon(hi)) << 32);
}
PN_DEV float lo_of(uint64_t v) { return __uint_as_float((uint32_t)v); }
PN_DEV float hi_of(uint64_t v) { return __uint_as_float((uint32_t)(v >> 32)); }
PN_DEV bool ready64(uint64_t v) { return (uint32_t)v != kSent32; }
PN_DEV bool ready32(uint32_t v) { return v != kSent32; }

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

}  // namespace pn
