// Host-side helpers shared by the solver drivers: error reporting, workspace carving,
// device properties, the per-iteration control kernels and the iteration loop with
// optional hipGraph capture.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "pnewton.h"
#include "pn_device.hpp"

namespace pn {

void set_error(const char* fmt, ...);
pn_status hip_fail(hipError_t e, const char* what, const char* file, int line);

#define PN_HIP(call)                                                            \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) return ::pn::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define PN_TRY(expr)                        \
    do {                                    \
        pn_status s_ = (expr);              \
        if (s_ < 0) return s_;              \
    } while (0)

// Bit pattern of a float (graph-cache keys).
inline uintptr_t float_bits(float v) {
    uint32_t u;
    std::memcpy(&u, &v, sizeof u);
    return (uintptr_t)u;
}

struct HostBatch {
    int B = 0;
    int64_t N = 0;
    std::vector<int64_t> offsets;   // B+1
    int64_t Tmax = 0;
    int64_t len(int b) const { return offsets[b + 1] - offsets[b]; }
};

// Carves 256-byte aligned pieces out of the caller's workspace (or only measures when
// base is null).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

int cu_count();

// No-allocation mode of the calling thread: pageable host staging, direct launches, no event
// timing (the static-scratch entry point sets it around its call).
void set_noalloc(bool on);
bool noalloc();

// Event timing of kernel launches (pn_profile_begin / pn_profile_read).
bool profiling();
// Records an event pair around `launch(stream)` when profiling, else just launches.
void prof_launch(const char* family, hipStream_t stream, const std::function<void(hipStream_t)>& launch);
// Resolves the pending event pairs of this thread (after the stream was synchronised).
void prof_collect();

// Tile table: tile_start[b] = number of tiles of sequences < b, for tiles of L steps.
std::vector<int32_t> tile_starts(const HostBatch& hb, int L);

// argument validation of the entry points (api.hip)
pn_opts resolve_opts(const pn_opts* o);
pn_status check_cell(const pn_cell_desc* cell);
pn_status check_batch(const pn_batch* batch, HostBatch& hb);
pn_status check_opts(const pn_opts& o);
// workspace of pn_autotune (autotune.hip)
pn_status autotune_workspace(int op, const pn_cell_desc& c, const pn_batch& b,
                             const HostBatch& hb, const pn_opts& o, size_t* bytes);

// State shared by every iterative solver (lives in the workspace).
struct IterState {
    Ctrl* ctrl;
    SeqState* seq;
    int64_t* offsets;      // device copy [B+1]
    int32_t* tile_start;   // device [B+1]
    TileInfo* tiles;       // device [ntiles]: every tile's geometry, indexed by slot
    GroupInfo* groups;     // device [ngroups], indexed by group slot
    int32_t* group_start;  // device [B+1]: group slots of sequence b
    int ngroups;
};
// Tile slots of sequence b are tile_start[b] .. tile_start[b+1]-1, numbered in the order a
// sequence is scanned (from its start, or from its end for reverse scans).
// Groups cut each sequence's slots into runs of `gt` tiles (the last one shorter).
void carve_iter_state(Carver& c, IterState& st, int B, int ntiles, int ngroups = 0);
// Number of groups of `gt` tiles over the sequences of a batch.
int count_groups(const std::vector<int32_t>& tstart, int B, int gt);

// Uploads offsets / tile table, resets the per-sequence state and the control block.
// Tiles are L steps long; with `reverse` a sequence is scanned from its end (its last tile
// gets the sequence's first slot).
// `gt` > 0 also fills the group table (the state must have been carved with
// count_groups(tstart, B, gt) groups).
pn_status init_iter_state(const IterState& st, const HostBatch& hb,
                          const std::vector<int32_t>& tstart, int L, bool reverse,
                          int max_iters, float tol, float reset_abs, hipStream_t stream,
                          int gt = 0, int stop = PN_STOP_RESID_INF);

// Launches the end-of-iteration decision kernel (stop tests, counters).
// `pending_current`: the resets counted during the iteration belong to the iterate that was
// tested (solvers that form s^(k) at the start of iteration k), not to the next one.
void launch_decide(const IterState& st, int B, hipStream_t stream, bool pending_current = false);

// out[i] = sum over k < nparts of part[k * P + i] (FP64 sums in a fixed order, one FP32
// rounding): the reduction of per-workgroup gradient partials.
void launch_partial_sum(const float* part, int nparts, int P, float* out, hipStream_t stream);

// Runs `one_iter` (which enqueues one iteration: main kernels + decide) until every
// sequence is done, checking convergence on the host every `graph_iters` iterations;
// with use_graph the batch of iterations is captured once and replayed.
pn_status run_iterations(const IterState& st, int max_launches, int graph_iters,
                         bool use_graph, const std::vector<uintptr_t>& graph_key,
                         const std::function<void(hipStream_t)>& one_iter,
                         hipStream_t stream);

// Copies the final iterate from the alternate buffer for sequences whose final parity is
// odd, and reads the per-sequence info back to the host.
pn_status finish_iterations(const IterState& st, const HostBatch& hb, int D, size_t elem,
                            void* s_user, const void* s_alt, hipStream_t stream,
                            pn_seq_info* info, bool* all_converged);

}  // namespace pn
