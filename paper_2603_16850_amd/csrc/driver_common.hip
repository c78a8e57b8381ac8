// Host helpers and control kernels shared by every iterative solver.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace pn {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

const char* last_error() { return g_last_error.c_str(); }

pn_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
    set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return PN_ERR_HIP;
}

int cu_count() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) n = p.multiProcessorCount;
        if (n <= 0) n = 256;
    }
    return n;
}

// ---- event timing ------------------------------------------------------------------------
namespace {
struct ProfPending {
    std::string family;
    std::pair<hipEvent_t, hipEvent_t> ev;
    int iter;               // iteration the launch belongs to (-1: outside an iteration loop)
};
struct ProfRec {
    bool on = false;
    int cur_iter = -1;
    std::map<std::string, std::pair<double, int64_t>> totals;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<ProfPending> pending;
};
ProfRec& prof() {
    static thread_local ProfRec r;
    return r;
}
}  // namespace

// No-allocation mode of the calling thread (the entry point that works from the library's
// static scratch array): no pinned host buffers, no graph instantiation, no event timing.
static thread_local bool g_noalloc = false;
void set_noalloc(bool on) { g_noalloc = on; }
bool noalloc() { return g_noalloc; }

bool profiling() { return prof().on && !g_noalloc; }

void prof_launch(const char* family, hipStream_t stream,
                 const std::function<void(hipStream_t)>& launch) {
    ProfRec& r = prof();
    if (!r.on || g_noalloc) {
        launch(stream);
        return;
    }
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!r.pool.empty()) {
        ev = r.pool.back();
        r.pool.pop_back();
    } else {
        (void)hipEventCreate(&ev.first);
        (void)hipEventCreate(&ev.second);
    }
    (void)hipEventRecord(ev.first, stream);
    launch(stream);
    (void)hipEventRecord(ev.second, stream);
    r.pending.push_back({family, ev, r.cur_iter});
}

// Launches of iterations after `last` found every sequence stopped and returned at once: they
// are counted apart, under the family name with "#idle" appended.
static void prof_drop_after(int last) {
    ProfRec& r = prof();
    std::vector<ProfPending> keep;
    for (auto& p : r.pending) {
        if (p.iter > last) {
            float ms = 0.f;
            if (hipEventSynchronize(p.ev.second) == hipSuccess &&
                hipEventElapsedTime(&ms, p.ev.first, p.ev.second) == hipSuccess) {
                auto& t = r.totals[p.family + "#idle"];
                t.first += ms;
                t.second += 1;
            }
            r.pool.push_back(p.ev);
        } else {
            keep.push_back(p);
        }
    }
    r.pending.swap(keep);
}

void prof_collect() {
    ProfRec& r = prof();
    for (auto& p : r.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.ev.second) == hipSuccess &&
            hipEventElapsedTime(&ms, p.ev.first, p.ev.second) == hipSuccess) {
            auto& t = r.totals[p.family];
            t.first += ms;
            t.second += 1;
        }
        r.pool.push_back(p.ev);
    }
    r.pending.clear();
    r.cur_iter = -1;
}

void profile_begin() {
    ProfRec& r = prof();
    r.on = true;
    r.totals.clear();
}
void profile_end() { prof().on = false; }
int profile_read(const char* family, double* ms, int64_t* n) {
    ProfRec& r = prof();
    auto it = r.totals.find(family);
    if (it == r.totals.end()) return 0;
    if (ms) *ms = it->second.first;
    if (n) *n = it->second.second;
    return 1;
}

std::vector<int32_t> tile_starts(const HostBatch& hb, int L) {
    std::vector<int32_t> ts(hb.B + 1, 0);
    for (int b = 0; b < hb.B; ++b) ts[b + 1] = ts[b] + (int32_t)((hb.len(b) + L - 1) / L);
    return ts;
}

void carve_iter_state(Carver& c, IterState& st, int B, int ntiles, int ngroups) {
    st.ctrl = c.take<Ctrl>(1);
    st.seq = c.take<SeqState>(B);
    st.offsets = c.take<int64_t>(B + 1);
    st.tile_start = c.take<int32_t>(B + 1);
    st.tiles = c.take<TileInfo>(std::max(ntiles, 1));
    st.groups = c.take<GroupInfo>(std::max(ngroups, 1));
    st.group_start = c.take<int32_t>(B + 1);
    st.ngroups = ngroups;
}

int count_groups(const std::vector<int32_t>& tstart, int B, int gt) {
    int n = 0;
    for (int b = 0; b < B; ++b) n += (tstart[b + 1] - tstart[b] + gt - 1) / gt;
    return n;
}

__global__ void init_state_kernel(Ctrl* ctrl, SeqState* seq, const int64_t* offsets, int B,
                                  int max_iters, float tol, float reset_abs, int stop_delta) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        SeqState q;
        const bool empty = offsets[b + 1] == offsets[b];
        q.status = empty ? kConverged : kActive;
        q.iters = 0;
        q.resets = 0;
        q.resets_pending = 0;
        q.parity = 0;
        q.maxr = 0;
        q.final_resid = 0.0f;
        q.frozen = 0;
        q.frozen_prev = 0;
        q.maxd = 0;
        seq[b] = q;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl c;
        c.iter = 0;
        c.all_done = 0;
        c.max_iters = max_iters;
        c.tol = tol;
        c.reset_abs = reset_abs;
        c.done_iter = -1;
        c.stop_delta = stop_delta;
        *ctrl = c;
    }
}

namespace {
// Thread-local pinned staging buffers, grown as needed and kept until the process ends.  Copies
// from or to pinned memory are asynchronous DMA (a pageable copy stages through a driver buffer
// and stalls the stream); a buffer is reused only by the next call on the same thread, after
// the previous call synchronised its stream.
void* pinned_staging(int which, size_t bytes) {
    if (g_noalloc) {
        // pageable host memory (plain host heap, no HIP allocation); the copies through it
        // are staged by the runtime
        static thread_local std::vector<char> pageable[2];
        if (pageable[which].size() < bytes) pageable[which].resize(bytes);
        return pageable[which].data();
    }
    struct Buf { void* p = nullptr; size_t n = 0; };
    static thread_local Buf bufs[2];
    Buf& b = bufs[which];
    if (b.n < bytes) {
        if (b.p) (void)hipHostFree(b.p);
        b.p = nullptr;
        b.n = 0;
        const size_t n = std::max(bytes, (size_t)64 << 10);
        if (hipHostMalloc(&b.p, n, hipHostMallocDefault) != hipSuccess) return nullptr;
        b.n = n;
    }
    return b.p;
}
}  // namespace

// Tile and group tables from the offsets, one thread per tile (and per group): the same
// geometry the host used to build (a host loop over a large ragged batch's 10^5 tiles cost
// about 2 ms per call while the device waited, plus a 4 MB upload).  Sequence b of slot i is
// the last b with tile_start[b] <= i (empty sequences own no slot).
__global__ void build_tables_kernel(const int64_t* __restrict__ offsets,
                                    const int32_t* __restrict__ tstart,
                                    const int32_t* __restrict__ gstart, int B, int L, int reverse,
                                    int g, int ntiles, int ngroups, TileInfo* __restrict__ tiles,
                                    GroupInfo* __restrict__ groups) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    auto owner = [&](const int32_t* start, int v) {
        int lo = 0, hi = B - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= v) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    if (i < ntiles) {
        const int b = owner(tstart, i);
        const int nt = tstart[b + 1] - tstart[b], k = i - tstart[b];
        const int lt = reverse ? nt - 1 - k : k;                     // tile index in time
        TileInfo ti;
        ti.slot = i;
        ti.b = b;
        ti.len = (int)min((int64_t)L, offsets[b + 1] - offsets[b] - (int64_t)lt * L);
        ti.flags = (k == 0 ? kTileScanFirst : 0) | (lt == 0 ? kTileTimeFirst : 0);
        ti.row0 = offsets[b] + (int64_t)lt * L;
        ti.gslot = gstart[b] + k / g;
        ti.hgslot = k > 0 ? gstart[b] + (k - 1) / g : -1;
        tiles[i] = ti;
    }
    if (groups && i < ngroups) {
        const int b = owner(gstart, i);
        const int nt = tstart[b + 1] - tstart[b], j = i - gstart[b];
        groups[i] = GroupInfo{b, tstart[b] + j * g, min(g, nt - j * g), gstart[b]};
    }
}

pn_status init_iter_state(const IterState& st, const HostBatch& hb,
                          const std::vector<int32_t>& tstart, int L, bool reverse,
                          int max_iters, float tol, float reset_abs, hipStream_t stream,
                          int gt, int stop) {
    // The host sends the offsets, the tile starts and the group starts (O(B) values); the
    // tables themselves are built on the device.
    static thread_local std::vector<int32_t> gstart;
    const int ntiles = tstart[hb.B];
    gstart.assign(hb.B + 1, 0);
    const int g = gt > 0 ? gt : 1;
    for (int b = 0; b < hb.B; ++b) gstart[b + 1] = gstart[b] + (tstart[b + 1] - tstart[b] + g - 1) / g;
    const int ngroups = gt > 0 ? gstart[hb.B] : 0;
    if (gt > 0 && ngroups != st.ngroups) {
        set_error("internal: group table size %d, carved %d", ngroups, st.ngroups);
        return PN_ERR_INTERNAL;
    }
    // offsets and tile_start are carved next to each other, group_start after the tables
    char* const d0 = (char*)st.offsets;
    const size_t head = (size_t)((char*)(st.tile_start + hb.B + 1) - d0);
    const size_t gbytes = sizeof(int32_t) * (hb.B + 1);
    char* h = (char*)pinned_staging(0, head + gbytes);
    if (!h) {
        set_error("hipHostMalloc of %zu bytes for the tile tables failed", head + gbytes);
        return PN_ERR_HIP;
    }
    std::memcpy(h, hb.offsets.data(), sizeof(int64_t) * (hb.B + 1));
    std::memcpy(h + ((char*)st.tile_start - d0), tstart.data(), sizeof(int32_t) * (hb.B + 1));
    std::memcpy(h + head, gstart.data(), gbytes);
    PN_HIP(hipMemcpyAsync(d0, h, head, hipMemcpyHostToDevice, stream));
    PN_HIP(hipMemcpyAsync(st.group_start, h + head, gbytes, hipMemcpyHostToDevice, stream));
    const int nthreads = std::max(ntiles, ngroups);
    if (nthreads > 0) {
        hipLaunchKernelGGL(build_tables_kernel, dim3((nthreads + 255) / 256), dim3(256), 0,
                           stream, (const int64_t*)st.offsets, (const int32_t*)st.tile_start,
                           (const int32_t*)st.group_start, hb.B, L, reverse ? 1 : 0, g, ntiles,
                           ngroups, st.tiles, gt > 0 ? st.groups : nullptr);
        PN_HIP(hipGetLastError());
    }
    int blocks = std::min(64, (hb.B + 255) / 256);
    hipLaunchKernelGGL(init_state_kernel, dim3(std::max(1, blocks)), dim3(256), 0, stream,
                       st.ctrl, st.seq, st.offsets, hb.B, max_iters, tol, reset_abs,
                       stop == PN_STOP_DELTA_INF ? 1 : 0);
    PN_HIP(hipGetLastError());
    return PN_OK;
}

// ---- input scan for non-finite values (opts->check_inputs) ---------------------------------
// flag |= 1 if any element of p[0 .. n) is NaN or infinite.  Grid-stride, one write per wave
// that finds one.
template <class T>
__global__ void nonfinite_kernel(const T* __restrict__ p, int64_t n, int* flag) {
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(p[i]);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ void clear_flag_kernel(int* flag) { *flag = 0; }

pn_status check_finite(std::initializer_list<std::pair<const void*, int64_t>> arrays, int dtype,
                       int* flag_dev, hipStream_t stream) {
    static thread_local int* pinned_flag = nullptr;
    static thread_local int pageable_flag = 0;
    if (!g_noalloc && !pinned_flag &&
        hipHostMalloc((void**)&pinned_flag, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        pinned_flag = nullptr;
        set_error("hipHostMalloc of the input-check flag failed");
        return PN_ERR_HIP;
    }
    int* hflag = g_noalloc ? &pageable_flag : pinned_flag;
    // cleared by a kernel rather than a memset node, so the check stays capturable
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, stream, flag_dev);
    for (const auto& a : arrays) {
        if (!a.first || a.second <= 0) continue;
        const int64_t n = a.second;
        const int blocks = (int)std::min<int64_t>(2048, (n + 255) / 256);
        if (dtype == PN_F64)
            hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                               (const double*)a.first, n, flag_dev);
        else
            hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(blocks), dim3(256), 0, stream,
                               (const float*)a.first, n, flag_dev);
    }
    PN_HIP(hipGetLastError());
    PN_HIP(hipMemcpyAsync(hflag, flag_dev, sizeof(int), hipMemcpyDeviceToHost, stream));
    PN_HIP(hipStreamSynchronize(stream));
    if (*hflag) {
        set_error("an input holds a NaN or an infinity");
        return PN_ERR_NONFINITE_INPUT;
    }
    return PN_OK;
}

// ---- sum of per-workgroup partials ------------------------------------------------------------
// out[i] = sum_k part[k * P + i] in FP64, rounded once to FP32.  A workgroup takes 64 columns and
// splits the partials over 16 rows of threads (loads of a row are coalesced over the columns);
// the 16 row sums are added in a fixed order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(1024) partial_sum_kernel(const float* __restrict__ part,
                                                            int nparts, int P,
                                                            float* __restrict__ out) {
    __shared__ double red[16][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + c;
    double acc = 0.0;
    if (i < P) {
#pragma unroll 8
        for (int k = r; k < nparts; k += 16) acc += (double)part[(size_t)k * P + i];
    }
    red[r][c] = acc;
    __syncthreads();
    if (r == 0 && i < P) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += red[q][c];
        out[i] = (float)t;
    }
}

void launch_partial_sum(const float* part, int nparts, int P, float* out, hipStream_t stream) {
    if (P <= 0) return;
    hipLaunchKernelGGL(partial_sum_kernel, dim3((P + 63) / 64), dim3(1024), 0, stream, part,
                       nparts, P, out);
}

// One workgroup: apply the stopping test of iteration k to every active sequence.  The tested
// quantity is the residual max of the iterate s^(k), or with the update-norm rule the max of
// the update that formed it (never passed at k = 0, before any update).
// resets_pending counts the rows reset while this iteration produced an iterate: the next
// iterate s^(k+1) (kept only if the sequence goes on), or with `pending_current` the iterate
// s^(k) just tested (always kept).
__global__ void decide_kernel(Ctrl* ctrl, SeqState* seq, int B, int pending_current) {
    __shared__ int any_active;
    const int k = ctrl->iter;
    const float tol = ctrl->tol;
    const int cap = ctrl->max_iters;
    const bool by_delta = ctrl->stop_delta != 0;
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        SeqState q = seq[b];
        if (q.status == kActive) {
            const float m = __uint_as_float(q.maxr);
            const bool pass = by_delta ? (k > 0 && __uint_as_float(q.maxd) < tol) : (m < tol);
            if (pass || k >= cap) {
                q.status = pass ? kConverged : kCapped;
                q.iters = k;
                q.parity = k & 1;
                q.final_resid = m;
                if (pending_current) q.resets += q.resets_pending;
            } else {
                q.resets += q.resets_pending;
                any_active = 1;
            }
            q.maxr = 0;
            q.maxd = 0;
            q.resets_pending = 0;
            seq[b] = q;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (!any_active && !ctrl->all_done) ctrl->done_iter = k;
        ctrl->iter = k + 1;
        ctrl->all_done = any_active ? 0 : 1;
    }
}

void launch_decide(const IterState& st, int B, hipStream_t stream, bool pending_current) {
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(256), 0, stream, st.ctrl, st.seq, B,
                       pending_current ? 1 : 0);
}

// ---- iteration loop with optional graph capture -------------------------------------------

namespace {
// Instantiated graphs of `n` iterations, kept per key (solver, kernels, buffers, shapes) so
// that later calls on the same buffers skip instantiation.  A call always captures its own
// iterations first and brings the cached executable up to date with hipGraphExecUpdate, so
// the kernels run with exactly the arguments of this call (plan values and workspace offsets
// that move with the shapes included) whether or not the key says everything; a capture whose
// node structure differs (another plan) is instantiated afresh.  Executables are shared
// pointers: an entry evicted from the cache is destroyed only after the last call holding it
// has synchronised its stream and let go of it.
struct ExecHolder {
    hipGraphExec_t exec = nullptr;
    ~ExecHolder() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};
using ExecPtr = std::shared_ptr<ExecHolder>;
struct CacheEntry {
    ExecPtr exec;
    uint64_t last_use = 0;
};
struct GraphCache {
    std::mutex mu;
    std::map<std::vector<uintptr_t>, CacheEntry> execs;
    uint64_t tick = 0;
};
constexpr size_t kGraphCacheMax = 64;
GraphCache& graph_cache() {
    static GraphCache* c = new GraphCache();   // lives until process exit
    return *c;
}

struct PinnedCtrl {
    Ctrl* p = nullptr;
    PinnedCtrl() { (void)hipHostMalloc((void**)&p, sizeof(Ctrl), hipHostMallocDefault); }
};
Ctrl* pinned_ctrl() {
    if (g_noalloc) {
        static thread_local Ctrl pageable;
        return &pageable;
    }
    static thread_local PinnedCtrl pc;
    return pc.p;
}

// Captures n iterations on this thread's capture stream.
pn_status capture_iterations(int n, const std::function<void(hipStream_t)>& one_iter,
                             hipGraph_t* graph) {
    static thread_local hipStream_t cs = nullptr;
    if (!cs) PN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    PN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < n; ++i) one_iter(cs);
    PN_HIP(hipStreamEndCapture(cs, graph));
    return PN_OK;
}

// The executable for this call's captured graph: the cached one of `key` updated to it, or a
// new instantiation (then cached, evicting the least recently used entries beyond the limit).
pn_status exec_for(const std::vector<uintptr_t>& key, hipGraph_t graph, ExecPtr* out) {
    GraphCache& gc = graph_cache();
    ExecPtr cand;
    {
        std::lock_guard<std::mutex> lock(gc.mu);
        auto it = gc.execs.find(key);
        if (it != gc.execs.end()) {
            cand = it->second.exec;
            it->second.last_use = ++gc.tick;
        }
    }
    if (cand) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(cand->exec, graph, &err_node, &res) == hipSuccess &&
            res == hipGraphExecUpdateSuccess) {
            *out = cand;
            return PN_OK;
        }
        (void)hipGetLastError();       // a failed update is not an error of the call
    }
    auto fresh = std::make_shared<ExecHolder>();
    PN_HIP(hipGraphInstantiate(&fresh->exec, graph, nullptr, nullptr, 0));
    {
        std::lock_guard<std::mutex> lock(gc.mu);
        gc.execs[key] = CacheEntry{fresh, ++gc.tick};
        while (gc.execs.size() > kGraphCacheMax) {
            auto oldest = gc.execs.begin();
            for (auto it = gc.execs.begin(); it != gc.execs.end(); ++it)
                if (it->second.last_use < oldest->second.last_use) oldest = it;
            gc.execs.erase(oldest);    // destroyed when its last holder lets go
        }
    }
    *out = fresh;
    return PN_OK;
}
}  // namespace

pn_status run_iterations(const IterState& st, int max_launches, int graph_iters,
                         bool use_graph, const std::vector<uintptr_t>& graph_key,
                         const std::function<void(hipStream_t)>& one_iter,
                         hipStream_t stream) {
    Ctrl* hc = pinned_ctrl();
    if (!hc) {
        set_error("hipHostMalloc of the control readback buffer failed");
        return PN_ERR_HIP;
    }
    graph_iters = std::max(1, graph_iters);
    int launched = 0;
    ExecPtr exec;       // this call's executable, held until the call returns
    while (launched < max_launches) {
        const int n = std::min(graph_iters, max_launches - launched);
        if (use_graph && n == graph_iters && !profiling() && !g_noalloc) {
            if (!exec) {
                int dev = 0;
                PN_HIP(hipGetDevice(&dev));
                std::vector<uintptr_t> key = graph_key;
                key.push_back((uintptr_t)n);
                key.push_back((uintptr_t)dev);
                hipGraph_t graph = nullptr;
                PN_TRY(capture_iterations(n, one_iter, &graph));
                const pn_status r = exec_for(key, graph, &exec);
                (void)hipGraphDestroy(graph);
                PN_TRY(r);
            }
            PN_HIP(hipGraphLaunch(exec->exec, stream));
        } else {
            for (int i = 0; i < n; ++i) {
                prof().cur_iter = launched + i;
                one_iter(stream);
            }
            prof().cur_iter = -1;
            PN_HIP(hipGetLastError());
        }
        launched += n;
        PN_HIP(hipMemcpyAsync(hc, st.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
        PN_HIP(hipStreamSynchronize(stream));
        if (hc->all_done && profiling()) prof_drop_after(hc->done_iter);
        if (hc->all_done) break;
    }
    return PN_OK;
}

template <class T>
__global__ void copy_odd_parity_kernel(const SeqState* seq, const int64_t* offsets, int D,
                                       T* dst, const T* src) {
    const int b = blockIdx.y;
    if (seq[b].parity == 0) return;
    const int64_t a = offsets[b] * D, e = offsets[b + 1] * D;
    for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < e;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

pn_status finish_iterations(const IterState& st, const HostBatch& hb, int D, size_t elem,
                            void* s_user, const void* s_alt, hipStream_t stream,
                            pn_seq_info* info, bool* all_converged) {
    if (s_alt) {
        const int64_t per = hb.Tmax * D;
        int gx = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (per + 255) / 256));
        dim3 grid(gx, hb.B);
        if (elem == 4)
            hipLaunchKernelGGL(copy_odd_parity_kernel<float>, grid, dim3(256), 0, stream,
                               st.seq, st.offsets, D, (float*)s_user, (const float*)s_alt);
        else
            hipLaunchKernelGGL(copy_odd_parity_kernel<double>, grid, dim3(256), 0, stream,
                               st.seq, st.offsets, D, (double*)s_user, (const double*)s_alt);
        PN_HIP(hipGetLastError());
    }
    // control block and per-sequence states (carved next to each other) in one pinned copy
    const size_t span = (size_t)((char*)(st.seq + hb.B) - (char*)st.ctrl);
    char* h = (char*)pinned_staging(1, span);
    if (!h) {
        set_error("hipHostMalloc of %zu bytes for the solver state failed", span);
        return PN_ERR_HIP;
    }
    PN_HIP(hipMemcpyAsync(h, st.ctrl, span, hipMemcpyDeviceToHost, stream));
    PN_HIP(hipStreamSynchronize(stream));
    Ctrl hc;
    std::memcpy(&hc, h, sizeof(Ctrl));
    const SeqState* hs = (const SeqState*)(h + ((char*)st.seq - (char*)st.ctrl));
    bool allc = true;
    for (int b = 0; b < hb.B; ++b) {
        const bool conv = hs[b].status == kConverged;
        allc = allc && conv;
        if (info) {
            info[b].iters = hs[b].iters;
            info[b].converged = conv ? 1 : 0;
            info[b].resets = hs[b].resets;
            info[b].pad_ = 0;
            info[b].max_resid = hs[b].final_resid;
        }
    }
    *all_converged = allc;
    prof_collect();
    return PN_OK;
}

}  // namespace pn
