// Scan-tile autotuner: measures the tile and group lengths of the two-pass scans on the
// caller's inputs and keeps the fastest per shape class (in the process, and optionally in a
// JSON file named by PN_AUTOTUNE_CACHE).  Host code only: every candidate is an ordinary call
// of the public solve entry points, timed with HIP events on the caller's stream.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pn_host.hpp"

namespace pn {

namespace {

struct Cand {
    int tile;
    int group;
};

std::mutex g_mu;
std::map<std::string, Cand> g_cache;          // measured or loaded in this process

int bit_length(int64_t v) {
    int n = 0;
    while (v > 0) { ++n; v >>= 1; }
    return n;
}

std::vector<Cand> candidates(int op, const pn_cell_desc& c, const pn_opts& o) {
    static const int kGroups[] = {0, 1, 2, 4, 8, 16};
    std::vector<Cand> v;
    if (op == PN_OP_DEER && c.cell == PN_CELL_GRU && c.dtype == PN_F32 &&
        (o.jac == PN_JAC_DIAG || o.jac == PN_JAC_PICARD || o.jac == PN_JAC_JACOBI)) {
        for (int t : {32, 64, 128})
            for (int g : kGroups) v.push_back({t, g});
    } else if (op == PN_OP_ADJOINT && c.cell == PN_CELL_GRU && o.jac == PN_JAC_DENSE) {
        // the dense reverse scan's group length sets how many chain waves there are against
        // the resident slots, so its optimum falls between the powers of two
        for (int g : {0, 1, 2, 3, 4, 5, 6, 8, 16}) v.push_back({0, g});
    } else if ((op == PN_OP_DEER && c.cell == PN_CELL_TANH && o.jac == PN_JAC_DENSE &&
                c.dtype == PN_F32) ||
               op == PN_OP_ADJOINT) {
        for (int g : kGroups) v.push_back({0, g});
    } else if (op == PN_OP_ELK) {
        for (int t : {0, 16, 32, 64, 128, 256}) v.push_back({t, 0});
    } else {
        v.push_back({0, 0});
    }
    return v;
}

std::string make_key(int op, const pn_cell_desc& c, const HostBatch& hb, const pn_opts& o,
                     double lambda) {
    char buf[320];
    std::snprintf(buf, sizeof buf,
                  "gfx950/cu%d/op%d/cell%d/D%d/Dx%d/dt%d/jac%d/cmp%d/damp%d/kf%d/sm%d/fz%d/"
                  "graph%d_%d/B%d/N%d/T%d",
                  cu_count(), op, c.cell, c.D, c.Dx, c.dtype, o.jac, o.compose, o.damping,
                  op == PN_OP_ELK && lambda > 0 ? 1 : 0, o.smooth, o.freeze_prefix,
                  o.use_graph, o.graph_iters, hb.B, bit_length(hb.N), bit_length(hb.Tmax));
    return buf;
}

// The cache file: a JSON object {"key": [tile, group], ...}, one entry a line.
void load_file(const char* path, std::map<std::string, Cand>& out) {
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        const char* q0 = std::strchr(line, '"');
        if (!q0) continue;
        const char* q1 = std::strchr(q0 + 1, '"');
        if (!q1) continue;
        int t = 0, g = 0;
        const char* br = std::strchr(q1, '[');
        if (!br || std::sscanf(br, "[%d , %d]", &t, &g) != 2) continue;
        out[std::string(q0 + 1, q1)] = Cand{t, g};
    }
    std::fclose(f);
}

void store_file(const char* path, const std::string& key, Cand c) {
    std::map<std::string, Cand> all;
    load_file(path, all);                     // keep entries other processes wrote
    all[key] = c;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;                           // an unwritable cache only costs a re-tune
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : all)
        std::fprintf(f, "  \"%s\": [%d, %d]%s\n", kv.first.c_str(), kv.second.tile,
                     kv.second.group, ++i < all.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t saved_bytes(int op, const pn_cell_desc& c, const HostBatch& hb) {
    if (op == PN_OP_ADJOINT) return 0;
    return round256((size_t)hb.N * c.D * (c.dtype == PN_F64 ? 8 : 4));
}

pn_status run_op(int op, const pn_cell_desc& c, const pn_batch& b, const void* const* bufs,
                 double lambda, const pn_opts& o, void* ws, size_t wsb, void* stream) {
    switch (op) {
        case PN_OP_DEER:
            return deer_solve(&c, &b, bufs[0], bufs[1], (void*)bufs[2], &o, ws, wsb, stream,
                              nullptr);
        case PN_OP_ELK:
            return elk_solve(&c, &b, bufs[0], bufs[1], (void*)bufs[2], lambda, &o, ws, wsb,
                             stream, nullptr);
        case PN_OP_ADJOINT:
            return deer_adjoint(&c, &b, bufs[0], bufs[1], bufs[2], bufs[3], (void*)bufs[4],
                                (void*)bufs[5], (void*)bufs[6], &o, ws, wsb, stream, nullptr);
        default:
            set_error("pn_autotune: unknown op %d", op);
            return PN_ERR_INVALID_ARG;
    }
}

}  // namespace

pn_status autotune_workspace(int op, const pn_cell_desc& c, const pn_batch& b,
                             const HostBatch& hb, const pn_opts& o, size_t* bytes) {
    if (op != PN_OP_DEER && op != PN_OP_ELK && op != PN_OP_ADJOINT) {
        set_error("PN_OP_TUNE applies to PN_OP_DEER, PN_OP_ELK or PN_OP_ADJOINT");
        return PN_ERR_INVALID_ARG;
    }
    size_t need = 0;
    bool any = false;
    for (const Cand& k : candidates(op, c, o)) {
        pn_opts oc = o;
        oc.tile = k.tile;
        oc.group = k.group;
        size_t n = 0;
        if (pn_workspace_bytes(op, &c, &b, &oc, &n) == PN_OK) {
            need = std::max(need, n);
            any = true;
        }
    }
    if (!any) return pn_workspace_bytes(op, &c, &b, &o, bytes);   // its own error
    *bytes = saved_bytes(op, c, hb) + need;
    return PN_OK;
}

}  // namespace pn

using namespace pn;

extern "C" pn_status pn_autotune(int op, const pn_cell_desc* cell, const pn_batch* batch,
                                 const void* const* bufs, double lambda, const pn_opts* opts,
                                 int32_t probe_iters, void* workspace, size_t workspace_bytes,
                                 void* stream, pn_tuned* out) {
    if (!out || !bufs) { set_error("pn_autotune: out and bufs must not be NULL"); return PN_ERR_INVALID_ARG; }
    if (op != PN_OP_DEER && op != PN_OP_ELK && op != PN_OP_ADJOINT) {
        set_error("pn_autotune: op must be PN_OP_DEER, PN_OP_ELK or PN_OP_ADJOINT");
        return PN_ERR_INVALID_ARG;
    }
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    const pn_opts o = resolve_opts(opts);
    PN_TRY(check_opts(o));
    if (probe_iters <= 0) probe_iters = 3;
    if (probe_iters > 64) { set_error("probe_iters must be at most 64"); return PN_ERR_INVALID_ARG; }
    if (!bufs[0] || !bufs[1] || !bufs[2] ||
        (op == PN_OP_ADJOINT && (!bufs[3] || !bufs[6]))) {
        set_error("pn_autotune: a required buffer is NULL");
        return PN_ERR_INVALID_ARG;
    }
    std::memset(out, 0, sizeof *out);
    const std::string key = make_key(op, *cell, hb, o, lambda);
    const char* path = std::getenv("PN_AUTOTUNE_CACHE");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it == g_cache.end() && path && *path) {
            std::map<std::string, Cand> file;
            load_file(path, file);
            auto f = file.find(key);
            if (f != file.end()) it = g_cache.emplace(key, f->second).first;
        }
        if (it != g_cache.end()) {
            out->tile = it->second.tile;
            out->group = it->second.group;
            out->from_cache = 1;
            return PN_OK;
        }
    }
    size_t need = 0;
    PN_TRY(autotune_workspace(op, *cell, *batch, hb, o, &need));
    if (!workspace || workspace_bytes < need) {
        set_error("pn_autotune: workspace of %zu bytes needed", need);
        return PN_ERR_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t sv = saved_bytes(op, *cell, hb);
    char* save = (char*)workspace;
    void* ws = save + sv;
    const size_t wsb = workspace_bytes - sv;
    void* s = (void*)bufs[2];
    if (sv) PN_HIP(hipMemcpyAsync(save, s, sv, hipMemcpyDeviceToDevice, st));
    hipEvent_t e0, e1;
    PN_HIP(hipEventCreate(&e0));
    PN_HIP(hipEventCreate(&e1));
    const std::vector<Cand> cands = candidates(op, *cell, o);
    // The dense GRU adjoint is not an iteration of equal launches (one map pass, a walk, chain
    // passes until its residual test passes): its candidates are timed as whole calls at the
    // caller's tolerance, and ms_per_iter reports milliseconds per call.
    const bool whole = op == PN_OP_ADJOINT && cell->cell == PN_CELL_GRU && o.jac == PN_JAC_DENSE;
    const int per = whole ? 1 : probe_iters;
    double best = INFINITY;
    Cand bestc{o.tile, o.group};
    pn_status err = PN_OK;
    for (const Cand& k : cands) {
        if (out->ncand >= PN_TUNE_MAX_CAND) break;
        pn_opts oc = o;
        oc.tile = k.tile;
        oc.group = k.group;
        oc.tol = 1e-300;                      // below any FP32 residual: every probe iteration runs
        oc.max_iters = probe_iters;
        oc.fp64_final_residual = 0;
        if (whole) {                          // the GRU dense adjoint: time whole calls
            oc.tol = o.tol;
            oc.max_iters = 0;
        }
        float ms = -1.f;
        pn_status r = PN_OK;
        // a warm-up call (plan, graph), then two timed ones: the faster counts (a single timing
        // moves by a few per cent, about the gap between neighbouring candidates)
        for (int rep = 0; rep < 3 && r >= 0; ++rep) {
            if (sv && (r = (hipMemcpyAsync(s, save, sv, hipMemcpyDeviceToDevice, st) == hipSuccess
                                ? PN_OK : PN_ERR_HIP)) < 0)
                break;
            if (rep >= 1 && hipEventRecord(e0, st) != hipSuccess) { r = PN_ERR_HIP; break; }
            r = run_op(op, *cell, *batch, bufs, lambda, oc, ws, wsb, stream);
            if (rep >= 1 && r >= 0) {
                float t = 0.f;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                    r = PN_ERR_HIP;
                    ms = -1.f;
                } else if (ms < 0.f || t < ms) {
                    ms = t;
                }
            }
        }
        if (r == PN_ERR_INVALID_ARG || r == PN_ERR_UNSUPPORTED) {
            ms = -1.f;                        // the route does not take this candidate
        } else if (r < 0) {
            err = r;
            break;
        }
        const int i = out->ncand++;
        out->cand_tile[i] = k.tile;
        out->cand_group[i] = k.group;
        out->cand_ms[i] = ms < 0 ? -1.f : ms / per;
        if (ms >= 0 && ms < best) {
            best = ms;
            bestc = k;
        }
    }
    if (sv) hipMemcpyAsync(s, save, sv, hipMemcpyDeviceToDevice, st);
    hipStreamSynchronize(st);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (err < 0) return err;
    if (!std::isfinite(best)) {
        set_error("pn_autotune: no candidate ran for this route");
        return PN_ERR_UNSUPPORTED;
    }
    out->tile = bestc.tile;
    out->group = bestc.group;
    out->ms_per_iter = best / per;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = bestc;
    if (path && *path) store_file(path, key, bestc);
    return PN_OK;
}

extern "C" void pn_autotune_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
}
