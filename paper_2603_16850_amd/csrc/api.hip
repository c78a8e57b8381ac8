// extern "C" entry points: argument validation (before any HIP call) and dispatch.
#include <cmath>
#include <cstring>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

using namespace pn;

// layouts the Python binding mirrors with ctypes
static_assert(sizeof(pn_opts) == 80, "pn_opts layout");
static_assert(sizeof(pn_cell_desc) == 24 && sizeof(pn_batch) == 24 && sizeof(pn_seq_info) == 24,
              "struct layouts");

// validation shared with the autotuner
namespace pn {

pn_opts resolve_opts(const pn_opts* o) {
    pn_opts r;
    pn_default_opts(&r);
    if (o) r = *o;
    if (r.graph_iters <= 0) r.graph_iters = 4;
    if (!(r.reset_abs > 0)) r.reset_abs = 1e4;
    return r;
}

pn_status check_cell(const pn_cell_desc* cell) {
    if (!cell) { set_error("cell descriptor is NULL"); return PN_ERR_INVALID_ARG; }
    if (cell->cell < PN_CELL_GRU || cell->cell > PN_CELL_AFFINE_STEPS) {
        set_error("unknown cell kind %d", cell->cell);
        return PN_ERR_INVALID_ARG;
    }
    if (cell->D < 1 || cell->Dx < 1 || cell->D > 4096 || cell->Dx > 4096) {
        set_error("bad sizes D=%d Dx=%d", cell->D, cell->Dx);
        return PN_ERR_INVALID_ARG;
    }
    if (cell->dtype != PN_F32 && cell->dtype != PN_F64) {
        set_error("unknown dtype %d", cell->dtype);
        return PN_ERR_INVALID_ARG;
    }
    if (!cell->params) { set_error("params is NULL"); return PN_ERR_INVALID_ARG; }
    return PN_OK;
}

pn_status check_batch(const pn_batch* batch, HostBatch& hb) {
    if (!batch) { set_error("batch descriptor is NULL"); return PN_ERR_INVALID_ARG; }
    if (batch->B < 1 || batch->N < 0) {
        set_error("bad batch B=%d N=%lld", batch->B, (long long)batch->N);
        return PN_ERR_INVALID_ARG;
    }
    hb.B = batch->B;
    hb.N = batch->N;
    hb.offsets.assign(batch->B + 1, 0);
    if (batch->offsets) {
        if (batch->offsets[0] != 0) { set_error("offsets[0] must be 0"); return PN_ERR_INVALID_ARG; }
        for (int b = 0; b < batch->B; ++b) {
            if (batch->offsets[b + 1] < batch->offsets[b]) {
                set_error("offsets must be non-decreasing (at %d)", b);
                return PN_ERR_INVALID_ARG;
            }
            hb.offsets[b + 1] = batch->offsets[b + 1];
        }
        if (hb.offsets[batch->B] != batch->N) {
            set_error("offsets[B]=%lld differs from N=%lld", (long long)hb.offsets[batch->B],
                      (long long)batch->N);
            return PN_ERR_INVALID_ARG;
        }
    } else {
        if (batch->N % batch->B) { set_error("N not divisible by B and no offsets given"); return PN_ERR_INVALID_ARG; }
        const int64_t T = batch->N / batch->B;
        for (int b = 0; b <= batch->B; ++b) hb.offsets[b] = (int64_t)b * T;
    }
    hb.Tmax = 0;
    for (int b = 0; b < hb.B; ++b) hb.Tmax = std::max(hb.Tmax, hb.len(b));
    if (hb.Tmax > (int64_t)1 << 30) { set_error("sequence too long"); return PN_ERR_INVALID_ARG; }
    return PN_OK;
}

pn_status check_opts(const pn_opts& o) {
    if (o.jac < PN_JAC_DENSE || o.jac > PN_JAC_JACOBI) { set_error("unknown jac %d", o.jac); return PN_ERR_INVALID_ARG; }
    if (o.compose != PN_COMPOSE_NATIVE && o.compose != PN_COMPOSE_BF16) {
        set_error("unknown compose %d", o.compose);
        return PN_ERR_INVALID_ARG;
    }
    if (!(o.tol > 0) || !std::isfinite(o.tol)) { set_error("tol must be positive and finite"); return PN_ERR_INVALID_ARG; }
    if (o.tile < 0) { set_error("tile must be >= 0"); return PN_ERR_INVALID_ARG; }
    if (o.group < 0 || o.group > 64) { set_error("group must be 0..64"); return PN_ERR_INVALID_ARG; }
    if (o.freeze_prefix != 0 && o.freeze_prefix != 1) {
        set_error("freeze_prefix must be 0 or 1");
        return PN_ERR_INVALID_ARG;
    }
    if (o.smooth != 0 && o.smooth != 1) {
        set_error("smooth must be 0 or 1");
        return PN_ERR_INVALID_ARG;
    }
    if (o.stop != PN_STOP_RESID_INF && o.stop != PN_STOP_DELTA_INF) {
        set_error("unknown stop rule %d", o.stop);
        return PN_ERR_INVALID_ARG;
    }
    if (o.check_inputs != 0 && o.check_inputs != 1) {
        set_error("check_inputs must be 0 or 1");
        return PN_ERR_INVALID_ARG;
    }
    if (o.damping < PN_DAMP_NONE || o.damping > PN_DAMP_CLIP) {
        set_error("unknown damping %d", o.damping);
        return PN_ERR_INVALID_ARG;
    }
    if (o.damping == PN_DAMP_SCALE && !(o.damp_k >= 0.f && o.damp_k <= 1.f)) {
        set_error("damp_k must lie in [0, 1]");
        return PN_ERR_INVALID_ARG;
    }
    if (o.damping == PN_DAMP_CLIP) {
        if (!(o.clip_lo >= -1.f && o.clip_lo <= o.clip_hi && o.clip_hi <= 1.f)) {
            set_error("clip bounds must satisfy -1 <= clip_lo <= clip_hi <= 1");
            return PN_ERR_INVALID_ARG;
        }
        if (o.jac == PN_JAC_DENSE) {
            set_error("clip damping applies to diagonal transitions only");
            return PN_ERR_INVALID_ARG;
        }
    }
    return PN_OK;
}

}  // namespace pn

namespace {

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

pn_status check_ptrs(std::initializer_list<const void*> must, const HostBatch& hb) {
    if (hb.N == 0) return PN_OK;
    for (const void* p : must) {
        if (!p) { set_error("a required array pointer is NULL"); return PN_ERR_INVALID_ARG; }
        if (!aligned16(p)) { set_error("device arrays must be 16-byte aligned"); return PN_ERR_INVALID_ARG; }
    }
    return PN_OK;
}

pn_status check_ws(void* ws, size_t have, size_t need) {
    if (need == 0) return PN_OK;
    if (!ws || have < need) {
        set_error("workspace too small: need %zu bytes, have %zu", need, have);
        return PN_ERR_WORKSPACE;
    }
    if (((uintptr_t)ws & 255u) != 0) { set_error("workspace must be 256-byte aligned"); return PN_ERR_WORKSPACE; }
    return PN_OK;
}

// Which solver serves a deer_solve call.
enum class Route { None, GruQuasi, GruDenseAdj, GruDense64, TanhDense, MfDense, Elk, Affine };

bool affine_cell(int cell) { return cell == PN_CELL_AFFINE || cell == PN_CELL_AFFINE_STEPS; }

// Number of packed parameters of a cell (the affine cell with per-step matrices holds N of them).
int64_t param_count(const pn_cell_desc& c, int64_t N) {
    const int64_t D = c.D, Dx = c.Dx;
    switch (c.cell) {
        case PN_CELL_GRU: return 3 * D * Dx + 3 * D * D + 4 * D;
        case PN_CELL_AFFINE_STEPS: return N * D * D + D * Dx + D;
        default: return D * D + D * Dx + D;
    }
}

// Bytes the input scan adds at the end of a workspace.
constexpr size_t kCheckBytes = 256;

Route route_deer(const pn_cell_desc& c, const pn_opts& o) {
    if (affine_cell(c.cell) && c.dtype == PN_F32 && o.compose == PN_COMPOSE_NATIVE &&
        o.damping == PN_DAMP_NONE && affine_supported(c.D, c.Dx))
        return Route::Affine;
    if (c.cell == PN_CELL_GRU && c.dtype == PN_F32 && o.compose == PN_COMPOSE_NATIVE &&
        (o.jac == PN_JAC_DIAG || o.jac == PN_JAC_PICARD || o.jac == PN_JAC_JACOBI) &&
        gru_quasi_supported(c.D, c.Dx))
        return Route::GruQuasi;
    if (c.cell == PN_CELL_GRU && o.jac == PN_JAC_DENSE && c.dtype == PN_F64 &&
        o.damping == PN_DAMP_NONE && gru_dense64_supported(c.D, c.Dx))
        return Route::GruDense64;
    if (c.cell == PN_CELL_TANH && o.jac == PN_JAC_DENSE && c.dtype == PN_F32 &&
        o.damping != PN_DAMP_CLIP && tanh_dense_supported(c.D, c.Dx))
        return Route::TanhDense;
    if (c.cell == PN_CELL_MEANFIELD && o.jac == PN_JAC_DENSE && c.dtype == PN_F32 &&
        o.damping == PN_DAMP_NONE && mf_dense_supported(c.D, c.Dx))
        return Route::MfDense;
    return Route::None;
}

// GRU: iterated reverse diagonal scans with an exact VJP residual (damping as the forward);
// tanh D = 32: reverse dense scans (FP32 or BF16 maps), undamped.
Route route_adjoint(const pn_cell_desc& c, const pn_opts& o) {
    if (c.dtype != PN_F32) return Route::None;
    if (c.cell == PN_CELL_GRU && o.jac == PN_JAC_DIAG && gru_quasi_supported(c.D, c.Dx))
        return Route::GruQuasi;
    if (c.cell == PN_CELL_GRU && o.jac == PN_JAC_DENSE && o.damping == PN_DAMP_NONE &&
        gru_quasi_supported(c.D, c.Dx))
        return Route::GruDenseAdj;
    if (c.cell == PN_CELL_TANH && o.jac == PN_JAC_DENSE && o.damping == PN_DAMP_NONE &&
        tanh_dense_supported(c.D, c.Dx))
        return Route::TanhDense;
    return Route::None;
}

}  // namespace

extern "C" {

void pn_default_opts(pn_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->jac = PN_JAC_DIAG;
    o->compose = PN_COMPOSE_NATIVE;
    o->tol = 1e-5;
    o->max_iters = 0;
    o->graph_iters = 4;
    o->reset_abs = 1e4;
    o->fp64_final_residual = 0;
    o->use_graph = 1;
    o->tile = 0;
    o->group = 0;
    o->damping = PN_DAMP_NONE;
    o->damp_k = 0.f;
    o->clip_lo = -1.f;
    o->clip_hi = 1.f;
}

int pn_abi_version(void) { return PN_ABI_VERSION; }

void pn_profile_begin(void) { pn::profile_begin(); }
void pn_profile_end(void) { pn::profile_end(); }
int pn_profile_read(const char* family, double* total_ms, int64_t* launches) {
    if (!family) return 0;
    return pn::profile_read(family, total_ms, launches);
}

const char* pn_last_error(void) { return pn::last_error(); }

const char* pn_status_str(int s) {
    switch (s) {
        case PN_OK: return "PN_OK";
        case PN_NOT_CONVERGED: return "PN_NOT_CONVERGED";
        case PN_ERR_INVALID_ARG: return "PN_ERR_INVALID_ARG";
        case PN_ERR_UNSUPPORTED: return "PN_ERR_UNSUPPORTED";
        case PN_ERR_WORKSPACE: return "PN_ERR_WORKSPACE";
        case PN_ERR_NONFINITE_INPUT: return "PN_ERR_NONFINITE_INPUT";
        case PN_ERR_HIP: return "PN_ERR_HIP";
        case PN_ERR_INTERNAL: return "PN_ERR_INTERNAL";
        default: return "unknown status";
    }
}

pn_status pn_workspace_bytes(int op, const pn_cell_desc* cell, const pn_batch* batch,
                             const pn_opts* opts, size_t* bytes) {
    if (!bytes) { set_error("bytes is NULL"); return PN_ERR_INVALID_ARG; }
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    const pn_opts o = resolve_opts(opts);
    PN_TRY(check_opts(o));
    if (op & PN_OP_TUNE) return autotune_workspace(op & ~PN_OP_TUNE, *cell, *batch, hb, o, bytes);
    if (o.check_inputs && (op == PN_OP_DEER || op == PN_OP_ELK || op == PN_OP_ADJOINT)) {
        pn_opts plain = o;
        plain.check_inputs = 0;
        PN_TRY(pn_workspace_bytes(op, cell, batch, &plain, bytes));
        *bytes = ((*bytes + 255) & ~size_t(255)) + kCheckBytes;
        return PN_OK;
    }
    switch (op) {
        case PN_OP_DEER:
            switch (route_deer(*cell, o)) {
                case Route::GruQuasi: *bytes = gru_quasi_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                case Route::GruDense64: *bytes = gru_dense64_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                case Route::TanhDense: *bytes = tanh_dense_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                case Route::MfDense: *bytes = mf_dense_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                case Route::Affine: *bytes = affine_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                default: break;
            }
            break;
        case PN_OP_ELK:
            if ((cell->cell == PN_CELL_TANH || cell->cell == PN_CELL_MEANFIELD) &&
                cell->dtype == PN_F32 && elk_supported(cell->D, cell->Dx)) {
                *bytes = elk_workspace(cell->D, cell->Dx, hb, o);
                return PN_OK;
            }
            break;
        case PN_OP_ADJOINT:
            switch (route_adjoint(*cell, o)) {
                case Route::GruQuasi:
                case Route::GruDenseAdj: *bytes = gru_adjoint_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                case Route::TanhDense: *bytes = tanh_adjoint_workspace(cell->D, cell->Dx, hb, o); return PN_OK;
                default: break;
            }
            break;
        case PN_OP_SEQ:
            if (cell->dtype == PN_F32 && seq_supported(cell->cell, cell->D, cell->Dx)) {
                *bytes = seq_workspace(cell->cell, cell->D, cell->Dx, hb);
                return PN_OK;
            }
            break;
        case PN_OP_RESIDUAL64:
            if (cell->dtype == PN_F32 && residual64_supported(cell->cell, cell->D, cell->Dx)) {
                *bytes = residual64_workspace(cell->cell, cell->D, cell->Dx, hb);
                return PN_OK;
            }
            break;
        case PN_OP_LLE:
            if (cell->dtype == PN_F32 && lle_supported(cell->cell, cell->D, cell->Dx)) {
                *bytes = lle_workspace(hb);
                return PN_OK;
            }
            break;
        default:
            set_error("unknown op %d", op);
            return PN_ERR_INVALID_ARG;
    }
    set_error("combination not built: op=%d cell=%d D=%d Dx=%d dtype=%d jac=%d compose=%d", op,
              cell->cell, cell->D, cell->Dx, cell->dtype, o.jac, o.compose);
    return PN_ERR_UNSUPPORTED;
}

pn_status deer_solve(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                     const void* s0, void* s, const pn_opts* opts, void* workspace,
                     size_t workspace_bytes, void* stream, pn_seq_info* info) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    const pn_opts o = resolve_opts(opts);
    PN_TRY(check_opts(o));
    PN_TRY(check_ptrs({x, s0, s, cell->params}, hb));
    const Route r = route_deer(*cell, o);
    if (r == Route::None) {
        set_error("deer_solve not built for cell=%d D=%d Dx=%d dtype=%d jac=%d compose=%d",
                  cell->cell, cell->D, cell->Dx, cell->dtype, o.jac, o.compose);
        return PN_ERR_UNSUPPORTED;
    }
    if (o.smooth) {
        set_error("the smoother is built for elk_solve only");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.freeze_prefix && r != Route::GruQuasi) {
        set_error("deer_solve skips converged prefixes on the GRU diagonal path only");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.stop == PN_STOP_DELTA_INF && r != Route::GruQuasi && r != Route::Affine) {
        set_error("the update-norm stopping rule is built for the GRU diagonal path and the "
                  "affine cells");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.stop == PN_STOP_DELTA_INF && o.freeze_prefix) {
        set_error("converged-prefix skipping decides on residuals: use PN_STOP_RESID_INF");
        return PN_ERR_UNSUPPORTED;
    }
    size_t need = 0;
    PN_TRY(pn_workspace_bytes(PN_OP_DEER, cell, batch, &o, &need));
    PN_TRY(check_ws(workspace, workspace_bytes, need));
    hipStream_t st = (hipStream_t)stream;
    if (o.check_inputs) {
        const int64_t P = param_count(*cell, hb.N);
        PN_TRY(check_finite({{x, hb.N * cell->Dx}, {s0, (int64_t)hb.B * cell->D},
                             {cell->params, P}},
                            cell->dtype, (int*)((char*)workspace + need - kCheckBytes), st));
    }
    bool conv = true;
    switch (r) {
        case Route::GruQuasi:
            PN_TRY(gru_quasi_forward(*cell, hb, (const float*)x, (const float*)s0, (float*)s, o,
                                     workspace, st, info, &conv));
            break;
        case Route::GruDense64:
            PN_TRY(gru_dense64_forward(*cell, hb, (const double*)x, (const double*)s0, (double*)s,
                                       o, workspace, st, info, &conv));
            break;
        case Route::TanhDense:
            PN_TRY(tanh_dense_forward(*cell, hb, (const float*)x, (const float*)s0, (float*)s, o,
                                      workspace, st, info, &conv));
            break;
        case Route::MfDense:
            PN_TRY(mf_dense_forward(*cell, hb, (const float*)x, (const float*)s0, (float*)s, o,
                                    workspace, st, info, &conv));
            break;
        case Route::Affine:
            PN_TRY(affine_forward(*cell, hb, (const float*)x, (const float*)s0, (float*)s, o,
                                  workspace, st, info, &conv));
            break;
        default:
            return PN_ERR_INTERNAL;
    }
    return conv ? PN_OK : PN_NOT_CONVERGED;
}

pn_status elk_solve(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                    const void* s0, void* s, double lambda, const pn_opts* opts,
                    void* workspace, size_t workspace_bytes, void* stream, pn_seq_info* info) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    pn_opts o = resolve_opts(opts);
    if (!opts) o.jac = PN_JAC_DENSE;          // ELK proper unless quasi-ELK is asked for
    PN_TRY(check_opts(o));
    if (!(lambda >= 0) || !std::isfinite(lambda)) { set_error("lambda must be finite and >= 0"); return PN_ERR_INVALID_ARG; }
    if (o.jac != PN_JAC_DENSE && o.jac != PN_JAC_DIAG) {
        set_error("elk_solve takes PN_JAC_DENSE (ELK) or PN_JAC_DIAG (quasi-ELK)");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.damping != PN_DAMP_NONE) {
        set_error("elk_solve damps through lambda; damping must be PN_DAMP_NONE");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.smooth && o.freeze_prefix) {
        set_error("the smoother does not combine with converged-prefix skipping");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.stop != PN_STOP_RESID_INF) {
        set_error("elk_solve stops on the residual (PN_STOP_RESID_INF)");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.group != 0) {
        set_error("elk_solve takes its group length as tile (group must be 0)");
        return PN_ERR_INVALID_ARG;
    }
    if (o.tile % 16 != 0 || o.tile > 1024) {
        set_error("elk_solve tile must be 0 or a multiple of 16 up to 1024");
        return PN_ERR_UNSUPPORTED;
    }
    PN_TRY(check_ptrs({x, s0, s, cell->params}, hb));
    if (!((cell->cell == PN_CELL_TANH || cell->cell == PN_CELL_MEANFIELD) &&
          cell->dtype == PN_F32 && elk_supported(cell->D, cell->Dx))) {
        set_error("elk_solve not built for cell=%d D=%d Dx=%d dtype=%d", cell->cell, cell->D,
                  cell->Dx, cell->dtype);
        return PN_ERR_UNSUPPORTED;
    }
    size_t need = 0;
    PN_TRY(pn_workspace_bytes(PN_OP_ELK, cell, batch, &o, &need));
    PN_TRY(check_ws(workspace, workspace_bytes, need));
    if (o.check_inputs)
        PN_TRY(check_finite({{x, hb.N * cell->Dx}, {s0, (int64_t)hb.B * cell->D},
                             {cell->params, param_count(*cell, hb.N)}},
                            cell->dtype, (int*)((char*)workspace + need - kCheckBytes),
                            (hipStream_t)stream));
    bool conv = true;
    PN_TRY(elk_forward(*cell, hb, (const float*)x, (const float*)s0, (float*)s, lambda, o,
                       workspace, (hipStream_t)stream, info, &conv));
    return conv ? PN_OK : PN_NOT_CONVERGED;
}

pn_status deer_adjoint(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                       const void* s0, const void* s, const void* gs, void* gx, void* gs0,
                       void* gparams, const pn_opts* opts, void* workspace,
                       size_t workspace_bytes, void* stream, pn_seq_info* info) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    const pn_opts o = resolve_opts(opts);
    PN_TRY(check_opts(o));
    PN_TRY(check_ptrs({x, s0, s, gs, cell->params}, hb));
    if (!gparams) { set_error("gparams is NULL"); return PN_ERR_INVALID_ARG; }
    if ((gx && !aligned16(gx)) || (gs0 && !aligned16(gs0)) || !aligned16(gparams)) {
        set_error("gradient arrays must be 16-byte aligned");
        return PN_ERR_INVALID_ARG;
    }
    const Route r = route_adjoint(*cell, o);
    if (r == Route::None) {
        set_error("deer_adjoint not built for cell=%d D=%d Dx=%d dtype=%d jac=%d damping=%d",
                  cell->cell, cell->D, cell->Dx, cell->dtype, o.jac, o.damping);
        return PN_ERR_UNSUPPORTED;
    }
    if (o.smooth) {
        set_error("the smoother is built for elk_solve only");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.freeze_prefix && r != Route::GruQuasi) {
        set_error("deer_adjoint skips converged prefixes on the GRU diagonal path only");
        return PN_ERR_UNSUPPORTED;
    }
    if (o.stop != PN_STOP_RESID_INF) {
        set_error("deer_adjoint stops on its residual (PN_STOP_RESID_INF)");
        return PN_ERR_UNSUPPORTED;
    }
    size_t need = 0;
    PN_TRY(pn_workspace_bytes(PN_OP_ADJOINT, cell, batch, &o, &need));
    PN_TRY(check_ws(workspace, workspace_bytes, need));
    if (o.check_inputs)
        PN_TRY(check_finite({{x, hb.N * cell->Dx}, {s0, (int64_t)hb.B * cell->D},
                             {s, hb.N * cell->D}, {gs, hb.N * cell->D},
                             {cell->params, param_count(*cell, hb.N)}},
                            cell->dtype, (int*)((char*)workspace + need - kCheckBytes),
                            (hipStream_t)stream));
    bool conv = true;
    if (r == Route::GruQuasi || r == Route::GruDenseAdj)
        PN_TRY(gru_adjoint(*cell, hb, (const float*)x, (const float*)s0, (const float*)s,
                           (const float*)gs, (float*)gx, (float*)gs0, (float*)gparams, o,
                           workspace, (hipStream_t)stream, info, &conv));
    else
        PN_TRY(tanh_adjoint(*cell, hb, (const float*)x, (const float*)s0, (const float*)s,
                            (const float*)gs, (float*)gx, (float*)gs0, (float*)gparams, o,
                            workspace, (hipStream_t)stream, info, &conv));
    return conv ? PN_OK : PN_NOT_CONVERGED;
}

pn_status seq_rollout(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                      const void* s0, void* s, void* workspace, size_t workspace_bytes,
                      void* stream) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    PN_TRY(check_ptrs({x, s0, s, cell->params}, hb));
    if (cell->dtype != PN_F32 || !seq_supported(cell->cell, cell->D, cell->Dx)) {
        set_error("seq_rollout not built for cell=%d D=%d Dx=%d dtype=%d", cell->cell, cell->D,
                  cell->Dx, cell->dtype);
        return PN_ERR_UNSUPPORTED;
    }
    PN_TRY(check_ws(workspace, workspace_bytes, seq_workspace(cell->cell, cell->D, cell->Dx, hb)));
    return seq_rollout_run(*cell, hb, (const float*)x, (const float*)s0, (float*)s, workspace,
                           (hipStream_t)stream);
}

pn_status seq_bptt(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                   const void* s0, const void* s, const void* gs, void* gx, void* gs0,
                   void* gparams, void* workspace, size_t workspace_bytes, void* stream) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    PN_TRY(check_ptrs({x, s0, s, gs, cell->params}, hb));
    if (!gparams) { set_error("gparams is NULL"); return PN_ERR_INVALID_ARG; }
    if ((gx && !aligned16(gx)) || (gs0 && !aligned16(gs0)) || !aligned16(gparams)) {
        set_error("gradient arrays must be 16-byte aligned");
        return PN_ERR_INVALID_ARG;
    }
    const bool gru = cell->cell == PN_CELL_GRU && seq_supported(cell->cell, cell->D, cell->Dx);
    const bool tanh = cell->cell == PN_CELL_TANH && tanh_dense_supported(cell->D, cell->Dx);
    if (cell->dtype != PN_F32 || !(gru || tanh)) {
        set_error("seq_bptt not built for cell=%d D=%d Dx=%d dtype=%d", cell->cell, cell->D,
                  cell->Dx, cell->dtype);
        return PN_ERR_UNSUPPORTED;
    }
    PN_TRY(check_ws(workspace, workspace_bytes, seq_workspace(cell->cell, cell->D, cell->Dx, hb)));
    if (tanh)
        return tanh_seq_bptt(*cell, hb, (const float*)x, (const float*)s0, (const float*)s,
                             (const float*)gs, (float*)gx, (float*)gs0, (float*)gparams,
                             workspace, (hipStream_t)stream);
    return seq_bptt_run(*cell, hb, (const float*)x, (const float*)s0, (const float*)s,
                        (const float*)gs, (float*)gx, (float*)gs0, (float*)gparams, workspace,
                        (hipStream_t)stream);
}

pn_status pn_residual_f64(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                          const void* s0, const void* s, void* workspace,
                          size_t workspace_bytes, void* stream, double* max_resid) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    PN_TRY(check_ptrs({x, s0, s, cell->params}, hb));
    if (!max_resid) { set_error("max_resid is NULL"); return PN_ERR_INVALID_ARG; }
    if (cell->dtype != PN_F32 || !residual64_supported(cell->cell, cell->D, cell->Dx)) {
        set_error("pn_residual_f64 not built for cell=%d D=%d Dx=%d", cell->cell, cell->D, cell->Dx);
        return PN_ERR_UNSUPPORTED;
    }
    const size_t need = residual64_workspace(cell->cell, cell->D, cell->Dx, hb);
    PN_TRY(check_ws(workspace, workspace_bytes, need));
    return residual64_run(*cell, hb, (const float*)x, (const float*)s0, (const float*)s,
                          workspace, (hipStream_t)stream, max_resid);
}

pn_status pn_lle_estimate(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                          const void* s0, const void* s, const void* u0, void* workspace,
                          size_t workspace_bytes, void* stream, double* lle) {
    PN_TRY(check_cell(cell));
    HostBatch hb;
    PN_TRY(check_batch(batch, hb));
    PN_TRY(check_ptrs({x, s0, s, u0, cell->params}, hb));
    if (!lle) { set_error("lle is NULL"); return PN_ERR_INVALID_ARG; }
    if (cell->dtype != PN_F32 || !lle_supported(cell->cell, cell->D, cell->Dx)) {
        set_error("pn_lle_estimate not built for cell=%d D=%d Dx=%d", cell->cell, cell->D,
                  cell->Dx);
        return PN_ERR_UNSUPPORTED;
    }
    PN_TRY(check_ws(workspace, workspace_bytes, lle_workspace(hb)));
    return lle_run(*cell, hb, (const float*)x, (const float*)s0, (const float*)s,
                   (const float*)u0, workspace, (hipStream_t)stream, lle);
}

}  // extern "C"
