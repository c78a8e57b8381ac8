// deer_solve_noalloc: deer_solve for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation).  Its scratch
// space is a file-scope device array of fixed size instead of a caller workspace; the kernels
// are those of deer_solve.  The array's device address is looked up once per device with
// hipGetSymbolAddress (the array's name in host code is a host-side stand-in, not a device
// address) and only that address is passed on.  Every call on a device shares that device's
// array, so calls that overlap on one device race; each call initialises all the scratch it
// reads (tables, solver state, iterates) before reading it.
#include <mutex>

#include "pn_host.hpp"
#include "pn_solvers.hpp"

namespace {

static __device__ __align__(256) char scratch[PN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on its first use there).
pn_status scratch_ptr(void** out) {
    int dev = 0;
    PN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        pn::set_error("deer_solve_noalloc: device %d beyond the %d devices it keeps scratch for",
                      dev, kMaxDevices);
        return PN_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return pn::hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e,
                                "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return PN_OK;
}

struct NoallocScope {
    NoallocScope() { pn::set_noalloc(true); }
    ~NoallocScope() { pn::set_noalloc(false); }
};

}  // namespace

extern "C" pn_status deer_solve_noalloc(const pn_cell_desc* cell, const pn_batch* batch,
                                        const void* x, const void* s0, void* s,
                                        const pn_opts* opts, void* stream, pn_seq_info* info) {
    size_t need = 0;
    PN_TRY(pn_workspace_bytes(PN_OP_DEER, cell, batch, opts, &need));
    if (need > (size_t)PN_NOALLOC_SCRATCH_BYTES) {
        pn::set_error("deer_solve_noalloc: these shapes need %zu bytes of scratch; the static "
                      "scratch holds %zu (use deer_solve with a workspace)",
                      need, (size_t)PN_NOALLOC_SCRATCH_BYTES);
        return PN_ERR_WORKSPACE;
    }
    void* ws = nullptr;
    PN_TRY(scratch_ptr(&ws));
    NoallocScope scope;
    return deer_solve(cell, batch, x, s0, s, opts, ws, (size_t)PN_NOALLOC_SCRATCH_BYTES, stream,
                      info);
}
