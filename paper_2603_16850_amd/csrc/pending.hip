// Entry points whose solvers are not built yet report PN_ERR_UNSUPPORTED.
#include "pn_solvers.hpp"

namespace pn {

bool gru_dense64_supported(int, int) { return false; }
size_t gru_dense64_workspace(int, int, const HostBatch&, const pn_opts&) { return 0; }
pn_status gru_dense64_forward(const pn_cell_desc&, const HostBatch&, const double*, const double*,
                              double*, const pn_opts&, void*, hipStream_t, pn_seq_info*, bool*) {
    return PN_ERR_UNSUPPORTED;
}
bool tanh_dense_supported(int, int) { return false; }
size_t tanh_dense_workspace(int, int, const HostBatch&, const pn_opts&) { return 0; }
pn_status tanh_dense_forward(const pn_cell_desc&, const HostBatch&, const float*, const float*,
                             float*, const pn_opts&, void*, hipStream_t, pn_seq_info*, bool*) {
    return PN_ERR_UNSUPPORTED;
}
bool elk_supported(int, int) { return false; }
size_t elk_workspace(int, int, const HostBatch&, const pn_opts&) { return 0; }
pn_status elk_forward(const pn_cell_desc&, const HostBatch&, const float*, const float*, float*,
                      double, const pn_opts&, void*, hipStream_t, pn_seq_info*, bool*) {
    return PN_ERR_UNSUPPORTED;
}
bool residual64_supported(int, int, int) { return false; }
size_t residual64_workspace(int, int, int, const HostBatch&) { return 0; }
pn_status residual64_run(const pn_cell_desc&, const HostBatch&, const float*, const float*,
                         const float*, void*, hipStream_t, double*) { return PN_ERR_UNSUPPORTED; }

}  // namespace pn
