// Solver drivers behind the C ABI (one translation unit each).
#pragma once
#include <initializer_list>
#include <utility>

#include "pn_host.hpp"

namespace pn {

const char* last_error();
void profile_begin();
void profile_end();
int profile_read(const char* family, double* ms, int64_t* n);

// quasi-DEER (and Picard / Jacobi), GRU, FP32: per-group linearise + scan, carry, apply
bool gru_quasi_supported(int D, int Dx);
int gru_quasi_tile(int D, int Dx, const pn_opts& o);
// tiles per group for a launch of `resident` workgroups over `ntiles` tiles
int gru_group_tiles(int ntiles, int resident);
// workgroups of `kern` (nt threads) resident on the device at once
int gru_resident(const void* kern, int nt);
size_t gru_quasi_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status gru_quasi_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                            const float* s0, float* s, const pn_opts& o, void* ws,
                            hipStream_t stream, pn_seq_info* info, bool* all_conv);

// exact adjoint of the GRU by iterated reverse diagonal scans + parameter gradients
size_t gru_adjoint_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status gru_adjoint(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                      const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                      float* gparams, const pn_opts& o, void* ws, hipStream_t stream,
                      pn_seq_info* info, bool* all_conv);

// the same adjoint as one reverse dense scan (GRU, D in {16, 32, 48, 64}): chains of FP32
// VJPs inside groups of consecutive steps, per-group maps composed on MFMA (BF16 or FP32),
// carries refined by the exact residual.  Needs the gate rows from the adjoint's prep pass
// and its group table (groups of the tiles from each sequence's end); fills seq[] and lam.
size_t gru_adj_dense_bytes(int D, int ngroups, int B);
pn_status gru_adj_dense_solve(int D, const float* gates, const float* gs, const float* U,
                              float* lam, const IterState& st, int ngroups, int B,
                              const float* gmax, float tol, bool bf16, int max_passes,
                              void* dense_ws, hipStream_t stream);

// DEER, GRU, FP64, small dense D (whole solve in one workgroup per sequence)
bool gru_dense64_supported(int D, int Dx);
size_t gru_dense64_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status gru_dense64_forward(const pn_cell_desc& cd, const HostBatch& hb, const double* x,
                              const double* s0, double* s, const pn_opts& o, void* ws,
                              hipStream_t stream, pn_seq_info* info, bool* all_conv);

// DEER, tanh-RNN, FP32 residual, dense scan composed on MFMA (BF16 or FP32)
bool tanh_dense_supported(int D, int Dx);
size_t tanh_dense_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status tanh_dense_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                             const float* s0, float* s, const pn_opts& o, void* ws,
                             hipStream_t stream, pn_seq_info* info, bool* all_conv);

// exact adjoint of the dense tanh-RNN: reverse dense scans (FP32 or BF16 maps, exact FP32
// residual) + parameter gradients
size_t tanh_adjoint_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status tanh_adjoint(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                       const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                       float* gparams, const pn_opts& o, void* ws, hipStream_t stream,
                       pn_seq_info* info, bool* all_conv);
pn_status tanh_seq_bptt(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                        const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                        float* gparams, void* ws, hipStream_t stream);

// DEER for the mean-field cell at 16 < D <= 128 (two-level dense scan, FP32 residual, BF16 or
// FP32 compose), its sequential rollout and LLE estimate
bool mf_dense_supported(int D, int Dx);
size_t mf_dense_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status mf_dense_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                           const float* s0, float* s, const pn_opts& o, void* ws,
                           hipStream_t stream, pn_seq_info* info, bool* all_conv);
size_t mf_seq_workspace(int D, const HostBatch& hb);
pn_status mf_seq_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                     const float* s0, float* s, void* ws, hipStream_t stream);
pn_status mf_lle_run(const pn_cell_desc& cd, const HostBatch& hb, const float* s0,
                     const float* s, const float* u0, void* ws, hipStream_t stream, double* lle);

// ELK, tanh-RNN, FP32
bool elk_supported(int D, int Dx);
size_t elk_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status elk_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                      const float* s0, float* s, double lambda, const pn_opts& o, void* ws,
                      hipStream_t stream, pn_seq_info* info, bool* all_conv);

// DEER / quasi-DEER / Picard / Jacobi on the affine test cells (D <= 16, FP32)
bool affine_supported(int D, int Dx);
size_t affine_workspace(int D, int Dx, const HostBatch& hb, const pn_opts& o);
pn_status affine_forward(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                         const float* s0, float* s, const pn_opts& o, void* ws,
                         hipStream_t stream, pn_seq_info* info, bool* all_conv);

// opts->check_inputs: scans the arrays for NaN / infinity (flag: 4 bytes of device memory)
pn_status check_finite(std::initializer_list<std::pair<const void*, int64_t>> arrays, int dtype,
                       int* flag_dev, hipStream_t stream);

// sequential baselines
bool seq_supported(int cell, int D, int Dx);
size_t seq_workspace(int cell, int D, int Dx, const HostBatch& hb);
pn_status seq_rollout_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                          const float* s0, float* s, void* ws, hipStream_t stream);
pn_status seq_bptt_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                       const float* s0, const float* s, const float* gs, float* gx, float* gs0,
                       float* gparams, void* ws, hipStream_t stream);

// largest Lyapunov exponent along a trajectory
bool lle_supported(int cell, int D, int Dx);
size_t lle_workspace(const HostBatch& hb);
pn_status lle_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x, const float* s0,
                  const float* s, const float* u0, void* ws, hipStream_t stream, double* lle);

// FP64 residual of an FP32 trajectory
bool residual64_supported(int cell, int D, int Dx);
size_t residual64_workspace(int cell, int D, int Dx, const HostBatch& hb);
pn_status residual64_run(const pn_cell_desc& cd, const HostBatch& hb, const float* x,
                         const float* s0, const float* s, void* ws, hipStream_t stream,
                         double* max_resid);

}  // namespace pn
