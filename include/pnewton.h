/*
 * pnewton.h -- C ABI of the MI355X (gfx950) parallel Newton library.
 *
 * The library evaluates a nonlinear recurrence s_t = f(s_{t-1}, x_t), t = 1..T, for many
 * sequences at once by Newton iterations over the whole trajectory (DEER), by the diagonal
 * quasi-Newton variant (quasi-DEER), or by the Levenberg-Marquardt / Kalman-filter variant
 * (ELK), and differentiates the result by the reverse-time adjoint recurrence.
 *
 * What each call computes (thesis sections; "eq." names are the thesis's equation labels):
 *   - residual r_t = s_t - f_t(s_{t-1})                       (Ch. 2, eq. r_def)
 *   - Newton step: Delta_1 = -r_1, Delta_t = A~_t Delta_{t-1} - r_t, s <- s + Delta,
 *     with A~_t = df/ds_{t-1} (DEER, eq. lin_rr) or its diagonal (quasi-DEER, eq. quasi_lds),
 *     evaluated for all t by an associative scan of affine maps (eq. bin_op_affine)
 *   - loop and stopping rule                                  (Alg. alg:deer)
 *   - ELK step: the filtered means of the linear-Gaussian SSM of Prop. prop:ELK
 *   - adjoint lambda_t = g_t + A_{t+1}^T lambda_{t+1} and the parameter gradient
 *     sum_t (df_t/dtheta)^T lambda_t                         (Ch. 3, eqs. bptt..unrolled_bwds)
 *
 * Conventions shared by every entry point
 *   - All array arguments except `offsets`, `info` and the host result arrays are DEVICE
 *     pointers, contiguous, row-major, in the dtype named by pn_cell_desc.dtype.  The caller
 *     owns every buffer; the library never allocates device memory on these paths: scratch
 *     space comes from the caller's workspace (size from pn_workspace_bytes).
 *   - Sequences lie back to back: sequence b owns rows offsets[b] .. offsets[b+1]-1 of
 *     x [N, Dx] and s [N, D]; s0 is [B, D].  `offsets` is a HOST array of B+1 int64 values
 *     (offsets[0] = 0, non-decreasing, offsets[B] = N), or NULL for B sequences of N/B steps.
 *   - Work is enqueued on `stream` (a hipStream_t, may be NULL for the default stream).
 *     Solvers synchronise that stream to read their per-sequence convergence state once
 *     every opts->graph_iters iterations; they return only after all their work finished.
 *   - Arguments are validated before any HIP call.  A negative status means nothing was
 *     written to the outputs.  PN_NOT_CONVERGED (> 0) means the outputs hold the last
 *     iterate.  pn_last_error() gives a message for the last failing call on the thread.
 *   - Calls are reentrant given distinct workspaces; calls sharing a workspace must be
 *     ordered on one stream.
 */
#ifndef PNEWTON_H
#define PNEWTON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PN_ABI_VERSION 1

typedef enum {
    PN_OK = 0,
    PN_NOT_CONVERGED = 1,        /* outputs valid: the last iterate / last adjoint iterate */
    PN_ERR_INVALID_ARG = -1,
    PN_ERR_UNSUPPORTED = -2,     /* valid arguments, combination not built into the library */
    PN_ERR_WORKSPACE = -3,       /* workspace NULL or smaller than pn_workspace_bytes */
    PN_ERR_NONFINITE_INPUT = -4, /* opts->check_inputs found a NaN or infinity in an input */
    PN_ERR_HIP = -5,             /* a HIP runtime call failed */
    PN_ERR_INTERNAL = -6         /* a host-side consistency check of the library failed (a bug) */
} pn_status;

typedef enum {
    PN_CELL_GRU = 0,    /* reset-after GRU (the thesis's GRU experiments cite the GRU paper):
                           z = sig(W_z x + U_z h + b_z), r = sig(W_r x + U_r h + b_r),
                           n = tanh(W_n x + b_n + r*(U_n h + b_hn)), f = (1-z)*n + z*h.
                           params: [W_z;W_r;W_n] (3D x Dx) | [U_z;U_r;U_n] (3D x D) |
                                   [b_z;b_r;b_n] (3D) | b_hn (D)                          */
    PN_CELL_TANH = 1,   /* f = tanh(W h + U x + b).
                           params: W (D x D) | U (D x Dx) | b (D)                         */
    PN_CELL_MEANFIELD = 2, /* f = W tanh(h) + U x + b: the mean-field RNN of the
                           predictability experiments (Ch. 5), whose state is a current;
                           A = W diag(1 - tanh(h)^2).  params as PN_CELL_TANH           */
    PN_CELL_AFFINE = 3, /* test cell, a linear dynamical system (Ch. 2, eq. lds):
                           f = M h + N x + c, so A = M and one DEER update is exact (the
                           residual's Jacobian is constant).  params: M (D x D) | N (D x Dx) |
                           c (D)                                                           */
    PN_CELL_AFFINE_STEPS = 4 /* test cell with a transition matrix per step:
                           f_t = M_t h + N x_t + c (the input-dependent LDS of the group word
                           problem, Ch. 6, Prop. cayley: permutation matrices M_t).  params:
                           M_t of every row in batch order ([N, D, D], M_t of row offsets[b] +
                           t - 1 for step t of sequence b) | N (D x Dx) | c (D)             */
} pn_cell;

typedef enum {
    PN_JAC_DENSE = 0,   /* A~_t = A_t (DEER)                                             */
    PN_JAC_DIAG = 1,    /* A~_t = diag(A_t), closed form (quasi-DEER)                     */
    PN_JAC_PICARD = 2,  /* A~_t = I: Picard iteration as quasi-DEER (Prop. picard)         */
    PN_JAC_JACOBI = 3   /* A~_t = 0: Jacobi iteration, s_t <- f(s_{t-1}) for all t at once
                           (Table fxd_pt_sum).  One Jacobi iteration from s = 0 is the
                           initialisation s_t^(0) = f(0, x_t) discussed in Ch. 3          */
} pn_jac;

typedef enum {
    PN_DAMP_NONE = 0,
    PN_DAMP_SCALE = 1,  /* scale-ELK (Sec. "Further extensions: scale- and clip-ELK"):
                           A~_t <- (1 - k) A~_t with k = damp_k in [0, 1]; k = 0 is the
                           undamped method, k = 1 makes every iteration a Jacobi step       */
    PN_DAMP_CLIP = 2    /* clip-ELK (same section): every entry of a diagonal A~_t clipped to
                           [clip_lo, clip_hi], -1 <= clip_lo <= clip_hi <= 1 (the thesis's
                           default is [-1, 1]); diagonal transitions only                   */
} pn_damping;

typedef enum { PN_F32 = 0, PN_F64 = 1 } pn_dtype;

typedef enum {
    PN_STOP_RESID_INF = 0,  /* stop a sequence when max_t,d |r_t| < tol at the current iterate
                               (ComputeError of Alg. alg:deer as the residual)             */
    PN_STOP_DELTA_INF = 1   /* stop when the last update max_t,d |s^(i) - s^(i-1)| < tol (the
                               update norm of the Ch. 3 GRU experiments); no sequence stops
                               before its first update, and max_iters <= 0 means T + 1
                               updates (Alg. alg:deer's loop bound i = 0..T: the zero update
                               after the exact trajectory is what this rule sees)         */
} pn_stop;

typedef enum {
    PN_COMPOSE_NATIVE = 0,  /* dense scan products in the solve dtype                      */
    PN_COMPOSE_BF16 = 1     /* dense scan products on BF16 MFMA with FP32 accumulation;
                               residuals stay FP32 so the iteration refines itself          */
} pn_compose;

typedef struct {
    int32_t cell;           /* pn_cell */
    int32_t D;              /* state size */
    int32_t Dx;             /* input size */
    int32_t dtype;          /* pn_dtype of x, s0, s, params and all gradients */
    const void* params;     /* device, packed as documented in pn_cell */
} pn_cell_desc;

typedef struct {
    int32_t B;              /* number of sequences (>= 1) */
    int32_t pad_;
    int64_t N;              /* total steps, = offsets[B] */
    const int64_t* offsets; /* HOST [B+1], or NULL for uniform length N/B */
} pn_batch;

typedef struct {
    int32_t jac;              /* pn_jac */
    int32_t compose;          /* pn_compose */
    double tol;               /* stop a sequence when max_t,d |r| < tol (forward), or when the
                                 adjoint residual max |rho| <= tol * max(1, max |g|)        */
    int32_t max_iters;        /* <= 0: the longest sequence length (Prop. global_convergence) */
    int32_t graph_iters;      /* iterations per captured HIP graph between host checks (>= 1) */
    double reset_abs;         /* reset a time-step vector of the iterate to 0 when any entry is
                                 non-finite or exceeds this magnitude (<= 0: 1e4)             */
    int32_t fp64_final_residual; /* ELK / F32: also report the FP64 residual of the result   */
    int32_t use_graph;        /* 1: capture graph_iters iterations in a hipGraph; 0: launch */
    int32_t tile;             /* scan tile length in steps; 0: autotuned / default          */
    int32_t damping;          /* pn_damping (deer_solve only; ELK damps through lambda)     */
    float damp_k;             /* PN_DAMP_SCALE: k                                            */
    float clip_lo;            /* PN_DAMP_CLIP: bounds                                        */
    float clip_hi;
    int32_t freeze_prefix;    /* elk_solve: 1 = stop updating each sequence's converged prefix
                                 (whole groups of `tile` steps whose residual is below tol,
                                 counted from the start; the filter restarts after them) */
    int32_t smooth;           /* elk_solve: 1 = take the smoothed means (the exact LM step of
                                 Prop. ELK, Kalman filter plus RTS backward pass); 0 = the
                                 filtered means                                            */
    int32_t group;            /* chunks of `tile` steps per group of the two-pass scans (the
                                 local pass works a group at a time, the carry pass walks the
                                 groups): 1..64, or 0 = chosen by the library's cost model.
                                 Used by deer_solve (GRU diagonal, tanh dense) and
                                 deer_adjoint; elk_solve takes its group length as `tile`
                                 and requires 0 here.  pn_autotune measures it.            */
    int32_t stop;             /* pn_stop (forward solves).  PN_STOP_DELTA_INF is built for
                                 deer_solve on the GRU diagonal path and the affine cells;
                                 other routes return PN_ERR_UNSUPPORTED for it             */
    int32_t check_inputs;     /* 1: before solving, scan x, s0 and params (deer_adjoint also s
                                 and gs) for NaN / infinity and return PN_ERR_NONFINITE_INPUT
                                 if any is found (one extra pass over the inputs and a stream
                                 synchronisation; the workspace grows by 256 bytes)        */
} pn_opts;

typedef struct {
    int32_t iters;          /* Newton (or adjoint) updates applied to the returned iterate */
    int32_t converged;      /* 1 if the stopping test passed */
    int32_t resets;         /* time-step vectors reset by the overflow guard (kept iterates) */
    int32_t pad_;
    double max_resid;       /* residual max-norm of the returned iterate (FP64 when requested) */
} pn_seq_info;

/* Operation codes for pn_workspace_bytes. */
#define PN_OP_DEER 0
#define PN_OP_ELK 1
#define PN_OP_ADJOINT 2
#define PN_OP_RESIDUAL64 3

/* Fill *opts with defaults: quasi (diag), native compose, tol 1e-5, max_iters = T,
   graph_iters 4, reset_abs 1e4, graph capture on, tile 0, no damping (k = 0, clip [-1, 1]),
   residual stopping rule, no input scan. */
void pn_default_opts(pn_opts* opts);

/* Bytes of device workspace `op` needs for these shapes (0 is possible).  *bytes is set on
   PN_OK.  The workspace must be 256-byte aligned. */
pn_status pn_workspace_bytes(int op, const pn_cell_desc* cell, const pn_batch* batch,
                             const pn_opts* opts, size_t* bytes);

/* DEER / quasi-DEER (Alg. alg:deer with eq. lin_rr or eq. quasi_lds).
   s [N, D] is read as the initial guess s^(0) and overwritten with the result.
   info: HOST array [B] (may be NULL).  Built combinations:
     GRU,  PN_JAC_DIAG / PN_JAC_PICARD / PN_JAC_JACOBI, F32, (D, Dx) in
           {(16,8), (16,16), (32,8), (32,16), (32,32), (48,24), (48,48), (64,16), (64,32),
            (64,64)}, tile 0 (default), 32, 64 or 128 (not 128 at (64,64)), any damping
     GRU,  PN_JAC_DENSE, F64, 1 <= D <= 4, 1 <= Dx <= 16, no damping
     TANH, PN_JAC_DENSE, F32, D = 32, Dx in {16, 32}, compose native or BF16, no damping or
           PN_DAMP_SCALE
     MEANFIELD, PN_JAC_DENSE, F32, 16 < D <= 128, 1 <= Dx <= 1024, compose native or BF16,
           no damping (a two-level dense scan: per-group maps on MFMA, FP32 residual and
           chains, the reset guard; opts->group = tiles of 32 steps per group, 0 = cost model)
     AFFINE, AFFINE_STEPS, any jac, F32, 1 <= D <= 16, 1 <= Dx <= 64, no damping (the test
           cells: the dense transition is M or M_t itself)
   (MEANFIELD at D = 16 runs DEER through elk_solve with lambda = 0.)
   Anything else returns PN_ERR_UNSUPPORTED. */
pn_status deer_solve(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                     const void* s0, void* s, const pn_opts* opts, void* workspace,
                     size_t workspace_bytes, void* stream, pn_seq_info* info);

/* deer_solve without a workspace, for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same arguments,
   kernels and results as deer_solve; the scratch space is a static device array of
   PN_NOALLOC_SCRATCH_BYTES per device, held until the process ends.  Shapes whose
   pn_workspace_bytes(PN_OP_DEER, ...) exceeds it return PN_ERR_WORKSPACE.  The call allocates
   nothing (no hipMalloc, no pinned host memory, no graph instantiation): iterations are
   launched directly whatever opts->use_graph says, host readbacks go through pageable memory,
   pn_profile_* timing is off.  Calls that overlap on one device share its scratch and race:
   order them (one stream, or one host thread at a time per device). */
#define PN_NOALLOC_SCRATCH_BYTES (64u << 20)
pn_status deer_solve_noalloc(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                             const void* s0, void* s, const pn_opts* opts, void* stream,
                             pn_seq_info* info);

/* ELK (Ch. 4): each iteration replaces the Newton step by the filtered means of the LGSSM
   of Prop. prop:ELK with emission noise 1/lambda (lambda >= 0; lambda = 0 is DEER).  With
   PN_JAC_DIAG the LGSSM uses diag(A_t): quasi-ELK (Ch. 4, "quasi-ELK").
   Built: TANH or MEANFIELD, PN_JAC_DENSE or PN_JAC_DIAG, F32, D = 16, Dx = 16, no damping;
   (lambda = 0 with PN_JAC_DENSE is DEER on these cells); tile 0
   (chosen from the shapes) or a multiple of 16 up to 1024: the steps one workgroup folds
   into one filter element.  With fp64_final_residual the stopping test of every iterate is evaluated in FP64 and the
   reported max_resid is the FP64 residual of the returned FP32 iterate. */
pn_status elk_solve(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                    const void* s0, void* s, double lambda, const pn_opts* opts,
                    void* workspace, size_t workspace_bytes, void* stream, pn_seq_info* info);

/* Adjoint of the solution s (Ch. 3, "Training and the backwards pass"): given
   gs = dL/ds [N, D] (partial derivative of the loss at each state), computes the total
   derivatives lambda_t = dL/ds_t of the recurrence, then
     gparams (packed like params, overwritten) = sum_t (df_t/dtheta)^T lambda_t,
     gx [N, Dx] = (df_t/dx_t)^T lambda_t   (may be NULL),
     gs0 [B, D] = A_1^T lambda_1           (may be NULL).
   With PN_JAC_DIAG the reverse recurrence is solved by iterated reverse scans with
   diag(A_t) and an exact VJP residual (converges to the exact adjoint); with PN_JAC_DENSE
   by reverse scans with the dense transposed Jacobians (the DEER backward pass of Ch. 3):
   for the tanh-RNN A_t^T = W^T diag(d_t) rebuilt on chip, composed in FP32
   (PN_COMPOSE_NATIVE: one update reaches the adjoint) or BF16 (PN_COMPOSE_BF16: the exact
   FP32 residual drives further updates); for the GRU a two-level scan over groups of
   consecutive steps (opts->group tiles of 32 steps each, 0 = about N / 2^20 tiles): the
   exact recurrence inside every group in FP32, the groups' maps (products of A_t^T)
   composed in BF16 or FP32 on MFMA, the carries between groups refined while the residual
   at the group boundaries fails the test (each refinement one more update; max_iters <= 0
   means 8).  Stopping rule of all: max |rho_t| <= tol * max(1, max |g_t|) per sequence,
   rho_t = lambda_t - g_t - A_{t+1}^T lambda_{t+1}; info reports the adjoint updates.
   Built: GRU, F32, PN_JAC_DIAG (same shapes as deer_solve) and PN_JAC_DENSE (D in
   {16, 32, 48, 64}, no damping, no prefix skipping); TANH, PN_JAC_DENSE, F32, D = 32,
   Dx in {16, 32}, no damping. */
pn_status deer_adjoint(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                       const void* s0, const void* s, const void* gs, void* gx, void* gs0,
                       void* gparams, const pn_opts* opts, void* workspace,
                       size_t workspace_bytes, void* stream, pn_seq_info* info);

/* Sequential baselines on the GPU (one workgroup per sequence walks the steps in order, the
   input projections W x_t + b of all steps computed beforehand in parallel, as cuDNN-style
   RNN layers do): the rollout s_t = f(s_{t-1}, x_t) (Ch. 2, eq. ssm), and backpropagation
   through that rollout -- the reverse recurrence lambda_t = g_t + A_{t+1}^T lambda_{t+1} one
   step at a time, then the parallel gradient reductions -- with the outputs of deer_adjoint.
   Workspace from pn_workspace_bytes(PN_OP_SEQ, ...).  Built: GRU F32 (the deer_solve GRU
   shapes), TANH F32 ((D, Dx) in {(16,16), (32,16), (32,32), (64,32), (16,8), (4,4)}),
   MEANFIELD F32 (D = Dx = 16, and 16 < D <= 128 with 1 <= Dx <= 1024). seq_bptt: GRU, and
   TANH F32 with D = 32, Dx in {16, 32}. */
#define PN_OP_SEQ 4
pn_status seq_rollout(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                      const void* s0, void* s, void* workspace, size_t workspace_bytes,
                      void* stream);
pn_status seq_bptt(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                   const void* s0, const void* s, const void* gs, void* gx, void* gs0,
                   void* gparams, void* workspace, size_t workspace_bytes, void* stream);

/* FP64 residual max-norm per sequence of an FP32 trajectory (inputs upcast to FP64):
   max_resid: HOST array [B].  Built: TANH, MEANFIELD and GRU, F32. */
pn_status pn_residual_f64(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                          const void* s0, const void* s, void* workspace,
                          size_t workspace_bytes, void* stream, double* max_resid);

/* Largest Lyapunov exponent along a trajectory (Alg. LLE_estimate, Ch. 5): per sequence,
   u_t = A_t u_{t-1} with A_t = df/ds_{t-1} at the trajectory's previous state (s_0 first),
   lambda_t = ||u_t||, u_t <- u_t / lambda_t, lle = (1/T) sum_t log lambda_t.
   s [N, D]: the trajectory (device); u0 [B, D]: starting vectors (device, normalised here,
   nonzero); lle: HOST array [B] (0 for an empty sequence).  Log stretches are summed in FP64.
   Workspace from pn_workspace_bytes(PN_OP_LLE, ...).  Built: TANH and MEANFIELD, F32,
   D = Dx = 16; MEANFIELD, F32, 16 < D <= 128.  A zero stretch (u mapped to 0) gives -inf for
   that sequence. */
#define PN_OP_LLE 5
pn_status pn_lle_estimate(const pn_cell_desc* cell, const pn_batch* batch, const void* x,
                          const void* s0, const void* s, const void* u0, void* workspace,
                          size_t workspace_bytes, void* stream, double* lle);

/* Kernel timing with HIP events, for benchmarking.  Between pn_profile_begin() and
   pn_profile_end() the solvers called on this thread launch their iterations directly (no
   graph) and record a HIP event pair around every launch of their main kernels on the caller's
   stream; pn_profile_read() returns the summed duration and launch count of a kernel family
   (launches of iterations after the one that stopped the last sequence return at once; they
   are counted under the family name followed by "#idle"):
     deer_solve GRU diagonal: "gru_quasi_local", "carry_scan";
     deer_adjoint GRU: "gru_adj_prep", "gru_adj_grad", and with PN_JAC_DIAG
       "gru_adj_local", "carry_scan", with PN_JAC_DENSE "gru_adj_dmap", "gru_adj_dwalk",
       "gru_adj_dchain", "gru_adj_dcheck";
     deer_solve tanh dense: "tanh_dense_local", "dense_carry";
     deer_adjoint tanh dense: "tanh_adj_prep", "tanh_adj_local", "dense_carry", "tanh_adj_grad";
     deer_solve GRU FP64: "gru_dense64_solve";
     elk_solve: "elk_local", "elk_carry", and with the smoother "elk_smooth",
       "elk_back_carry", "elk_back_apply";
     deer_solve affine cells: "affine_local", "affine_carry";
     seq_rollout: "seq_rollout"; seq_bptt: "seq_adj".
   Returns 0 if the family was not launched since pn_profile_begin(). */
/* Scan-tile autotuner (batching, "scan tile sizes chosen by a project-written autotuner").
   pn_autotune times op (PN_OP_DEER, PN_OP_ELK or PN_OP_ADJOINT) on the caller's own inputs
   once per candidate (tile, group) -- a warm-up call, then a timed call of probe_iters
   iterations with tol ~ 0 so that every candidate runs them all, HIP events on `stream`
   around the whole call (host checks included) -- and returns the fastest in *out.
   Candidates: deer_solve GRU diagonal: tile in {32, 64, 128} x group in {0, 1, 2, 4, 8, 16};
   deer_solve tanh dense and deer_adjoint: group in {0, 1, 2, 4, 8, 16}; elk_solve: tile in
   {0, 16, 32, 64, 128, 256}; other routes: the single candidate (0, 0).
   Results are kept per process under a key of the route's shapes and options (cell, D, Dx,
   dtype, jac, compose, damping, lambda > 0, smooth, freeze_prefix, graph options, B and
   the bit lengths of N and of the longest sequence); a known key returns at once with
   out->from_cache = 1 and runs nothing.  When the environment variable PN_AUTOTUNE_CACHE
   names a file, a key missing in the process is looked up in that file (JSON object of
   "key": [tile, group] entries) and every newly measured key is written back to it.
   bufs: the op's device buffers in the order of its solve call --
     PN_OP_DEER, PN_OP_ELK: {x, s0, s}; s is restored before return (the workspace keeps a
       copy), so it may hold the caller's initial guess;
     PN_OP_ADJOINT: {x, s0, s, gs, gx, gs0, gparams}; gx, gs0 may be NULL; the outputs
       gx, gs0, gparams hold unspecified values afterwards.
   lambda: elk_solve's lambda (ignored otherwise).  probe_iters: 1..64 (<= 0: 3); each
   candidate runs once to warm up and twice timed (the faster counts), probe_iters
   iterations with the stopping test disabled, except for the GRU
   adjoint with PN_JAC_DENSE (one map pass, then chain passes until its own test passes),
   whose candidates (group 0, 1, 2, 3, 4, 5, 6, 8, 16) are timed as whole calls at opts->tol
   (ms_per_iter: ms per call).
   workspace: at least pn_workspace_bytes(op | PN_OP_TUNE, ...) bytes (256-byte aligned).
   Errors: those of the solve call (a candidate that the route rejects is skipped);
   PN_ERR_HIP if timing fails. */
#define PN_OP_TUNE 0x100
#define PN_TUNE_MAX_CAND 32
typedef struct {
    int32_t tile;             /* best candidate's pn_opts.tile */
    int32_t group;            /* best candidate's pn_opts.group */
    double ms_per_iter;       /* its time per iteration (0 when from_cache) */
    int32_t from_cache;       /* 1: taken from the process or file cache, nothing was run */
    int32_t ncand;            /* candidates timed (0 when from_cache) */
    int32_t cand_tile[PN_TUNE_MAX_CAND];
    int32_t cand_group[PN_TUNE_MAX_CAND];
    float cand_ms[PN_TUNE_MAX_CAND];   /* ms per iteration; < 0: the route rejected it */
} pn_tuned;
pn_status pn_autotune(int op, const pn_cell_desc* cell, const pn_batch* batch,
                      const void* const* bufs, double lambda, const pn_opts* opts,
                      int32_t probe_iters, void* workspace, size_t workspace_bytes,
                      void* stream, pn_tuned* out);
/* Forget the in-process autotune results (the cache file is left as it is). */
void pn_autotune_reset(void);

/* Copy-bandwidth probe: copies `bytes` (a positive multiple of 16) from src to dst (device,
   16-byte aligned, not overlapping) with plain streaming kernels — two forms (four 16-byte
   loads in flight per thread; one per thread and iteration with non-temporal hints) on grids
   of 1, 2, 3, 4, 6 and 8 workgroups of 256 threads per CU — each once untimed and then `reps`
   times between HIP events on `stream`, and returns in *gbs (host) the best achieved rate
   counting read plus write bytes (2 * bytes * reps / time).  It gives the HBM rate a simple
   kernel reaches on the device, next to the published peak, and dispatches of known size for
   scaling the FETCH_SIZE / WRITE_SIZE counters (kernels copy_probe_kernel<0>, <1>).  Runs 12
   configurations: about 12 * (reps + 1) copies of `bytes`. */
pn_status pn_copy_probe(const void* src, void* dst, size_t bytes, int reps, void* stream,
                        double* gbs);

void pn_profile_begin(void);
void pn_profile_end(void);
int pn_profile_read(const char* family, double* total_ms, int64_t* launches);

const char* pn_status_str(int status);
const char* pn_last_error(void);
int pn_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PNEWTON_H */
