"""Seeded synthetic workloads: random cells, inputs and sequence lengths.

This module only draws random numbers; it holds none of the method's arithmetic and is
the one piece shared by the HIP path's callers and the test oracle.

Every draw uses ``numpy.random.default_rng(seed)`` (PCG64) in float64 and a fixed order:
  1. sequence lengths (ragged workloads only): integers uniform on [t_min, t_max];
  2. weights: GRU W_z, W_r, W_n (D x Dx) then U_z, U_r, U_n (D x D), all N(0, 1/D);
     tanh-RNN W (D x D) ~ N(0, g^2/D) then U (D x Dx) ~ N(0, 1/D);
  3. biases are zero (no draw);
  4. inputs x [N, Dx] ~ N(0, 1) (times the workload's input scale), sequences back to back.
The initial state s_0 and the initial guess are zero.

The mean-field RNN (cell "meanfield", Ch. 5 predictability experiments) draws W (D x D) ~
N(0, g^2/D) with its diagonal then set to zero (no self-coupling), takes U = I (Dx = D) and
zero biases, drives every sequence by the mild sinusoid x_t[i] = 0.1 sin(0.05 t + i) (t the
step within the sequence, no draw), and draws s_0 [B, D] ~ N(0, 1) after W.

These are the shapes of the thesis's synthetic "untrained GRU" evaluation benchmark (a
randomly initialised GRU, Ch. 3) and of its mean-field tanh RNN family, whose gain g sets
the regime (predictable for g < 1, chaotic above; Ch. 5).
"""
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    cell: str                 # "gru" | "tanh" | "meanfield"
    D: int
    Dx: int
    B: int
    T: int = 0                # uniform length (0 when ragged)
    t_min: int = 0            # ragged lengths ~ U{t_min..t_max}
    t_max: int = 0
    gain: float = 1.0         # tanh-RNN recurrent gain g
    method: str = "deer"      # "deer" | "elk"
    jac: str = "diag"         # "diag" | "dense"
    dtype: str = "f32"        # "f32" | "f64"
    compose: str = "native"   # "native" | "bf16"
    tol: float = 1e-5
    lambdas: tuple = ()
    backward: bool = False
    input_scale: float = 1.0  # inputs x ~ N(0, input_scale^2)

    def scaled(self, **kw):
        return replace(self, **kw)


# The five workloads (sizes as quoted for the method's benchmark suite).
GRU4_DENSE_F64 = Workload("gru4-dense-f64", "gru", D=4, Dx=4, B=1, T=1024,
                          jac="dense", dtype="f64", tol=1e-10)
GRU64_QUASI = Workload("gru64-quasi-f32", "gru", D=64, Dx=32, B=16, T=65536,
                       jac="diag", tol=1e-5, backward=True)
TANH32_DENSE_BF16 = Workload("tanh32-dense-bf16", "tanh", D=32, Dx=16, B=32, T=16384,
                             gain=0.9, jac="dense", compose="bf16", tol=1e-5)
TANH16_ELK = Workload("tanh16-elk-chaotic", "tanh", D=16, Dx=16, B=8, T=8192,
                      gain=1.5, method="elk", jac="dense", tol=1e-6,
                      lambdas=(1e-2, 1e-1, 1.0))
GRU48_RAGGED = Workload("gru48-ragged-quasi", "gru", D=48, Dx=24, B=256,
                        t_min=512, t_max=32768, jac="diag", tol=1e-5, backward=True)

# The ELK workload in its chaotic regime.  At D = 16 the stated input drive (x ~ N(0, 1))
# suppresses chaos (largest Lyapunov exponent -0.19 .. -0.30 for seeds 0-2), and with weaker
# drive most draws of W at gain 1.5 settle to non-chaotic motion as well; with inputs scaled by
# 0.1, seed CHAOTIC_SEED (the first of seeds 0..11 found with a positive exponent) gives
# +0.018 .. +0.026 on all 8 sequences (Alg. alg:LLE_estimate on the FP64 rollout).
TANH16_ELK_CHAOTIC = replace(TANH16_ELK, name="tanh16-elk-chaotic-lowdrive", input_scale=0.1)
CHAOTIC_SEED = 9

# The mean-field RNN of the LLE-threshold sweep (Ch. 5): DEER (ELK with lambda = 0), T = 1000
# (the length the thesis highlights), the gain g swept per run.
MEANFIELD16 = Workload("meanfield16-lle-sweep", "meanfield", D=16, Dx=16, B=1, T=1000,
                       gain=1.0, method="deer", jac="dense", tol=1e-5)
# The same family at the thesis's state size D = 100 (one sequence per seed).
MEANFIELD100 = Workload("meanfield100-lle-sweep", "meanfield", D=100, Dx=100, B=1, T=1000,
                        gain=1.0, method="deer", jac="dense", tol=1e-5)

ALL = {w.name: w for w in (GRU4_DENSE_F64, GRU64_QUASI, TANH32_DENSE_BF16, TANH16_ELK,
                           GRU48_RAGGED)}


@dataclass
class Instance:
    work: Workload
    params: np.ndarray        # packed float64 parameters
    x: np.ndarray             # [N, Dx] float64
    s0: np.ndarray            # [B, D] float64
    offsets: np.ndarray       # [B+1] int64
    seed: int = 0

    @property
    def N(self):
        return int(self.offsets[-1])

    @property
    def lengths(self):
        return np.diff(self.offsets)


def draw_lengths(rng, work: Workload):
    if work.T:
        return np.full(work.B, work.T, dtype=np.int64)
    return rng.integers(work.t_min, work.t_max + 1, size=work.B).astype(np.int64)


def draw_params(rng, work: Workload):
    D, Dx = work.D, work.Dx
    if work.cell == "gru":
        sd = np.sqrt(1.0 / D)
        W = [rng.normal(0.0, sd, size=(D, Dx)) for _ in range(3)]
        U = [rng.normal(0.0, sd, size=(D, D)) for _ in range(3)]
        return np.concatenate([w.ravel() for w in W] + [u.ravel() for u in U]
                              + [np.zeros(3 * D), np.zeros(D)])
    if work.cell == "meanfield":
        W = rng.normal(0.0, work.gain / np.sqrt(D), size=(D, D))
        np.fill_diagonal(W, 0.0)
        return np.concatenate([W.ravel(), np.eye(D, Dx).ravel(), np.zeros(D)])
    if work.cell == "tanh":
        W = rng.normal(0.0, work.gain / np.sqrt(D), size=(D, D))
        U = rng.normal(0.0, np.sqrt(1.0 / D), size=(D, Dx))
        return np.concatenate([W.ravel(), U.ravel(), np.zeros(D)])
    raise ValueError(work.cell)


def make_instance(work: Workload, seed: int = 0, lengths: Optional[np.ndarray] = None):
    rng = np.random.default_rng(seed)
    lens = draw_lengths(rng, work)
    if lengths is not None:
        lens = np.asarray(lengths, np.int64)
    params = draw_params(rng, work)
    offsets = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    if work.cell == "meanfield":
        steps = np.concatenate([np.arange(n) for n in lens]) if lens.size else np.zeros(0)
        x = 0.1 * np.sin(0.05 * steps[:, None] + np.arange(work.Dx)[None, :])
        s0 = rng.standard_normal(size=(lens.size, work.D))
        return Instance(work, params, x, s0, offsets, seed)
    x = rng.standard_normal(size=(int(offsets[-1]), work.Dx))
    if work.input_scale != 1.0:
        x = x * work.input_scale
    s0 = np.zeros((lens.size, work.D))
    return Instance(work, params, x, s0, offsets, seed)
