"""Sequential evaluation of an SSM: the definition of the answer (test infrastructure).

Ch. 2, Problem Statement "Unrolling an SSM": given s_0, evaluate s_1..s_T with
s_t = f_t(s_{t-1}) (eq. ssm), the input x_t curried into f_t (eq. ssm_driven).
The true trajectory s* is the unique zero of the residual r_t = s_t - f_t(s_{t-1})
(eq. r_def), so every parallel Newton method must reach exactly this result.
"""
import numpy as np


def rollout(cell, x, s0):
    """One sequence: x [T, Dx], s0 [D] -> s [T, D], one step at a time."""
    x = np.asarray(x, np.float64)
    T = x.shape[0]
    s = np.empty((T, cell.D))
    h = np.asarray(s0, np.float64)
    for t in range(T):
        h = cell.f(h, x[t], t=t)
        s[t] = h
    return s


def rollout_batch(cell, x, s0, offsets):
    """Many sequences laid out back to back.

    x [N, Dx] holds sequence b in rows offsets[b]:offsets[b+1]; s0 [B, D].
    The loop runs over time only; at each t every sequence still running takes one
    step together (a vectorised form of ``rollout`` that does the same arithmetic).
    """
    x = np.asarray(x, np.float64)
    offsets = np.asarray(offsets, np.int64)
    B = offsets.size - 1
    lens = np.diff(offsets)
    s = np.empty((x.shape[0], cell.D))
    h = np.array(s0, np.float64).reshape(B, cell.D)
    for t in range(int(lens.max()) if B else 0):
        act = np.nonzero(lens > t)[0]
        rows = offsets[act] + t
        h_new = cell.f(h[act], x[rows], t=t)
        h[act] = h_new
        s[rows] = h_new
    return s
