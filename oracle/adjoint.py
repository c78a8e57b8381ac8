"""Backpropagation through time as a reverse linear recurrence (test infrastructure).

Ch. 3, "Training and the backwards pass": the chain rule through s_t = f_theta(s_{t-1})
(eqs. bptt, bptt_lds) is a linear dynamical system in reverse time whose transition
matrices are the transposed dynamics Jacobians A_t^T, and the parameter gradient is the sum
over t of (df/dtheta)^T applied to the adjoint (eq. unrolled_bwds).

For a loss L = sum_t l_t(s_t) with g_t = dl_t/ds_t, the total derivative
lambda_t = dL/ds_t obeys
    lambda_T = g_T,    lambda_t = g_t + A_{t+1}^T lambda_{t+1},
and then
    dL/dtheta = sum_t (df_t/dtheta)^T lambda_t,
    dL/dx_t   = (df_t/dx_t)^T lambda_t,
    dL/ds_0   = A_1^T lambda_1.
The oracle runs that recursion one step at a time.
"""
import numpy as np


def adjoint(cell, x, s0, s, g):
    """One sequence: returns (lam [T, D], dtheta packed, dx [T, Dx], ds0 [D])."""
    x = np.asarray(x, np.float64)
    s = np.asarray(s, np.float64)
    g = np.asarray(g, np.float64)
    T, D = s.shape
    h = np.concatenate([np.asarray(s0, np.float64)[None], s[:-1]], axis=0)
    lam = np.empty((T, D))
    nxt = np.zeros(D)
    for t in range(T - 1, -1, -1):
        if t == T - 1:
            lam[t] = g[t]
        else:
            lam[t] = g[t] + cell.vjp(h[t + 1], x[t + 1], lam[t + 1], t=t + 1)
    grads, dx = cell.param_vjp(h, x, lam)
    ds0 = cell.vjp(h[0], x[0], lam[0], t=0) if T else np.zeros(D)
    return lam, cell.pack_grad(grads), dx, ds0


def adjoint_batch(cell, x, s0, s, g, offsets):
    """Back-to-back batch, vectorised over sequences in reverse time.

    Returns (lam [N, D], dtheta packed (summed over the batch), dx [N, Dx], ds0 [B, D]).
    """
    x = np.asarray(x, np.float64)
    s = np.asarray(s, np.float64)
    g = np.asarray(g, np.float64)
    offsets = np.asarray(offsets, np.int64)
    B = offsets.size - 1
    lens = np.diff(offsets)
    D = cell.D
    s0 = np.asarray(s0, np.float64).reshape(B, D)
    # h[n] = state feeding step n (s_{t-1}, or s_0 at a sequence head)
    h = np.empty_like(s)
    h[1:] = s[:-1]
    h[offsets[:-1][lens > 0]] = s0[lens > 0]
    lam = np.empty_like(s)
    cur = np.zeros((B, D))
    Tmax = int(lens.max()) if B else 0
    for t in range(Tmax - 1, -1, -1):
        act = np.nonzero(lens > t)[0]
        rows = offsets[act] + t
        last = lens[act] == t + 1
        v = g[rows].copy()
        cont = ~last
        if cont.any():
            nrows = rows[cont] + 1
            v[cont] += cell.vjp(h[nrows], x[nrows], cur[act[cont]], t=t + 1)
        cur[act] = v
        lam[rows] = v
    grads, dx = cell.param_vjp(h, x, lam)
    ds0 = np.zeros((B, D))
    heads = offsets[:-1][lens > 0]
    ds0[lens > 0] = cell.vjp(h[heads], x[heads], lam[heads], t=0)
    return lam, cell.pack_grad(grads), dx, ds0


def adjoint_residual(cell, x, s0, s, g, lam):
    """rho_t = lambda_t - g_t - A_{t+1}^T lambda_{t+1} (zero at the exact adjoint)."""
    T, D = s.shape
    h = np.concatenate([np.asarray(s0, np.float64)[None], s[:-1]], axis=0)
    rho = lam - g
    if T > 1:
        rho[:-1] -= cell.vjp(h[1:], x[1:], lam[1:], t=np.arange(1, T))
    return rho
