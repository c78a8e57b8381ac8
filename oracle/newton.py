"""Sequential parallel-Newton loop (test infrastructure): Alg. alg:deer, one step at a time.

Each iteration, for the current guess s^(i):
  1. residual r_t = s_t - f_t(s_{t-1}) for every t, with s_0 fixed (eq. r_def);
  2. stop when max |r| < tol (the stopping quantity is left open by the thesis's
     ComputeError; the oracle uses the infinity norm of the residual, or optionally the
     infinity norm of the last update as in the Ch. 3 GRU experiments);
  3. transition matrices A~_t chosen per Tab. fxd_pt_sum:
        "dense"  (Newton / DEER)       A~_t = A_t = df_t/ds_{t-1}(s_{t-1})   (eq. lil_j)
        "diag"   (quasi-Newton)        A~_t = diag(A_t)                      (eq. quasi_lds)
        "picard"                        A~_t = I                              (Prop. prop:picard)
        "jacobi"                        A~_t = 0                              (Prop. prop:jacobi)
        "scale:k" (scale-ELK)           A~_t = (1 - k) A_t
        "clip"   (clip-ELK)            A~_t = clip(diag(A_t), -1, 1)
     or any callable returning them;
  4. the Newton step solves J~ Delta = -r by forward substitution (eq. lin_rr):
        Delta_1 = -r_1,   Delta_t = A~_t Delta_{t-1} - r_t;
  5. s <- s + Delta, then the reset heuristic (Ch. 3 global-convergence discussion and the
     trained AR-GRU experiment of Ch. 4): any time-step vector that is non-finite or has an
     entry larger than ``reset_abs`` in magnitude is set to zero.

Converged-prefix skipping (``freeze`` = a block length in steps, optional): convergence is
causal (the induction in the proof of Prop. prop:global_convergence), so after step 2 the
leading blocks of ``freeze`` steps whose residual is below tol are frozen: the step is
taken as exactly zero there, and steps 3-5 run on the rest of the sequence only, with
Delta = 0 entering it (the solve restarts at the first open block, like a sequence head).
Frozen states never change again, so their residuals stay below tol.

The iteration count is the number of updates applied; the result is returned as soon as
the stopping test passes on the current iterate.  The default cap is T updates with the
residual rule and T + 1 with the update-norm rule (the loop bound of Alg. alg:deer).  By Prop. prop:global_convergence the
loop ends within T updates for every choice of A~_t (exact arithmetic).
"""
import numpy as np


def linearize(cell, x, s0, s):
    """Residuals and the arguments every transition-matrix choice needs.

    Returns (h, r) where h[t] = s_{t-1} (h[0] = s_0) and r[t] = s_t - f_t(s_{t-1}).
    """
    T = x.shape[0]
    h = np.concatenate([np.asarray(s0, np.float64)[None], s[:-1]], axis=0)
    tt = np.arange(T)
    r = s - cell.f(h, x, t=tt)
    return h, r


def transition_matrices(cell, x, h, mode):
    """A~_t for every t as dense [T, D, D] matrices (diagonal modes stored densely)."""
    T, D = h.shape
    tt = np.arange(T)
    if callable(mode):
        return np.asarray(mode(cell, x, h), np.float64)
    if mode == "dense":
        return cell.jac(h, x, t=tt)
    if mode == "diag":
        return np.einsum("ti,ij->tij", cell.jac_diag(h, x, t=tt), np.eye(D))
    if mode == "picard":
        return np.broadcast_to(np.eye(D), (T, D, D)).copy()
    if mode == "jacobi":
        return np.zeros((T, D, D))
    if isinstance(mode, str) and (mode == "clip" or mode.startswith("clip:")):
        # clip-ELK (Sec. "Further extensions: scale- and clip-ELK"): each diagonal entry
        # clipped to [lo, hi], by default [-1, 1]
        lo, hi = (-1.0, 1.0) if mode == "clip" else map(float, mode.split(":")[1:3])
        d = np.clip(cell.jac_diag(h, x, t=tt), lo, hi)
        return np.einsum("ti,ij->tij", d, np.eye(D))
    if isinstance(mode, str) and mode.startswith("scale:"):
        # scale-ELK (same section): A~_t = (1 - k) A_t
        k = float(mode.split(":", 1)[1])
        return (1.0 - k) * cell.jac(h, x, t=tt)
    if isinstance(mode, str) and mode.startswith("diagscale:"):
        # scale-ELK on the quasi (diagonal) approximation: A~_t = (1 - k) diag(A_t)
        k = float(mode.split(":", 1)[1])
        return np.einsum("ti,ij->tij", (1.0 - k) * cell.jac_diag(h, x, t=tt), np.eye(D))
    raise ValueError(mode)


def forward_substitution(At, r):
    """Solve J~ Delta = -r for block-bidiagonal J~ (eq. big_j) by eq. lin_rr.

    At [T, D, D] (At[0] is never used: Delta_0 = 0 because s_0 is fixed), r [T, D].
    """
    T, D = r.shape
    delta = np.empty((T, D))
    prev = np.zeros(D)
    with np.errstate(over="ignore", invalid="ignore"):
        for t in range(T):
            prev = (At[t] @ prev if t > 0 else 0.0) - r[t]
            delta[t] = prev
    return delta


def apply_reset(s, reset_abs):
    """Reset heuristic: zero every time-step vector that is non-finite or too large."""
    with np.errstate(invalid="ignore"):
        bad = ~np.isfinite(s).all(axis=1) | (np.abs(s).max(axis=1) > reset_abs)
    s[bad] = 0.0
    return int(bad.sum())


def frozen_prefix(r, block, tol):
    """Start of the open part: ``block`` times the number of leading blocks of ``block``
    steps whose max |r| is below tol (NaN is not below)."""
    T = r.shape[0]
    t0 = 0
    while t0 < T:
        with np.errstate(invalid="ignore"):
            ok = bool(np.max(np.abs(r[t0:t0 + block])) < tol)
        if not ok:
            break
        t0 += block
    return min(t0, T)


def newton(cell, x, s0, s_init=None, mode="dense", tol=1e-10, max_iters=None,
           reset_abs=1e4, stop="resid", step=None, history=False, freeze=0):
    """Run the loop on one sequence.  ``step(cell, x, h, r, t0)`` replaces steps 3-4 on
    steps t0.. (used by ELK); ``freeze`` > 0 turns on converged-prefix skipping.

    Returns a dict: s, iters, converged, resets, max_resid, and optionally the list of
    iterates (``history``, s^(0) first) and residual norms.
    """
    x = np.asarray(x, np.float64)
    T, D = x.shape[0], cell.D
    s = np.zeros((T, D)) if s_init is None else np.array(s_init, np.float64)
    # Alg. alg:deer runs i = 0..T, an update and then the error test each time: T + 1
    # updates at most.  With the residual as the error, the exact trajectory (reached after
    # at most T updates) already passes the test before the last one; with the update norm
    # the (T+1)-th, zero update is what shows convergence.
    if max_iters is None:
        max_iters = T + 1 if stop == "delta" else T
    max_iters = int(max_iters)
    hist = [s.copy()] if history else None
    norms = []
    resets = 0
    i = 0
    while True:
        h, r = linearize(cell, x, s0, s)
        with np.errstate(invalid="ignore"):
            rn = float(np.max(np.abs(r))) if T else 0.0
        norms.append(rn)
        if stop == "resid" and rn < tol:
            return dict(s=s, iters=i, converged=True, resets=resets, max_resid=rn,
                        history=hist, resid_norms=norms)
        if i >= max_iters:
            return dict(s=s, iters=i, converged=False, resets=resets, max_resid=rn,
                        history=hist, resid_norms=norms)
        t0 = frozen_prefix(r, int(freeze), tol) if freeze else 0
        delta = np.zeros_like(s)
        if step is None:
            At = transition_matrices(cell, x, h, mode)
            delta[t0:] = forward_substitution(At[t0:], r[t0:])
        else:
            delta[t0:] = step(cell, x, h, r, t0)
        with np.errstate(invalid="ignore", over="ignore"):
            s = s + delta
        resets += apply_reset(s, reset_abs)
        i += 1
        if history:
            hist.append(s.copy())
        if stop == "delta":
            with np.errstate(invalid="ignore"):
                dn = float(np.max(np.abs(delta)))
            if dn < tol:
                _, r2 = linearize(cell, x, s0, s)
                return dict(s=s, iters=i, converged=True, resets=resets,
                            max_resid=float(np.max(np.abs(r2))), history=hist,
                            resid_norms=norms)


def newton_batch(cell, x, s0, offsets, **kw):
    """``newton`` on every sequence of a back-to-back batch; returns (s [N, D], infos)."""
    offsets = np.asarray(offsets, np.int64)
    s = np.empty((x.shape[0], cell.D))
    infos = []
    s_init = kw.pop("s_init", None)
    for b in range(offsets.size - 1):
        a, e = offsets[b], offsets[b + 1]
        init = None if s_init is None else s_init[a:e]
        out = newton(cell, x[a:e], s0[b], s_init=init, **kw)
        s[a:e] = out["s"]
        infos.append(out)
    return s, infos
