"""ELK: the Levenberg-Marquardt step as a Kalman filter (test infrastructure).

Ch. 4.  The LM step minimises the linearised merit (eq. linmerit) plus lambda/2 ||Delta||^2
(eq. lagrangian); Prop. prop:ELK identifies the minimiser with the posterior mode of a
linear-Gaussian SSM (eq. lgssm) whose dynamics are the linearisation of f (process noise
I, prior s_1 ~ N(f(s_0), I)) and whose emissions are the previous iterate s^(i) with noise
variance sigma^2 = 1/lambda.  ELK itself runs the Kalman *filter* and takes the filtered
means as the next iterate (Ch. 4, "Implementation Details").

Written in the step coordinates Delta_t = s_t - s^(i)_t the model reads
    Delta_t = A~_t Delta_{t-1} - r_t + w_t,   w_t ~ N(0, I),   Delta_0 = 0,
    0       = Delta_t + v_t,                  v_t ~ N(0, I / lambda),
and the filter of Sec. "Dynamics perspective on ELK" becomes
    predict:  m- = A~_t m - r_t,             P- = A~_t P A~_t^T + I
    update:   K  = P- (P- + I/lambda)^-1  =  lambda P- (lambda P- + I)^-1
              m  = (I - K) m-,               P  = (I - K) P-,      Delta_t = m,
starting from m = 0, P = 0.  The attenuation matrix of that section is Gamma_t = I - K.
With lambda = 0 the gain vanishes and the recursion is exactly the DEER step (eq. lin_rr).

The same filter can be evaluated by an associative scan over 5-tuples (A, b, C, eta, J)
(the parallel Kalman filter the thesis cites in Ch. 2).  ``kalman_leaf`` and
``kalman_combine`` write that element and its combination rule out for this model;
folding the leaves left to right reproduces the filter.
"""
import numpy as np

from . import newton as _newton


def filter_step(At, r, lam):
    """Sequential Kalman filter in Delta-coordinates.

    At [T, D, D] transition matrices (At[0] unused), r [T, D] residuals, lam >= 0.
    Returns (Delta [T, D], P [T, D, D] filtered covariances, Gamma [T, D, D]).
    """
    T, D = r.shape
    eye = np.eye(D)
    m = np.zeros(D)
    P = np.zeros((D, D))
    delta = np.empty((T, D))
    covs = np.empty((T, D, D))
    gammas = np.empty((T, D, D))
    with np.errstate(over="ignore", invalid="ignore"):
        for t in range(T):
            A = At[t] if t > 0 else np.zeros((D, D))
            m_pred = A @ m - r[t]
            P_pred = A @ P @ A.T + eye
            K = lam * P_pred @ np.linalg.inv(lam * P_pred + eye)
            G = eye - K
            m = G @ m_pred
            P = G @ P_pred
            P = 0.5 * (P + P.T)
            delta[t] = m
            covs[t] = P
            gammas[t] = G
    return delta, covs, gammas


def smoother_step(At, r, lam):
    """The exact Levenberg-Marquardt step: the posterior mode of the same LGSSM (Prop.
    prop:ELK), by the Kalman filter followed by the Rauch-Tung-Striebel backward pass
    (Sec. "Bayesian inference for linear Gaussian SSMs"):
        E_t = P_t A~_{t+1}^T (P-_{t+1})^-1,   m^s_t = m_t + E_t (m^s_{t+1} - m-_{t+1}),
    with m^s_T = m_T.  The means alone are needed, so the smoothed covariances are not formed.
    Returns Delta [T, D]."""
    T, D = r.shape
    eye = np.eye(D)
    m = np.zeros(D)
    P = np.zeros((D, D))
    ms, Ps, mp, Pp = (np.empty((T, D)), np.empty((T, D, D)), np.empty((T, D)),
                      np.empty((T, D, D)))
    with np.errstate(over="ignore", invalid="ignore"):
        for t in range(T):                                   # filter, keeping the predictions
            A = At[t] if t > 0 else np.zeros((D, D))
            mp[t] = A @ m - r[t]
            Pp[t] = A @ P @ A.T + eye
            G = np.linalg.inv(lam * Pp[t] + eye)
            m = G @ mp[t]
            P = G @ Pp[t]
            P = 0.5 * (P + P.T)
            ms[t], Ps[t] = m, P
        out = np.empty((T, D))
        if T:
            out[T - 1] = ms[T - 1]
        for t in range(T - 2, -1, -1):                       # backward pass
            E = Ps[t] @ At[t + 1].T @ np.linalg.inv(Pp[t + 1])
            out[t] = ms[t] + E @ (out[t + 1] - mp[t + 1])
    return out


def lm_step_dense(At, r, lam):
    """The same step by its definition: -(J^T J + lambda I)^-1 J^T r with the block
    bidiagonal Jacobian of the residual (identity blocks on the diagonal, -A~_t below)."""
    T, D = r.shape
    J = np.eye(T * D)
    for t in range(1, T):
        J[t * D:(t + 1) * D, (t - 1) * D:t * D] = -At[t]
    rhs = -J.T @ r.reshape(-1)
    return np.linalg.solve(J.T @ J + lam * np.eye(T * D), rhs).reshape(T, D)


def elk(cell, x, s0, lam, mode="dense", smoother=False, **kw):
    """The Newton loop of ``oracle.newton`` with its step replaced by the ELK filter (or,
    with ``smoother``, by the exact LM step)."""
    def step(cell_, x_, h, r, t0):
        # the step runs on steps t0.. from m = 0, P = 0 (t0 > 0: a frozen prefix)
        At = _newton.transition_matrices(cell_, x_, h, mode)
        if smoother:
            return smoother_step(At[t0:], r[t0:], lam)
        return filter_step(At[t0:], r[t0:], lam)[0]
    return _newton.newton(cell, x, s0, step=step, **kw)


# ---- associative-scan form -------------------------------------------------------------

def kalman_leaf(A_t, r_t, lam, first):
    """Element of the parallel Kalman filter for one step of the Delta-model.

    It encodes p(Delta_t | Delta_{t-1}, observation at t) = N(A Delta_{t-1} + b, C) together
    with the observation likelihood of Delta_{t-1} in information form exp(-x^T J x/2 + eta^T x).
    With observation noise I/lambda and process noise I, the Kalman gain of a single step is
    kappa I, kappa = lambda / (1 + lambda).  The first step has no predecessor (Delta_0 = 0).
    """
    D = r_t.size
    eye = np.eye(D)
    k = lam / (1.0 + lam)
    if first:
        return (np.zeros((D, D)), -r_t * (1.0 - k), eye * (1.0 - k),
                np.zeros(D), np.zeros((D, D)))
    return ((1.0 - k) * A_t, -r_t * (1.0 - k), eye * (1.0 - k),
            k * A_t.T @ r_t, k * A_t.T @ A_t)


def kalman_combine(ei, ej):
    """Combine an earlier element ei with a later element ej (conditional-Gaussian algebra)."""
    Ai, bi, Ci, etai, Ji = ei
    Aj, bj, Cj, etaj, Jj = ej
    D = bi.size
    eye = np.eye(D)
    G = np.linalg.inv(eye + Ci @ Jj)
    H = np.linalg.inv(eye + Jj @ Ci)
    A = Aj @ G @ Ai
    b = Aj @ G @ (bi + Ci @ etaj) + bj
    C = Aj @ G @ Ci @ Aj.T + Cj
    eta = Ai.T @ H @ (etaj - Jj @ bi) + etai
    J = Ai.T @ H @ Jj @ Ai + Ji
    return (A, b, C, eta, J)


def filter_by_elements(At, r, lam):
    """Fold the leaves left to right: Delta_t is b of the prefix 1..t, its covariance C."""
    T, D = r.shape
    delta = np.empty((T, D))
    covs = np.empty((T, D, D))
    acc = None
    for t in range(T):
        e = kalman_leaf(At[t], r[t], lam, first=(t == 0))
        acc = e if acc is None else kalman_combine(acc, e)
        delta[t] = acc[1]
        covs[t] = acc[2]
    return delta, covs
