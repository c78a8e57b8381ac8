"""Largest Lyapunov exponent (test infrastructure).

Def. def:predictable_systems: LLE = lim (1/T) log ||A_T ... A_1||; the system is predictable
when it is negative.  Alg. alg:LLE_estimate evaluates it stably by pushing a unit vector
through the Jacobians, renormalising each step and averaging the log stretch factors; the
thesis averages the estimate over three random unit starting vectors.
"""
import numpy as np


def lle_estimate(jacobians, u0):
    u = np.asarray(u0, np.float64)
    u = u / np.linalg.norm(u)
    total = 0.0
    T = len(jacobians)
    for t in range(T):
        u = jacobians[t] @ u
        stretch = np.linalg.norm(u)
        u = u / stretch
        total += np.log(stretch)
    return total / T


def lle_average(jacobians, n_vectors=3, seed=0):
    rng = np.random.default_rng(seed)
    D = jacobians[0].shape[0]
    vals = [lle_estimate(jacobians, rng.standard_normal(D)) for _ in range(n_vectors)]
    return float(np.mean(vals))


def trajectory_jacobians(cell, x, s0, s):
    """A_t = df/ds_{t-1} along the trajectory s (s_0 first)."""
    h = np.concatenate([np.asarray(s0, np.float64)[None], np.asarray(s, np.float64)[:-1]],
                       axis=0)
    return cell.jac(h, np.asarray(x, np.float64), t=np.arange(len(x)))


def trajectory_lle(cell, x, s0, s, n_vectors=3, seed=0):
    """LLE along a trajectory s (the Jacobians A_t evaluated at s_{t-1})."""
    h = np.concatenate([np.asarray(s0, np.float64)[None], s[:-1]], axis=0)
    J = cell.jac(h, x, t=np.arange(len(x)))
    return lle_average(J, n_vectors=n_vectors, seed=seed)
