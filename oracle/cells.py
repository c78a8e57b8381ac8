"""Dynamics functions f(s_{t-1}, x_t) of the oracle, in float64 (test infrastructure).

The thesis curries inputs into the dynamics (Ch. 2, eq. ssm_driven: f_t(s) = f(s, u_t)),
so every cell below maps a state h = s_{t-1} in R^D and an input x = x_t in R^Dx to
the next state s_t.  Leading batch axes are allowed on h and x.

For each cell the oracle provides:
  f(h, x)                  -- the next state;
  jac(h, x)                -- A_t = df/ds_{t-1} (eq. lil_j), dense D x D;
  jac_diag(h, x)           -- diag(A_t) in closed form (Ch. 3: the closed-form diagonal is
                              what lets quasi-DEER avoid forming A_t);
  vjp(h, x, v)             -- A_t^T v (Ch. 3, "Training and the backwards pass": a VJP gives
                              A_t^T times a vector without forming A_t);
  param_vjp(h, x, v)       -- (df/dtheta)^T v as a dict shaped like the parameters, and
                              (df/dx)^T v (the terms summed in eq. unrolled_bwds).

The thesis gives the GRU only by reference (its GRU experiments follow the original GRU
paper; the equations sat in a figure).  The oracle fixes the "reset-after" GRU:
    z = sigmoid(W_z x + U_z h + b_z)
    r = sigmoid(W_r x + U_r h + b_r)
    q = U_n h + b_hn
    n = tanh(W_n x + b_n + r * q)
    f = (1 - z) * n + z * h
Its Jacobian, written with a = (h - n) z (1 - z), b = (1 - z)(1 - n^2) r and
c = (1 - z)(1 - n^2) q r (1 - r), is
    A = diag(z) + diag(a) U_z + diag(b) U_n + diag(c) U_r.
The tanh-RNN is f = tanh(W h + U x + bias), A = diag(1 - f^2) W.  The mean-field RNN of
the predictability experiments (Ch. 5, "Experiments") places the nonlinearity before the
coupling, f = W tanh(h) + U x + bias (the state is a current), so A = W diag(1 - tanh(h)^2).
The affine cell
f = M h + N x + c (optionally with a per-step M_t) is a linear dynamical system (eq. lds),
used to pin the one-iteration properties.

Parameter packing (row-major, one flat float64 vector):
  GRU:    [W_z; W_r; W_n] (3D x Dx) | [U_z; U_r; U_n] (3D x D) | [b_z; b_r; b_n] (3D) | b_hn (D)
  tanh:   W (D x D) | U (D x Dx) | b (D)
  meanfield: W (D x D) | U (D x Dx) | b (D)
  affine: M (D x D) | N (D x Dx) | c (D)
"""
import numpy as np


def _sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def gru_param_count(D, Dx):
    return 3 * D * Dx + 3 * D * D + 3 * D + D


def tanh_param_count(D, Dx):
    return D * D + D * Dx + D


def affine_param_count(D, Dx):
    return D * D + D * Dx + D


class GRU:
    """Reset-after GRU cell (see module docstring for the equations)."""

    name = "gru"

    def __init__(self, params, D, Dx):
        p = np.asarray(params, dtype=np.float64).ravel()
        assert p.size == gru_param_count(D, Dx), (p.size, D, Dx)
        self.D, self.Dx = D, Dx
        o = 0
        W = p[o:o + 3 * D * Dx].reshape(3 * D, Dx); o += 3 * D * Dx
        U = p[o:o + 3 * D * D].reshape(3 * D, D); o += 3 * D * D
        b = p[o:o + 3 * D]; o += 3 * D
        self.b_hn = p[o:o + D].copy(); o += D
        self.W_z, self.W_r, self.W_n = W[:D].copy(), W[D:2 * D].copy(), W[2 * D:].copy()
        self.U_z, self.U_r, self.U_n = U[:D].copy(), U[D:2 * D].copy(), U[2 * D:].copy()
        self.b_z, self.b_r, self.b_n = b[:D].copy(), b[D:2 * D].copy(), b[2 * D:].copy()

    def gates(self, h, x):
        z = _sigmoid(x @ self.W_z.T + h @ self.U_z.T + self.b_z)
        r = _sigmoid(x @ self.W_r.T + h @ self.U_r.T + self.b_r)
        q = h @ self.U_n.T + self.b_hn
        n = np.tanh(x @ self.W_n.T + self.b_n + r * q)
        return z, r, q, n

    def f(self, h, x, t=None):
        z, r, q, n = self.gates(h, x)
        return (1.0 - z) * n + z * h

    def _coeffs(self, h, x):
        z, r, q, n = self.gates(h, x)
        a = (h - n) * z * (1.0 - z)
        e = (1.0 - z) * (1.0 - n * n)
        b = e * r
        c = e * q * r * (1.0 - r)
        return z, r, q, n, a, b, c, e

    def jac(self, h, x, t=None):
        z, r, q, n, a, b, c, e = self._coeffs(h, x)
        eye = np.eye(self.D)
        return (z[..., :, None] * eye
                + a[..., :, None] * self.U_z
                + b[..., :, None] * self.U_n
                + c[..., :, None] * self.U_r)

    def jac_diag(self, h, x, t=None):
        z, r, q, n, a, b, c, e = self._coeffs(h, x)
        return (z + a * np.diag(self.U_z) + b * np.diag(self.U_n)
                + c * np.diag(self.U_r))

    def vjp(self, h, x, v, t=None):
        z, r, q, n, a, b, c, e = self._coeffs(h, x)
        return (z * v + (a * v) @ self.U_z + (b * v) @ self.U_n
                + (c * v) @ self.U_r)

    def param_vjp(self, h, x, v, t=None):
        """(df/dtheta)^T v summed over leading axes, and (df/dx)^T v per row."""
        z, r, q, n, a, b, c, e = self._coeffs(h, x)
        h2 = h.reshape(-1, self.D)
        x2 = x.reshape(-1, self.Dx)
        dz = (a * v).reshape(-1, self.D)       # d/d(pre-activation of z)
        dn = (e * v).reshape(-1, self.D)       # d/d(pre-activation of n)
        dq = (b * v).reshape(-1, self.D)       # d/dq, q = U_n h + b_hn
        dr = (c * v).reshape(-1, self.D)       # d/d(pre-activation of r)
        g = {
            "W_z": dz.T @ x2, "W_r": dr.T @ x2, "W_n": dn.T @ x2,
            "U_z": dz.T @ h2, "U_r": dr.T @ h2, "U_n": dq.T @ h2,
            "b_z": dz.sum(0), "b_r": dr.sum(0), "b_n": dn.sum(0), "b_hn": dq.sum(0),
        }
        dx = (dz @ self.W_z + dr @ self.W_r + dn @ self.W_n).reshape(x.shape)
        return g, dx

    def pack_grad(self, g):
        return np.concatenate([
            g["W_z"].ravel(), g["W_r"].ravel(), g["W_n"].ravel(),
            g["U_z"].ravel(), g["U_r"].ravel(), g["U_n"].ravel(),
            g["b_z"], g["b_r"], g["b_n"], g["b_hn"]])


class TanhRNN:
    """f(h, x) = tanh(W h + U x + b);  A = diag(1 - f^2) W."""

    name = "tanh"

    def __init__(self, params, D, Dx):
        p = np.asarray(params, dtype=np.float64).ravel()
        assert p.size == tanh_param_count(D, Dx), (p.size, D, Dx)
        self.D, self.Dx = D, Dx
        o = 0
        self.W = p[o:o + D * D].reshape(D, D).copy(); o += D * D
        self.U = p[o:o + D * Dx].reshape(D, Dx).copy(); o += D * Dx
        self.b = p[o:o + D].copy()

    def f(self, h, x, t=None):
        return np.tanh(h @ self.W.T + x @ self.U.T + self.b)

    def jac(self, h, x, t=None):
        d = 1.0 - self.f(h, x) ** 2
        return d[..., :, None] * self.W

    def jac_diag(self, h, x, t=None):
        return (1.0 - self.f(h, x) ** 2) * np.diag(self.W)

    def vjp(self, h, x, v, t=None):
        d = 1.0 - self.f(h, x) ** 2
        return (d * v) @ self.W

    def param_vjp(self, h, x, v, t=None):
        d = 1.0 - self.f(h, x) ** 2
        delta = (d * v).reshape(-1, self.D)
        g = {"W": delta.T @ h.reshape(-1, self.D),
             "U": delta.T @ x.reshape(-1, self.Dx),
             "b": delta.sum(0)}
        dx = (delta @ self.U).reshape(x.shape)
        return g, dx

    def pack_grad(self, g):
        return np.concatenate([g["W"].ravel(), g["U"].ravel(), g["b"]])


class MeanFieldRNN:
    """f(h, x) = W tanh(h) + U x + b;  A = W diag(1 - tanh(h)^2)."""

    name = "meanfield"

    def __init__(self, params, D, Dx):
        p = np.asarray(params, dtype=np.float64).ravel()
        assert p.size == tanh_param_count(D, Dx), (p.size, D, Dx)
        self.D, self.Dx = D, Dx
        o = 0
        self.W = p[o:o + D * D].reshape(D, D).copy(); o += D * D
        self.U = p[o:o + D * Dx].reshape(D, Dx).copy(); o += D * Dx
        self.b = p[o:o + D].copy()

    def f(self, h, x, t=None):
        return np.tanh(h) @ self.W.T + x @ self.U.T + self.b

    def jac(self, h, x, t=None):
        d = 1.0 - np.tanh(h) ** 2
        return self.W * d[..., None, :]

    def jac_diag(self, h, x, t=None):
        return np.diag(self.W) * (1.0 - np.tanh(h) ** 2)

    def vjp(self, h, x, v, t=None):
        return (v @ self.W) * (1.0 - np.tanh(h) ** 2)


class Affine:
    """f(h, x) = M h + N x + c: a linear dynamical system (eq. lds).

    ``M_steps`` (shape [T, D, D]) optionally replaces M with a per-step matrix M_t, which
    is how the S5 permutation LDS of Ch. 6 is expressed; then f needs the step index.
    """

    name = "affine"

    def __init__(self, params, D, Dx, M_steps=None):
        p = np.asarray(params, dtype=np.float64).ravel()
        assert p.size == affine_param_count(D, Dx), (p.size, D, Dx)
        self.D, self.Dx = D, Dx
        o = 0
        self.M = p[o:o + D * D].reshape(D, D).copy(); o += D * D
        self.N = p[o:o + D * Dx].reshape(D, Dx).copy(); o += D * Dx
        self.c = p[o:o + D].copy()
        self.M_steps = None if M_steps is None else np.asarray(M_steps, np.float64)

    def _Mt(self, t, lead):
        """M_t for a scalar step index or an array of indices aligned with ``lead``."""
        if self.M_steps is None or t is None:
            return np.broadcast_to(self.M, lead + (self.D, self.D))
        return np.broadcast_to(self.M_steps[t], lead + (self.D, self.D))

    def f(self, h, x, t=None):
        M = self._Mt(t, h.shape[:-1])
        return np.einsum("...ij,...j->...i", M, h) + x @ self.N.T + self.c

    def jac(self, h, x, t=None):
        return self._Mt(t, h.shape[:-1]).copy()

    def jac_diag(self, h, x, t=None):
        return np.diagonal(self._Mt(t, h.shape[:-1]), axis1=-2, axis2=-1).copy()

    def vjp(self, h, x, v, t=None):
        return np.einsum("...ij,...i->...j", self._Mt(t, h.shape[:-1]), v)


def make_cell(kind, params, D, Dx, **kw):
    if kind == "gru":
        return GRU(params, D, Dx)
    if kind == "tanh":
        return TanhRNN(params, D, Dx)
    if kind == "meanfield":
        return MeanFieldRNN(params, D, Dx)
    if kind == "affine":
        return Affine(params, D, Dx, **kw)
    raise ValueError(kind)
