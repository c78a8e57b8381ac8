"""Pins of the oracle's cells against independent references (no GPU).

* f of the GRU equals torch.nn.GRUCell (PyTorch's GRU is the same reset-after cell), and
  f of the tanh-RNN equals torch.nn.RNNCell -- library routines, not a retyped formula.
* A_t, diag(A_t), A_t^T v and (df/dtheta)^T v equal torch.autograd in float64 and central
  finite differences.
"""
import numpy as np
import pytest
import torch

from oracle import cells

torch.set_default_dtype(torch.float64)


def _rand_gru(rng, D, Dx, bias=True):
    p = rng.normal(0, 1.0 / np.sqrt(D), size=cells.gru_param_count(D, Dx))
    if not bias:
        p[-4 * D:] = 0
    return p


def _rand_tanh(rng, D, Dx):
    return rng.normal(0, 1.0 / np.sqrt(D), size=cells.tanh_param_count(D, Dx))


def _torch_gru(cell):
    m = torch.nn.GRUCell(cell.Dx, cell.D).double()
    with torch.no_grad():
        # PyTorch stacks gates as (r, z, n); the oracle packs (z, r, n)
        m.weight_ih.copy_(torch.tensor(np.concatenate([cell.W_r, cell.W_z, cell.W_n])))
        m.weight_hh.copy_(torch.tensor(np.concatenate([cell.U_r, cell.U_z, cell.U_n])))
        m.bias_ih.copy_(torch.tensor(np.concatenate([cell.b_r, cell.b_z, cell.b_n])))
        m.bias_hh.copy_(torch.tensor(np.concatenate([np.zeros(cell.D), np.zeros(cell.D),
                                                     cell.b_hn])))
    return m


def _torch_tanh(cell):
    m = torch.nn.RNNCell(cell.Dx, cell.D, nonlinearity="tanh").double()
    with torch.no_grad():
        m.weight_ih.copy_(torch.tensor(cell.U))
        m.weight_hh.copy_(torch.tensor(cell.W))
        m.bias_ih.copy_(torch.tensor(cell.b))
        m.bias_hh.zero_()
    return m


@pytest.mark.parametrize("D,Dx", [(4, 4), (7, 3), (16, 8)])
def test_gru_matches_torch_grucell(D, Dx):
    rng = np.random.default_rng(1)
    cell = cells.GRU(_rand_gru(rng, D, Dx), D, Dx)
    h = rng.normal(size=(5, D))
    x = rng.normal(size=(5, Dx))
    ref = _torch_gru(cell)(torch.tensor(x), torch.tensor(h)).detach().numpy()
    np.testing.assert_allclose(cell.f(h, x), ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("D,Dx", [(4, 4), (16, 16)])
def test_tanh_matches_torch_rnncell(D, Dx):
    rng = np.random.default_rng(2)
    cell = cells.TanhRNN(_rand_tanh(rng, D, Dx), D, Dx)
    h = rng.normal(size=(5, D))
    x = rng.normal(size=(5, Dx))
    ref = _torch_tanh(cell)(torch.tensor(x), torch.tensor(h)).detach().numpy()
    np.testing.assert_allclose(cell.f(h, x), ref, rtol=0, atol=1e-14)


def _cases():
    rng = np.random.default_rng(3)
    out = []
    for D, Dx in [(4, 4), (6, 3)]:
        out.append(cells.GRU(_rand_gru(rng, D, Dx), D, Dx))
        out.append(cells.TanhRNN(_rand_tanh(rng, D, Dx), D, Dx))
        out.append(cells.Affine(rng.normal(size=cells.affine_param_count(D, Dx)), D, Dx))
    return out


@pytest.mark.parametrize("cell", _cases(), ids=lambda c: f"{c.name}{c.D}x{c.Dx}")
def test_jacobian_vs_autograd_and_fd(cell):
    rng = np.random.default_rng(4)
    h = rng.normal(size=cell.D)
    x = rng.normal(size=cell.Dx)
    A = cell.jac(h, x)
    ref = torch.autograd.functional.jacobian(
        lambda hh: torch.tensor(0.0) + _torch_f(cell, hh, torch.tensor(x)), torch.tensor(h))
    np.testing.assert_allclose(A, ref.numpy(), rtol=0, atol=1e-13)
    eps = 1e-6
    fd = np.stack([(cell.f(h + eps * e, x) - cell.f(h - eps * e, x)) / (2 * eps)
                   for e in np.eye(cell.D)], axis=1)
    np.testing.assert_allclose(A, fd, rtol=0, atol=1e-8)
    np.testing.assert_allclose(cell.jac_diag(h, x), np.diag(ref.numpy()), rtol=0, atol=1e-13)
    v = rng.normal(size=cell.D)
    np.testing.assert_allclose(cell.vjp(h, x, v), ref.numpy().T @ v, rtol=0, atol=1e-13)


def _torch_f(cell, h, x):
    if cell.name == "gru":
        return _torch_gru(cell)(x[None], h[None])[0]
    if cell.name == "tanh":
        return _torch_tanh(cell)(x[None], h[None])[0]
    return torch.tensor(cell.M) @ h + torch.tensor(cell.N) @ x + torch.tensor(cell.c)


@pytest.mark.parametrize("kind", ["gru", "tanh"])
def test_param_vjp_vs_autograd(kind):
    rng = np.random.default_rng(5)
    D, Dx, n = 5, 3, 7
    p = _rand_gru(rng, D, Dx) if kind == "gru" else _rand_tanh(rng, D, Dx)
    cell = cells.make_cell(kind, p, D, Dx)
    h = rng.normal(size=(n, D))
    x = rng.normal(size=(n, Dx))
    v = rng.normal(size=(n, D))
    g, dx = cell.param_vjp(h, x, v)
    got = cell.pack_grad(g)

    pt = torch.tensor(p, requires_grad=True)
    xt = torch.tensor(x, requires_grad=True)

    def f_of(pp, xx):
        c2 = cells.make_cell(kind, pp.detach().numpy(), D, Dx)
        return _torch_f_params(kind, pp, D, Dx, torch.tensor(h), xx)

    out = f_of(pt, xt)
    (out * torch.tensor(v)).sum().backward()
    np.testing.assert_allclose(got, pt.grad.numpy(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=0, atol=1e-12)


def _torch_f_params(kind, p, D, Dx, h, x):
    """f written with torch ops from the packed vector (independent of the numpy cells)."""
    if kind == "gru":
        o = 0
        W = p[o:o + 3 * D * Dx].reshape(3 * D, Dx); o += 3 * D * Dx
        U = p[o:o + 3 * D * D].reshape(3 * D, D); o += 3 * D * D
        b = p[o:o + 3 * D]; o += 3 * D
        bhn = p[o:o + D]
        gi = x @ W.T + b
        gh = h @ U.T
        z = torch.sigmoid(gi[:, :D] + gh[:, :D])
        r = torch.sigmoid(gi[:, D:2 * D] + gh[:, D:2 * D])
        n = torch.tanh(gi[:, 2 * D:] + r * (gh[:, 2 * D:] + bhn))
        return (1 - z) * n + z * h
    o = 0
    W = p[o:o + D * D].reshape(D, D); o += D * D
    U = p[o:o + D * Dx].reshape(D, Dx); o += D * Dx
    b = p[o:o + D]
    return torch.tanh(h @ W.T + x @ U.T + b)


def test_affine_per_step_matrices():
    rng = np.random.default_rng(6)
    D, Dx, T = 3, 2, 4
    Ms = rng.normal(size=(T, D, D))
    cell = cells.Affine(rng.normal(size=cells.affine_param_count(D, Dx)), D, Dx, M_steps=Ms)
    h = rng.normal(size=(T, D))
    x = rng.normal(size=(T, Dx))
    tt = np.arange(T)
    want = np.stack([Ms[t] @ h[t] + cell.N @ x[t] + cell.c for t in range(T)])
    np.testing.assert_allclose(cell.f(h, x, t=tt), want, atol=1e-14)
    np.testing.assert_allclose(cell.jac(h, x, t=tt), Ms, atol=0)
