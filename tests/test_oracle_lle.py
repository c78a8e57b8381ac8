"""Pins of the LLE estimate (Alg. LLE_estimate) and of the mean-field RNN cell.

Closed forms: a constant Jacobian gives the log spectral radius (power iteration); a
scalar linear map s -> a s gives log|a|.  The mean-field cell's Jacobian is checked by
central differences, its diagonal against the dense one.
"""
import numpy as np
import pytest

from oracle import cells, lle, rollout


def test_constant_jacobian_gives_log_spectral_radius():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((5, 5))
    ev = np.linalg.eigvals(M)
    rho = np.abs(ev).max()
    # keep a real, strictly dominant eigenvalue so the power iteration settles
    M = M + (2.0 * rho) * np.outer(np.ones(5), np.ones(5)) / 5
    rho = np.abs(np.linalg.eigvals(M)).max()
    est = lle.lle_estimate(np.broadcast_to(M, (4000, 5, 5)), rng.standard_normal(5))
    assert abs(est - np.log(rho)) < 2e-3


@pytest.mark.parametrize("a", [0.5, -1.7, 1.0])
def test_scalar_linear_map(a):
    J = np.full((100, 1, 1), a)
    assert abs(lle.lle_estimate(J, [1.0]) - np.log(abs(a))) < 1e-14


def _meanfield(D=6, Dx=6, seed=1, g=1.5):
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((D, D)) * g / np.sqrt(D)
    np.fill_diagonal(W, 0.0)
    p = np.concatenate([W.ravel(), np.eye(D, Dx).ravel(), 0.1 * rng.standard_normal(D)])
    return cells.MeanFieldRNN(p, D, Dx), rng


def test_meanfield_jacobian_by_differences():
    cell, rng = _meanfield()
    h, x = rng.standard_normal((3, 6)), rng.standard_normal((3, 6))
    J = cell.jac(h, x)
    eps = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = eps
        fd = (cell.f(h + e, x) - cell.f(h - e, x)) / (2 * eps)
        np.testing.assert_allclose(J[:, :, j], fd, rtol=0, atol=1e-8)
    np.testing.assert_allclose(cell.jac_diag(h, x), np.diagonal(J, axis1=1, axis2=2), atol=1e-15)
    v = rng.standard_normal((3, 6))
    np.testing.assert_allclose(cell.vjp(h, x, v), np.einsum("tij,ti->tj", J, v), atol=1e-14)


def test_meanfield_lle_grows_with_gain():
    """The gain g orders the LLE (the monotone relation the sweep relies on): a small gain
    contracts (negative LLE), a large one is chaotic (positive)."""
    out = []
    for g in (0.5, 3.0):
        cell, rng = _meanfield(D=16, Dx=16, seed=2, g=g)
        T = 3000
        x = 0.1 * np.sin(0.05 * np.arange(T)[:, None] + np.arange(16)[None, :])
        s0 = rng.standard_normal(16)
        s = rollout.rollout(cell, x, s0)
        out.append(lle.lle_estimate(lle.trajectory_jacobians(cell, x, s0, s),
                                    rng.standard_normal(16)))
    assert out[0] < 0 < out[1], out


def test_meanfield_rollout_is_rnncell_in_tanh_coordinates():
    """Ch. 5 defines the mean-field RNN by s_{t+1} = W tanh(s_t) + u_t (u_t = U x + b here).
    With h_t = tanh(s_t) the same recurrence reads h_{t+1} = tanh(W h_t + u_t): a tanh RNN,
    which torch.nn.RNNCell (h' = tanh(x W_ih^T + b_ih + h W_hh^T + b_hh)) evaluates
    independently of the oracle.  A transposed W, or tanh applied after the coupling (which
    would make s itself bounded by 1), fails this check."""
    import torch

    D, Dx, T = 7, 5, 60
    rng = np.random.default_rng(3)
    W = rng.standard_normal((D, D)) * 1.3 / np.sqrt(D)
    np.fill_diagonal(W, 0.0)
    U = rng.standard_normal((D, Dx))
    b = 0.2 * rng.standard_normal(D)
    W[0, 1], W[1, 0] = 0.9, -0.4          # clearly non-symmetric
    cell = cells.MeanFieldRNN(np.concatenate([W.ravel(), U.ravel(), b]), D, Dx)
    x = rng.standard_normal((T, Dx))
    s0 = 1.5 * rng.standard_normal(D)
    s = rollout.rollout(cell, x, s0)
    assert np.abs(s).max() > 1.0           # the state is a current, not a bounded rate

    m = torch.nn.RNNCell(Dx, D, nonlinearity="tanh").double()
    with torch.no_grad():
        m.weight_hh.copy_(torch.tensor(W))
        m.weight_ih.copy_(torch.tensor(U))
        m.bias_ih.copy_(torch.tensor(b))
        m.bias_hh.zero_()
        h = torch.tanh(torch.tensor(s0))[None]
        hs = []
        for t in range(T):
            h = m(torch.tensor(x[t])[None], h)
            hs.append(h[0].numpy().copy())
    np.testing.assert_allclose(np.tanh(s), np.array(hs), rtol=0, atol=1e-13)
    # and the state itself: s_t = W h_{t-1} + U x_t + b with the library's h
    hprev = np.concatenate([np.tanh(s0)[None], np.array(hs)[:-1]])
    np.testing.assert_allclose(s, hprev @ W.T + x @ U.T + b, rtol=0, atol=1e-13)


def test_chaotic_elk_workload_has_positive_lle():
    """The chaotic ELK workload (gain 1.5, inputs scaled by 0.1, its stated seed) is chaotic:
    a positive largest Lyapunov exponent on its sequences (checked on two of them)."""
    from paper_2603_16850_amd import workloads
    w = workloads.TANH16_ELK_CHAOTIC
    inst = workloads.make_instance(w, seed=workloads.CHAOTIC_SEED)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    for b in (0, 7):
        a, e = inst.offsets[b], inst.offsets[b + 1]
        s = rollout.rollout(cell, inst.x[a:e], inst.s0[b])
        assert lle.trajectory_lle(cell, inst.x[a:e], inst.s0[b], s) > 0.01, b
