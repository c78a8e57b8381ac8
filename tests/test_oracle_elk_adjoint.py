"""Pins of the oracle's ELK filter, adjoint and LLE estimator (no GPU)."""
import numpy as np
import pytest
import torch

from oracle import adjoint, cells, dense, elk, lle, newton, rollout
from paper_2603_16850_amd import workloads

torch.set_default_dtype(torch.float64)


def _tanh(rng, D, Dx, g, bias=0.1):
    p = np.concatenate([rng.normal(0, g / np.sqrt(D), size=D * D),
                        rng.normal(0, 1 / np.sqrt(D), size=D * Dx),
                        rng.normal(0, bias, size=D)])
    return cells.TanhRNN(p, D, Dx)


def _gru(rng, D, Dx):
    return cells.GRU(rng.normal(0, 1 / np.sqrt(D), size=cells.gru_param_count(D, Dx)), D, Dx)


def _rand_At_r(rng, T, D, scale=1.3):
    return rng.normal(size=(T, D, D)) * scale / np.sqrt(D), rng.normal(size=(T, D))


# ---- ELK ---------------------------------------------------------------------------------

def test_elk_lambda_zero_is_deer_step():
    rng = np.random.default_rng(20)
    At, r = _rand_At_r(rng, 30, 4)
    d, _, _ = elk.filter_step(At, r, 0.0)
    np.testing.assert_allclose(d, newton.forward_substitution(At, r), rtol=0, atol=1e-12)


def test_elk_large_lambda_gives_small_step():
    rng = np.random.default_rng(21)
    At, r = _rand_At_r(rng, 30, 4)
    d, _, _ = elk.filter_step(At, r, 1e9)
    assert np.abs(d).max() < 1e-7 * np.abs(r).max() * 10


@pytest.mark.parametrize("lam", [1e-2, 0.3, 1.0, 10.0])
def test_elk_filter_is_prefix_lm_solution(lam):
    """Filtered mean at t = last block of the LM step on the prefix 1..t (Prop. prop:ELK)."""
    rng = np.random.default_rng(22)
    T, D = 8, 3
    At, r = _rand_At_r(rng, T, D)
    d, _, _ = elk.filter_step(At, r, lam)
    for t in range(1, T + 1):
        lm = dense.lm_step_dense(At[:t], r[:t], lam)
        np.testing.assert_allclose(d[t - 1], lm[-1], rtol=0, atol=1e-12)


@pytest.mark.parametrize("lam", [0.0, 1e-2, 1.0])
def test_elk_scan_elements_reproduce_filter(lam):
    rng = np.random.default_rng(23)
    At, r = _rand_At_r(rng, 12, 3)
    d, P, _ = elk.filter_step(At, r, lam)
    d2, P2 = elk.filter_by_elements(At, r, lam)
    np.testing.assert_allclose(d2, d, rtol=0, atol=1e-12)
    np.testing.assert_allclose(P2, P, rtol=1e-12, atol=1e-12)


def test_elk_combine_is_associative():
    rng = np.random.default_rng(24)
    D, lam = 3, 0.4
    At, r = _rand_At_r(rng, 6, D)
    leaves = [elk.kalman_leaf(At[t], r[t], lam, first=(t == 0)) for t in range(6)]
    left = elk.kalman_combine(elk.kalman_combine(leaves[1], leaves[2]), leaves[3])
    right = elk.kalman_combine(leaves[1], elk.kalman_combine(leaves[2], leaves[3]))
    for a, b in zip(left, right):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    allb = dense.all_bracketings(leaves, elk.kalman_combine)
    for e in allb:
        np.testing.assert_allclose(e[1], allb[0][1], rtol=0, atol=1e-11)


@pytest.mark.parametrize("lam", [1e-2, 1.0, 5.0])
def test_elk_attenuation_bound(lam):
    """Gamma_t is SPD with eigenvalues in (0, 1/(1+lam)]; ||Gamma_t A_t|| <= ||A_t||/(1+lam)."""
    rng = np.random.default_rng(25)
    At, r = _rand_At_r(rng, 20, 4, scale=2.0)
    _, _, G = elk.filter_step(At, r, lam)
    for t in range(20):
        ev = np.linalg.eigvals(G[t]).real
        assert ev.min() > 0 and ev.max() <= 1 / (1 + lam) + 1e-12
        if t > 0:
            assert (np.linalg.norm(G[t] @ At[t], 2)
                    <= np.linalg.norm(At[t], 2) / (1 + lam) + 1e-12)


def test_elk_preserves_converged_prefix():
    rng = np.random.default_rng(26)
    At, r = _rand_At_r(rng, 15, 3)
    r[:6] = 0.0
    d, _, _ = elk.filter_step(At, r, 0.5)
    assert np.all(d[:6] == 0.0)


def test_elk_loop_reaches_rollout():
    rng = np.random.default_rng(27)
    cell = _tanh(rng, 4, 2, g=1.5)
    x = rng.normal(size=(60, 2))
    s0 = np.zeros(4)
    ref = rollout.rollout(cell, x, s0)
    for lam in [1e-2, 1.0]:
        out = elk.elk(cell, x, s0, lam, tol=1e-12, max_iters=2000)
        assert out["converged"]
        np.testing.assert_allclose(out["s"], ref, rtol=0, atol=1e-11)


# ---- adjoint -----------------------------------------------------------------------------

def _torch_loss_and_grads(kind, p, D, Dx, x, s0, offsets):
    """sum_t ||s_t||^2 through a plain torch loop; gradients by torch.autograd (FP64 CPU)."""
    pt = torch.tensor(p, requires_grad=True)
    xt = torch.tensor(x, requires_grad=True)
    s0t = torch.tensor(s0, requires_grad=True)
    if kind == "gru":
        o = 0
        W = pt[o:o + 3 * D * Dx].reshape(3 * D, Dx); o += 3 * D * Dx
        U = pt[o:o + 3 * D * D].reshape(3 * D, D); o += 3 * D * D
        b = pt[o:o + 3 * D]; o += 3 * D
        bhn = pt[o:o + D]

        def f(h, xx):
            gi = xx @ W.T + b
            gh = h @ U.T
            z = torch.sigmoid(gi[:D] + gh[:D])
            r = torch.sigmoid(gi[D:2 * D] + gh[D:2 * D])
            n = torch.tanh(gi[2 * D:] + r * (gh[2 * D:] + bhn))
            return (1 - z) * n + z * h
    else:
        W = pt[:D * D].reshape(D, D)
        U = pt[D * D:D * D + D * Dx].reshape(D, Dx)
        b = pt[D * D + D * Dx:]

        def f(h, xx):
            return torch.tanh(W @ h + U @ xx + b)
    loss = 0
    for bb in range(len(offsets) - 1):
        h = s0t[bb]
        for n in range(offsets[bb], offsets[bb + 1]):
            h = f(h, xt[n])
            loss = loss + (h * h).sum()
    loss.backward()
    return pt.grad.numpy(), xt.grad.numpy(), s0t.grad.numpy()


@pytest.mark.parametrize("kind", ["gru", "tanh"])
def test_adjoint_matches_torch_autograd(kind):
    rng = np.random.default_rng(28)
    D, Dx = 4, 3
    lens = np.array([9, 1, 14])
    offsets = np.concatenate([[0], np.cumsum(lens)])
    if kind == "gru":
        cell = _gru(rng, D, Dx)
        p = cell.pack_grad({"W_z": cell.W_z, "W_r": cell.W_r, "W_n": cell.W_n,
                            "U_z": cell.U_z, "U_r": cell.U_r, "U_n": cell.U_n,
                            "b_z": cell.b_z, "b_r": cell.b_r, "b_n": cell.b_n,
                            "b_hn": cell.b_hn})
    else:
        cell = _tanh(rng, D, Dx, g=0.9)
        p = np.concatenate([cell.W.ravel(), cell.U.ravel(), cell.b])
    x = rng.normal(size=(offsets[-1], Dx))
    s0 = rng.normal(size=(3, D)) * 0.3
    s = rollout.rollout_batch(cell, x, s0, offsets)
    lam, gp, gx, gs0 = adjoint.adjoint_batch(cell, x, s0, s, 2 * s, offsets)
    tp, tx, ts0 = _torch_loss_and_grads(kind, p, D, Dx, x, s0, offsets)
    np.testing.assert_allclose(gp, tp, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gx, tx, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gs0, ts0, rtol=0, atol=1e-12)
    # per-sequence form agrees with the batched one
    for bb in range(3):
        a, e = offsets[bb], offsets[bb + 1]
        l1, g1, x1, s01 = adjoint.adjoint(cell, x[a:e], s0[bb], s[a:e], 2 * s[a:e])
        np.testing.assert_allclose(l1, lam[a:e], atol=1e-13)
        np.testing.assert_allclose(s01, gs0[bb], atol=1e-13)
        rho = adjoint.adjoint_residual(cell, x[a:e], s0[bb], s[a:e], 2 * s[a:e], l1)
        assert np.abs(rho).max() < 1e-13


def test_adjoint_matches_finite_differences():
    rng = np.random.default_rng(29)
    D, Dx, T = 5, 3, 30
    p = rng.normal(0, 1 / np.sqrt(D), size=cells.gru_param_count(D, Dx))
    x = rng.normal(size=(T, Dx))
    s0 = np.zeros(D)

    def loss(pp):
        c = cells.GRU(pp, D, Dx)
        s = rollout.rollout(c, x, s0)
        return float((s * s).sum())

    cell = cells.GRU(p, D, Dx)
    s = rollout.rollout(cell, x, s0)
    _, gp, _, _ = adjoint.adjoint(cell, x, s0, s, 2 * s)
    for _ in range(3):
        v = rng.normal(size=p.size)
        h = 1e-6
        fd = (loss(p + h * v) - loss(p - h * v)) / (2 * h)
        assert abs(fd - gp @ v) < 1e-7 * max(1.0, abs(fd))


# ---- LLE -----------------------------------------------------------------------------------

def test_lle_of_logistic_map_is_ln2():
    """x <- 4 x (1 - x) has Lyapunov exponent ln 2 (a textbook closed form)."""
    xs = np.empty(200000)
    v = 0.1234567
    for t in range(xs.size):
        xs[t] = v
        v = 4 * v * (1 - v)
    jac = (4 - 8 * xs).reshape(-1, 1, 1)
    est = lle.lle_estimate(jac, np.ones(1))
    assert abs(est - np.log(2)) < 1e-2


def test_lle_of_constant_linear_map():
    a = np.diag([0.3, -0.9, 0.5])
    J = np.broadcast_to(a, (500, 3, 3))
    est = lle.lle_average(J, n_vectors=3, seed=1)
    assert abs(est - np.log(0.9)) < 1e-2


def test_predictable_workload_has_negative_lle():
    """The g = 0.9 tanh workload is in the predictable regime (Def. def:predictable_systems)."""
    w = workloads.ALL["tanh32-dense-bf16"].scaled(T=3000, B=1)
    inst = workloads.make_instance(w, seed=0)
    cell = cells.make_cell(w.cell, inst.params, w.D, w.Dx)
    s = rollout.rollout(cell, inst.x, inst.s0[0])
    assert lle.trajectory_lle(cell, inst.x, inst.s0[0], s) < 0


def test_mean_field_rnn_lle_grows_with_gain():
    """Ch. 5 mean-field RNN s' = W tanh(s) + u, W ~ N(0, g^2/D), no self-coupling, D = 100,
    mild sinusoidal input: the LLE rises with g from predictable to chaotic."""
    D, T = 100, 2500
    est = []
    for g in (0.5, 1.0, 2.0):
        rng = np.random.default_rng(0)
        W = rng.normal(0, g / np.sqrt(D), size=(D, D))
        np.fill_diagonal(W, 0.0)
        s = rng.normal(size=D)
        J = []
        for t in range(T):
            J.append(W * (1 - np.tanh(s) ** 2)[None, :])
            s = W @ np.tanh(s) + 0.1 * np.sin(0.05 * t + np.arange(D))
        est.append(lle.lle_average(J[500:]))
    assert est[0] < -0.3 and est[2] > 0.03 and est[0] < est[1] < est[2], est
