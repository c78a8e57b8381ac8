"""Oracle pins for the ELK smoother (the exact Levenberg-Marquardt step of Prop. ELK).

The RTS-based step is checked against the step's definition, -(J^T J + lambda I)^-1 J^T r
solved densely with the block-bidiagonal Jacobian; against its lambda = 0 limit (the DEER
step, forward substitution) and its large-lambda limit (gradient descent with step
1/lambda: lambda Delta -> -J^T r); and the smoothed and filtered means agree at the last
step (nothing observed after it).
"""
import numpy as np
import pytest

from oracle import cells, elk, newton, rollout
from paper_2603_16850_amd import workloads


def _random_problem(rng, T=7, D=3, rho=1.3):
    At = rng.standard_normal((T, D, D))
    At *= rho / np.abs(np.linalg.eigvals(At)).max(axis=1)[:, None, None]
    r = rng.standard_normal((T, D))
    return At, r


@pytest.mark.parametrize("lam", [1e-3, 0.1, 1.0, 10.0])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_smoother_is_the_lm_step(lam, seed):
    At, r = _random_problem(np.random.default_rng(seed))
    np.testing.assert_allclose(elk.smoother_step(At, r, lam), elk.lm_step_dense(At, r, lam),
                               rtol=0, atol=1e-10)


def test_smoother_on_tanh_jacobians():
    w = workloads.TANH16_ELK.scaled(B=1, T=12)
    inst = workloads.make_instance(w, seed=3)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    s = 0.3 * np.random.default_rng(4).standard_normal((12, w.D))
    h, r = newton.linearize(cell, inst.x, inst.s0[0], s)
    for mode in ("dense", "diag"):
        At = newton.transition_matrices(cell, inst.x, h, mode)
        for lam in (0.01, 1.0):
            np.testing.assert_allclose(elk.smoother_step(At, r, lam),
                                       elk.lm_step_dense(At, r, lam), rtol=0, atol=1e-10)


def test_smoother_limits():
    At, r = _random_problem(np.random.default_rng(5), T=9, D=4)
    # lambda = 0: the Gauss-Newton (DEER) step
    np.testing.assert_allclose(elk.smoother_step(At, r, 0.0),
                               newton.forward_substitution(At, r), rtol=0, atol=1e-9)
    # large lambda: lambda Delta -> -J^T r
    T, D = r.shape
    g = r.copy()
    for t in range(T - 1):
        g[t] -= At[t + 1].T @ r[t + 1]
    lam = 1e7
    np.testing.assert_allclose(lam * elk.smoother_step(At, r, lam), -g, rtol=0, atol=1e-4)
    # the last smoothed mean is the last filtered mean
    for lam in (0.05, 2.0):
        assert np.allclose(elk.smoother_step(At, r, lam)[-1], elk.filter_step(At, r, lam)[0][-1],
                           rtol=0, atol=1e-12)


def test_smoother_loop_converges_to_rollout():
    """On a contracting instance (gain 0.9) the smoothed-step loop reaches the rollout; it
    takes more iterations than the filtered step (the causal argument of Ch. 4)."""
    w = workloads.TANH16_ELK.scaled(B=1, T=200, gain=0.9)
    inst = workloads.make_instance(w, seed=6)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    ref = rollout.rollout(cell, inst.x, inst.s0[0])
    for lam in (0.01, 0.3):
        out = elk.elk(cell, inst.x, inst.s0[0], lam, smoother=True, tol=1e-9, max_iters=500)
        filt = elk.elk(cell, inst.x, inst.s0[0], lam, tol=1e-9, max_iters=500)
        assert out["converged"], out["iters"]
        assert np.abs(out["s"] - ref).max() < 1e-8
        assert out["iters"] >= filt["iters"]
