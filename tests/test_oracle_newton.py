"""Pins of the oracle's rollout and Newton loop against what the thesis fixes (no GPU)."""
import json
import os

import numpy as np
import pytest

from oracle import cells, dense, newton, rollout

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _gru(rng, D, Dx, scale=1.0):
    return cells.GRU(rng.normal(0, scale / np.sqrt(D), size=cells.gru_param_count(D, Dx)), D, Dx)


def _tanh(rng, D, Dx, g):
    p = np.concatenate([rng.normal(0, g / np.sqrt(D), size=D * D),
                        rng.normal(0, 1 / np.sqrt(D), size=D * Dx), rng.normal(0, 0.1, size=D)])
    return cells.TanhRNN(p, D, Dx)


def _scalar_affine(a, c=0.0):
    """f(s) = a s + c on a 1-D state with a 1-D (unused) input."""
    return cells.Affine(np.array([a, 0.0, c]), 1, 1)


# ---- the answer is the sequential rollout (eq. r_def: s* is the unique zero of r) -------

@pytest.mark.parametrize("mode", ["dense", "diag"])
def test_fixed_point_is_rollout(mode):
    rng = np.random.default_rng(10)
    cell = _gru(rng, 6, 3)
    x = rng.normal(size=(200, 3))
    s0 = rng.normal(size=6) * 0.3
    ref = rollout.rollout(cell, x, s0)
    out = newton.newton(cell, x, s0, mode=mode, tol=1e-13)
    assert out["converged"]
    np.testing.assert_allclose(out["s"], ref, rtol=0, atol=1e-12)


def test_rollout_batch_matches_per_sequence():
    rng = np.random.default_rng(11)
    cell = _gru(rng, 5, 2)
    lens = np.array([7, 1, 13, 0, 4])
    offsets = np.concatenate([[0], np.cumsum(lens)])
    x = rng.normal(size=(offsets[-1], 2))
    s0 = rng.normal(size=(5, 5))
    s = rollout.rollout_batch(cell, x, s0, offsets)
    for b in range(5):
        a, e = offsets[b], offsets[b + 1]
        np.testing.assert_allclose(s[a:e], rollout.rollout(cell, x[a:e], s0[b]), atol=0)


# ---- one-iteration properties (linear f: Lipschitz constant of J is zero) -------------

def test_affine_dense_converges_in_one_iteration():
    rng = np.random.default_rng(12)
    D, Dx, T = 5, 3, 64
    cell = cells.Affine(rng.normal(size=cells.affine_param_count(D, Dx)) * 0.4, D, Dx)
    x = rng.normal(size=(T, Dx))
    out = newton.newton(cell, x, rng.normal(size=D), mode="dense", tol=1e-12, reset_abs=np.inf)
    assert out["converged"] and out["iters"] == 1


def test_permutation_lds_converges_in_one_iteration():
    """S5 word problem (Ch. 6): per-step permutation matrices; Newton needs one iteration."""
    rng = np.random.default_rng(13)
    D, T = 5, 128
    Ms = np.stack([np.eye(D)[rng.permutation(D)] for _ in range(T)])
    cell = cells.Affine(np.zeros(cells.affine_param_count(D, 1)), D, 1, M_steps=Ms)
    s0 = np.eye(D)[0]
    out = newton.newton(cell, np.zeros((T, 1)), s0, mode="dense", tol=1e-12)
    assert out["converged"] and out["iters"] == 1
    ref = rollout.rollout(cell, np.zeros((T, 1)), s0)
    np.testing.assert_allclose(out["s"], ref, atol=1e-12)
    # quasi-DEER (diag) needs many more: a permutation has a mostly-zero diagonal
    slow = newton.newton(cell, np.zeros((T, 1)), s0, mode="diag", tol=1e-12)
    assert slow["converged"] and slow["iters"] > 10


def test_diagonal_affine_converges_in_one_quasi_iteration():
    rng = np.random.default_rng(14)
    D, Dx, T = 4, 2, 50
    p = np.concatenate([np.diag(rng.uniform(-1.2, 1.2, size=D)).ravel(),
                        rng.normal(size=D * Dx), rng.normal(size=D)])
    cell = cells.Affine(p, D, Dx)
    out = newton.newton(cell, rng.normal(size=(T, Dx)), rng.normal(size=D), mode="diag",
                        tol=1e-9, reset_abs=np.inf)
    assert out["converged"] and out["iters"] == 1


# ---- global convergence in <= T iterations, prefix exactness (Prop. global_convergence) --

@pytest.mark.parametrize("mode", ["dense", "diag", "picard", "jacobi", "clip", "scale:0.5",
                                  "diagscale:0.3", "clip:-0.5:0.8"])
@pytest.mark.parametrize("kind", ["gru", "chaotic_tanh"])
def test_at_most_T_iterations_and_prefix(mode, kind):
    rng = np.random.default_rng(15)
    T = 24
    cell = _gru(rng, 4, 2, scale=2.0) if kind == "gru" else _tanh(rng, 4, 2, g=2.5)
    x = rng.normal(size=(T, cell.Dx))
    s0 = rng.normal(size=4)
    ref = rollout.rollout(cell, x, s0)
    out = newton.newton(cell, x, s0, mode=mode, tol=1e-11, history=True, reset_abs=np.inf)
    assert out["converged"] and out["iters"] <= T
    for i, it in enumerate(out["history"]):
        if i == 0:
            continue
        np.testing.assert_allclose(it[:i], ref[:i], rtol=0, atol=1e-12)


def test_worked_doubling_example():
    g = _gold("worked_doubling.json")
    cell = _scalar_affine(g["f_scale"])
    x = np.zeros((2, 1))
    init = np.array(g["init"])[:, None]
    for mode, key in [("dense", "deer_iterates"), ("jacobi", "jacobi_iterates"),
                      ("picard", "picard_iterates")]:
        out = newton.newton(cell, x, np.array([g["s0"]]), s_init=init, mode=mode, tol=1e-14,
                            history=True, reset_abs=np.inf)
        got = [h[:, 0].tolist() for h in out["history"][1:]]
        assert got == g[key], (mode, got)
        assert out["s"][:, 0].tolist() == g["true"]


def test_tang_counterexample_needs_lower_triangular_update():
    """A non-lower-triangular G in s <- s - G r does not converge in T steps (Appendix)."""
    g = _gold("worked_doubling.json")
    cell = _scalar_affine(g["f_scale"])
    s = np.array(g["init"])[:, None]
    x = np.zeros((2, 1))
    seen = []
    for _ in range(2):
        _, r = newton.linearize(cell, x, np.array([g["s0"]]), s)
        G = np.eye(2) if np.all(r == 0) else np.array([[1.0, 1.0], [0.0, 1.0]])
        s = s - (G @ r[:, 0])[:, None]
        seen.append(s[:, 0].tolist())
    assert seen == g["tang_G_iterates"]


# ---- the scan equals the dense solve; J^{-1} blocks are Jacobian products ---------------

def test_forward_substitution_equals_dense_solve():
    rng = np.random.default_rng(16)
    T, D = 8, 3
    At = rng.normal(size=(T, D, D))
    r = rng.normal(size=(T, D))
    np.testing.assert_allclose(newton.forward_substitution(At, r),
                               dense.newton_step_dense(At, r), rtol=0, atol=1e-11)
    np.testing.assert_allclose(dense.J_inv_by_products(At), np.linalg.inv(dense.big_J(At)),
                               rtol=0, atol=1e-11)


def test_all_bracketings_agree():
    rng = np.random.default_rng(17)
    T, D = 8, 3
    elems = [(rng.normal(size=(D, D)) * 0.7, rng.normal(size=D)) for _ in range(T)]
    res = dense.all_bracketings(elems, dense.affine_op)
    assert len(res) == 429          # Catalan(7)
    A0, b0 = res[0]
    for A, b in res:
        np.testing.assert_allclose(A, A0, rtol=0, atol=1e-12)
        np.testing.assert_allclose(b, b0, rtol=0, atol=1e-12)
    # applied to Delta_0 = 0 the composed map gives the last step of the forward
    # substitution (eq. lin_rr) with c_t = b_t, i.e. r_t = -b_t
    At = np.stack([e[0] for e in elems])
    r = -np.stack([e[1] for e in elems])
    np.testing.assert_allclose(b0, newton.forward_substitution(At, r)[-1], rtol=0, atol=1e-11)


def test_tree_scan_matches_tables():
    g = _gold("tree_scan_T8.json")
    up, down = dense.tree_scan_trace(8)
    assert [[list(c) for c in row] for row in up] == g["upsweep"]
    assert [[list(c) for c in row] for row in down] == g["downsweep"]


# ---- closed forms from Ch. 6 -------------------------------------------------------------

@pytest.mark.parametrize("T", [3, 5, 8, 17])
@pytest.mark.parametrize("D", [1, 2])
def test_picard_inverse_norm_closed_form(T, D):
    At = np.broadcast_to(np.eye(D), (T, D, D)).copy()
    Jinv = np.linalg.inv(dense.big_J(At))
    got = np.linalg.norm(Jinv, 2)
    want = 1.0 / (2.0 * np.sin(np.pi / (2 * (2 * T + 1))))
    assert abs(got - want) < 1e-12 * want


def test_jacobi_error_slope_is_log10_alpha():
    rng = np.random.default_rng(18)
    for alpha in [0.3, 0.5, 0.8]:
        T = 2000
        cell = cells.Affine(np.array([alpha, 1.0, 0.0]), 1, 1)
        x = rng.normal(size=(T, 1))
        ref = rollout.rollout(cell, x, np.array([1.0]))
        out = newton.newton(cell, x, np.array([1.0]), mode="jacobi", tol=0, max_iters=8,
                            history=True)
        errs = [np.linalg.norm(h - ref) for h in out["history"]]
        slope = np.polyfit(np.arange(2, 9), np.log10(errs[2:9]), 1)[0]
        assert abs(slope - np.log10(alpha)) < 0.01 * abs(np.log10(alpha)), (alpha, slope)


# ---- reset heuristic ---------------------------------------------------------------------

def test_reset_keeps_global_convergence():
    rng = np.random.default_rng(19)
    T = 40
    cell = _gru(rng, 3, 2)
    x = rng.normal(size=(T, 2))
    s0 = np.zeros(3)
    init = rng.normal(size=(T, 3))
    init[5] = np.nan
    init[17] = 1e30
    out = newton.newton(cell, x, s0, s_init=init, mode="dense", tol=1e-12)
    assert out["converged"] and out["iters"] <= T
    np.testing.assert_allclose(out["s"], rollout.rollout(cell, x, s0), atol=1e-12)


# ---- damped transitions reduce to the undamped ones at their end points ------------------

@pytest.mark.parametrize("kind", ["gru", "tanh"])
def test_damping_end_points(kind):
    """scale:0 is DEER and diagscale:0 quasi-DEER; scale:1, diagscale:1 and clip:0:0 are Jacobi;
    clip with bounds wider than every diagonal entry is quasi-DEER (Sec. "Further extensions:
    scale- and clip-ELK").  Compared by the matrices and by two iterates of the loop."""
    rng = np.random.default_rng(16)
    T = 30
    cell = _gru(rng, 5, 3) if kind == "gru" else _tanh(rng, 5, 3, g=0.8)
    x = rng.normal(size=(T, cell.Dx))
    s0 = rng.normal(size=5)
    h = np.concatenate([s0[None], rng.normal(size=(T - 1, 5))])
    M = lambda m: newton.transition_matrices(cell, x, h, m)
    np.testing.assert_array_equal(M("scale:0"), M("dense"))
    np.testing.assert_array_equal(M("diagscale:0"), M("diag"))
    for m in ("scale:1", "diagscale:1", "clip:0:0"):
        np.testing.assert_array_equal(M(m), M("jacobi"))
    d = np.abs(np.einsum("tii->ti", M("diag"))).max()
    np.testing.assert_array_equal(M(f"clip:{-(d + 1)}:{d + 1}"), M("diag"))
    # clip really clips: every entry inside the bounds, the off-diagonal zero
    C = M("clip:-0.2:0.1")
    dd = np.einsum("tii->ti", C)
    assert dd.min() >= -0.2 and dd.max() <= 0.1
    np.testing.assert_array_equal(C - np.einsum("ti,ij->tij", dd, np.eye(5)), 0.0)
    for m, ref in (("diagscale:1", "jacobi"), ("scale:0", "dense")):
        a = newton.newton(cell, x, s0, mode=m, tol=1e-14, max_iters=2)["s"]
        b = newton.newton(cell, x, s0, mode=ref, tol=1e-14, max_iters=2)["s"]
        np.testing.assert_array_equal(a, b)


def test_worked_doubling_example_update_norm_stop():
    """stop="delta" (the Ch. 3 rule on the update norm) on the Appendix's doubling example:
    the updates and the counts are worked by hand in the golden file; the loop must stop on
    the first zero update, and never on the residual."""
    g = _gold("worked_doubling.json")
    cell = _scalar_affine(g["f_scale"])
    x = np.zeros((2, 1))
    init = np.array(g["init"])[:, None]
    for mode, key in [("dense", "deer_updates_delta_stop"),
                      ("jacobi", "jacobi_updates_delta_stop"),
                      ("picard", "picard_updates_delta_stop")]:
        out = newton.newton(cell, x, np.array([g["s0"]]), s_init=init, mode=mode, tol=1e-14,
                            history=True, reset_abs=np.inf, stop="delta")
        hist = [h[:, 0] for h in out["history"]]
        updates = [(b - a).tolist() for a, b in zip(hist[:-1], hist[1:])]
        assert updates == g[key], (mode, updates)
        assert out["converged"] and out["iters"] == len(g[key])
        assert out["s"][:, 0].tolist() == g["true"] and out["max_resid"] == 0.0


def test_update_norm_stop_respects_cap_and_agrees_at_convergence():
    """With the update-norm rule the loop still ends within T + 1 updates (one zero update
    after the exact trajectory, Prop. global_convergence), and reaches the rollout."""
    rng = np.random.default_rng(21)
    T = 20
    cell = _tanh(rng, 4, 2, g=2.5)
    x = rng.normal(size=(T, cell.Dx))
    s0 = rng.normal(size=4)
    ref = rollout.rollout(cell, x, s0)
    out = newton.newton(cell, x, s0, mode="jacobi", tol=1e-12, stop="delta", reset_abs=np.inf)
    assert out["converged"] and out["iters"] <= T + 1
    np.testing.assert_allclose(out["s"], ref, rtol=0, atol=1e-11)
    capped = newton.newton(cell, x, s0, mode="jacobi", tol=1e-12, stop="delta",
                           max_iters=3, reset_abs=np.inf)
    assert not capped["converged"] and capped["iters"] == 3
