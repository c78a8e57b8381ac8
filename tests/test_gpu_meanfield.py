"""GPU parity: the mean-field RNN (Ch. 5 predictability experiments) through the ELK/DEER
kernels, the sequential baseline, the FP64 residual and the LLE estimate (Alg. LLE_estimate).

Bars: per-iteration DEER / ELK / smoother iterates within 2e-5 of the oracle relative to
max(1, max |s|); the sequential rollout within 1e-5 of the FP64 rollout on a contracting
instance; the FP64 residual to 1e-12 of the oracle's float64 residual of the same FP32 data;
the LLE estimate within 1e-4 of the oracle's estimate on the same FP32 trajectory and
starting vector (log stretches of O(1) summed over T steps in FP32 arithmetic, FP64 sum).
"""
import numpy as np
import pytest

from oracle import cells, elk, lle, newton, rollout
from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _inst(g, lengths=(300, 1, 77), seed=40):
    w = workloads.MEANFIELD16.scaled(gain=g, B=len(lengths), T=0)
    inst = workloads.make_instance(w, seed=seed, lengths=np.array(lengths))
    return inst, cells.MeanFieldRNN(inst.params, 16, 16)


def _bar(ref):
    return 2e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("lam,jac,smooth", [(0.0, "dense", False), (0.1, "dense", False),
                                            (0.1, "dense", True), (0.05, "diag", False)])
@pytest.mark.parametrize("g", [0.8, 2.0])
def test_iterates_match_oracle(lib, g, lam, jac, smooth):
    inst, cell = _inst(g)
    for k in (1, 2, 5):
        s, info = lib.elk_solve(_t(inst.x), _t(inst.s0), _t(inst.params), lam, cell="meanfield",
                                offsets=inst.offsets, tol=1e-12, max_iters=k, jac=jac,
                                smooth=smooth, tile=32)
        s = s.cpu().double().numpy()
        for b in range(3):
            a, e = inst.offsets[b], inst.offsets[b + 1]
            out = elk.elk(cell, inst.x[a:e], inst.s0[b], lam, mode=jac, smoother=smooth,
                          tol=1e-12, max_iters=k)
            assert np.abs(s[a:e] - out["s"]).max() < _bar(out["s"]), (k, b)


def test_deer_converges_and_threshold(lib):
    """DEER (lambda = 0) reaches the rollout; the iteration count jumps once the LLE turns
    positive (the threshold of Ch. 5)."""
    iters = {}
    for g in (0.5, 2.0):
        w = workloads.MEANFIELD16.scaled(gain=g)
        inst = workloads.make_instance(w, seed=1)
        cell = cells.MeanFieldRNN(inst.params, 16, 16)
        ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
        s, info = lib.elk_solve(_t(inst.x), _t(inst.s0), _t(inst.params), 0.0, cell="meanfield",
                                offsets=inst.offsets, tol=w.tol, fp64_final_residual=True)
        if g == 0.5:
            assert info[0]["converged"] and info[0]["max_resid"] < w.tol
            assert np.abs(s.cpu().double().numpy() - ref).max() < 1e-5
        # the chaotic case may reach the iteration cap T before the FP32 residual settles
        iters[g] = info[0]["iters"]
    assert iters[2.0] > 10 * iters[0.5], iters


def test_seq_rollout_and_residual(lib):
    inst, cell = _inst(0.6, lengths=(500, 0, 64))
    s = lib.seq_rollout(_t(inst.x), _t(inst.s0), _t(inst.params), cell="meanfield",
                        offsets=inst.offsets)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    got = s.cpu().double().numpy()
    assert np.abs(got - ref).max() < 1e-5
    r64 = lib.residual_f64(_t(inst.x), _t(inst.s0), _t(inst.params), s, cell="meanfield",
                           offsets=inst.offsets)
    p32 = inst.params.astype(np.float32).astype(np.float64)
    c32 = cells.MeanFieldRNN(p32, 16, 16)
    x32 = inst.x.astype(np.float32).astype(np.float64)
    s032 = inst.s0.astype(np.float32).astype(np.float64)
    for b in range(3):
        a, e = inst.offsets[b], inst.offsets[b + 1]
        if e == a:
            assert r64[b] == 0.0
            continue
        _, r = newton.linearize(c32, x32[a:e], s032[b], got[a:e])
        assert abs(r64[b] - np.abs(r).max()) < 1e-12


@pytest.mark.parametrize("kind,g", [("meanfield", 0.6), ("meanfield", 2.0), ("tanh", 1.5)])
def test_lle_matches_oracle(lib, kind, g):
    if kind == "meanfield":
        inst, cell = _inst(g, lengths=(2000, 0, 333))
    else:
        w = workloads.TANH16_ELK.scaled(B=3, T=0, gain=g)
        inst = workloads.make_instance(w, seed=41, lengths=np.array([2000, 0, 333]))
        cell = cells.TanhRNN(inst.params, 16, 16)
    traj = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets).astype(np.float32)
    u0 = np.random.default_rng(42).standard_normal((3, 16))
    got = lib.lle_estimate(_t(inst.x), _t(inst.s0), _t(inst.params), _t(traj), _t(u0),
                           cell=kind, offsets=inst.offsets)
    p32 = inst.params.astype(np.float32).astype(np.float64)
    c32 = cells.make_cell(kind, p32, 16, 16)
    for b in range(3):
        a, e = inst.offsets[b], inst.offsets[b + 1]
        if e == a:
            assert got[b] == 0.0
            continue
        J = lle.trajectory_jacobians(c32, inst.x[a:e].astype(np.float32).astype(np.float64),
                                     inst.s0[b].astype(np.float32).astype(np.float64),
                                     traj[a:e].astype(np.float64))
        ref = lle.lle_estimate(J, u0[b].astype(np.float32).astype(np.float64))
        assert abs(got[b] - ref) < 1e-4, (b, got[b], ref)
