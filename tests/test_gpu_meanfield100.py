"""GPU parity: the mean-field RNN at the thesis's D = 100 (and other sizes up to 128) --
dense DEER by the two-level scan (FP32 or BF16 group maps, FP32 residual and chains), the
sequential rollout and the LLE estimate, against the FP64 oracle.

Bars: DEER iterates with FP32 maps within 2e-5 of the oracle's Newton iterates relative to
max(1, max |s|) on a predictable instance (each is exact Newton on the FP32 data); converged
trajectories (FP32 or BF16 maps) within 1e-5 of the FP64 rollout; the sequential rollout
within 1e-5 of it; the LLE estimate within 1e-4 of the oracle's on the same FP32 trajectory
and starting vector.
"""
import numpy as np
import pytest

from oracle import cells, lle, newton, rollout
from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _inst(g, D=100, lengths=(300, 1, 77), seed=50):
    w = workloads.MEANFIELD100.scaled(gain=g, D=D, Dx=D, B=len(lengths), T=0)
    inst = workloads.make_instance(w, seed=seed, lengths=np.array(lengths))
    return inst, cells.MeanFieldRNN(inst.params, D, D)


def _bar(ref):
    return 2e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("D", [100, 128, 40])
def test_fp32_map_iterates_match_oracle_newton(lib, D):
    inst, cell = _inst(0.8, D=D)
    for k in (1, 2, 4):
        s, info = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="meanfield",
                                 offsets=inst.offsets, jac="dense", compose="native",
                                 tol=1e-30, max_iters=k, group=2)
        # (the one-step sequence is exact after one update: residual 0 passes any tol)
        assert all((i["iters"] == k and not i["converged"]) or i["max_resid"] == 0.0
                   for i in info), info
        s = s.cpu().double().numpy()
        for b in range(len(inst.offsets) - 1):
            a, e = inst.offsets[b], inst.offsets[b + 1]
            out = newton.newton(cell, inst.x[a:e], inst.s0[b], mode="dense", tol=0.0,
                                max_iters=k)
            assert np.abs(s[a:e] - out["s"]).max() < _bar(out["s"]), (D, k, b)


@pytest.mark.parametrize("compose", ["bf16", "native"])
@pytest.mark.parametrize("group", [1, 3, 0])
def test_converges_to_the_rollout(lib, compose, group):
    inst, cell = _inst(0.9, lengths=(1000, 1, 333, 64))
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s, info = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="meanfield",
                             offsets=inst.offsets, jac="dense", compose=compose, tol=1e-6,
                             group=group)
    assert all(i["converged"] and i["max_resid"] < 1e-6 for i in info), info
    assert np.abs(s.cpu().double().numpy() - ref).max() < 1e-5
    # a predictable instance: a handful of Newton iterations
    assert max(i["iters"] for i in info) <= 8, info


def test_graph_and_direct_paths_agree(lib):
    import torch
    inst, cell = _inst(0.9, lengths=(700, 50))
    kw = dict(cell="meanfield", offsets=inst.offsets, jac="dense", compose="bf16", tol=1e-6)
    a, _ = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), use_graph=True, **kw)
    b, _ = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), use_graph=False, **kw)
    assert torch.equal(a, b)


def test_chaotic_instance_is_capped_or_exact(lib):
    """g = 2 is chaotic: DEER still ends at the rollout within T iterations (Prop.
    global_convergence) or reports the cap."""
    inst, cell = _inst(2.0, lengths=(120,), seed=51)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s, info = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="meanfield",
                             offsets=inst.offsets, jac="dense", compose="native", tol=1e-5)
    if info[0]["converged"]:
        assert info[0]["max_resid"] < 1e-5
    else:
        assert info[0]["iters"] == 120


def test_seq_rollout_and_lle(lib):
    inst, cell = _inst(0.7, lengths=(500, 0, 64))
    s = lib.seq_rollout(_t(inst.x), _t(inst.s0), _t(inst.params), cell="meanfield",
                        offsets=inst.offsets)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    got = s.cpu().double().numpy()
    assert np.abs(got - ref).max() < 1e-5
    u0 = np.random.default_rng(3).standard_normal((3, 100))
    est = lib.lle_estimate(_t(inst.x), _t(inst.s0), _t(inst.params), s, _t(u0),
                           cell="meanfield", offsets=inst.offsets)
    p32 = inst.params.astype(np.float32).astype(np.float64)
    c32 = cells.MeanFieldRNN(p32, 100, 100)
    assert est[1] == 0.0                       # the empty sequence
    for b in (0, 2):
        a, e = inst.offsets[b], inst.offsets[b + 1]
        J = lle.trajectory_jacobians(c32, inst.x[a:e].astype(np.float32).astype(np.float64),
                                     inst.s0[b].astype(np.float32).astype(np.float64), got[a:e])
        want = lle.lle_estimate(J, u0[b].astype(np.float32).astype(np.float64))
        assert abs(est[b] - want) < 1e-4, (b, est[b], want)
