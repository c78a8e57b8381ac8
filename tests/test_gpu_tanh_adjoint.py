"""GPU parity: exact adjoint of the dense tanh-RNN (reverse dense scans with FP32 or BF16 group
maps driven by the exact FP32 residual) and the parameter / input / initial-state gradients,
against the FP64 sequential adjoint of the oracle.

Both sides take the same FP32 trajectory s and the same g = 2 s.  Bar (per gradient tensor
W, U, b, dx, ds_0): max |g - g*| / max |g*| <= 1e-5.  The adjoint recurrence of these cells
contracts (gain 0.9), so FP32 rounding of the scan stays at the 1e-6 level; the parameter
gradients are FP32 per-workgroup partials summed in FP64.
"""
import numpy as np
import pytest

from oracle import adjoint, cells, rollout
from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def _check(cell, got, want, tol=TOL):
    D, Dx = cell.D, cell.Dx
    gp, gx, g0 = got
    wp, wx, w0 = want
    o = 0
    for name, n in (("W", D * D), ("U", D * Dx), ("b", D)):
        r = _rel(gp[o:o + n], wp[o:o + n])
        assert r < tol, (name, r)
        o += n
    assert _rel(gx, wx) < tol, ("gx", _rel(gx, wx))
    assert _rel(g0, w0) < tol, ("gs0", _rel(g0, w0))


def _case(Dx, lengths, seed):
    w = workloads.TANH32_DENSE_BF16.scaled(B=len(lengths), T=0)
    w = workloads.Workload(w.name, "tanh", D=32, Dx=Dx, B=len(lengths), gain=w.gain,
                           jac="dense", tol=1e-6)
    inst = workloads.make_instance(w, seed=seed, lengths=np.asarray(lengths))
    cell = cells.TanhRNN(inst.params, 32, Dx)
    s = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s32 = s.astype(np.float32).astype(np.float64)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, s32, 2 * s32, inst.offsets)[1:]
    return inst, cell, s32, want


def _run(lib, inst, s32, **kw):
    gp, gx, g0, info = lib.deer_adjoint(_t(inst.x), _t(inst.s0), _t(inst.params), _t(s32),
                                        _t(2 * s32), cell="tanh", offsets=inst.offsets,
                                        jac="dense", **kw)
    return tuple(v.cpu().double().numpy() for v in (gp, gx, g0)), info


@pytest.mark.parametrize("Dx", [16, 32])
@pytest.mark.parametrize("compose", ["native", "bf16"])
def test_adjoint_on_oracle_trajectory(lib, Dx, compose):
    """Ragged batch with an empty and a one-step sequence; chunks of 32 with ragged tails."""
    inst, cell, s32, want = _case(Dx, [300, 1, 0, 131, 65], seed=17)
    got, info = _run(lib, inst, s32, compose=compose, tol=1e-6)
    assert all(i["converged"] for i in info if i is not None)
    _check(cell, got, want)
    if compose == "native":
        # exact FP32 maps: one update reaches the adjoint, the next iteration confirms it
        assert max(i["iters"] for i in info if i is not None) <= 2


@pytest.mark.parametrize("compose,group", [("native", 1), ("bf16", 2), ("native", 0)])
def test_many_groups_match_oracle(lib, compose, group):
    """Long sequences cut into many groups: the carry runs over the reverse-ordered groups and
    every group's first chunk takes its halo row from the carry."""
    inst, cell, s32, want = _case(16, [5000, 2100, 33, 4097], seed=18)
    got, info = _run(lib, inst, s32, compose=compose, tol=1e-6, group=group)
    assert all(i["converged"] for i in info)
    _check(cell, got, want)


def test_sequential_baseline(lib):
    """seq_bptt on the dense tanh cell (the reverse recurrence walked step by step) meets the
    same bar against the oracle."""
    inst, cell, s32, want = _case(32, [300, 1, 0, 131, 65], seed=20)
    gp, gx, g0 = lib.seq_bptt(_t(inst.x), _t(inst.s0), _t(inst.params), _t(s32), _t(2 * s32),
                              cell="tanh", offsets=inst.offsets)
    _check(cell, tuple(v.cpu().double().numpy() for v in (gp, gx, g0)), want)


def test_autograd_function_full_path(lib):
    """deer() forward (dense BF16 DEER) and its backward (this adjoint) against the oracle's
    rollout and adjoint."""
    import torch
    w = workloads.TANH32_DENSE_BF16.scaled(B=3, T=1500)
    inst = workloads.make_instance(w, seed=19)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    x = _t(inst.x).requires_grad_(True)
    s0 = _t(inst.s0).requires_grad_(True)
    p = _t(inst.params).requires_grad_(True)
    s = lib.deer(x, s0, p, cell="tanh", offsets=inst.offsets, jac="dense", compose="bf16",
                 tol=1e-6)
    (s * s).sum().backward()
    sref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, sref, 2 * sref, inst.offsets)[1:]
    got = tuple(v.grad.cpu().double().numpy() for v in (p, x, s0))
    _check(cell, got, want)


def test_full_size(lib):
    """The dense tanh workload at full size (32 sequences of 16384 steps, Dx = 16), BF16 maps,
    the launch configuration the benchmark times, against the oracle's adjoint."""
    w = workloads.TANH32_DENSE_BF16
    inst = workloads.make_instance(w, seed=0)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    s = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s32 = s.astype(np.float32).astype(np.float64)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, s32, 2 * s32, inst.offsets)[1:]
    got, info = _run(lib, inst, s32, compose="bf16", tol=1e-6)
    assert all(i["converged"] for i in info)
    _check(cell, got, want)
