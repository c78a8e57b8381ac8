"""GPU parity: DEER with dense Jacobians for the tanh-RNN (D = 32), the chunk products composed
on MFMA in BF16 (FP32 accumulation) or FP32, against the FP64 oracle.

Bar: trajectory within 1e-5 relative of the sequential rollout for both compose modes (the
residual stays FP32, so BF16 products change the iteration count, not the fixed point);
FP32-compose iterates within 1e-5 of the oracle's sequential DEER iterates.
"""
import numpy as np
import pytest

from oracle import cells, newton, rollout
from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def _solve(lib, inst, compose, **kw):
    s, info = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="tanh",
                             offsets=inst.offsets, jac="dense", compose=compose, **kw)
    return s.cpu().double().numpy(), info


@pytest.mark.parametrize("compose", ["f32", "bf16"])
@pytest.mark.parametrize("Dx", [16, 32])
def test_ragged_matches_rollout(lib, compose, Dx):
    w = workloads.TANH32_DENSE_BF16.scaled(Dx=Dx, B=4, T=0)
    inst = workloads.make_instance(w, seed=21, lengths=np.array([700, 1, 0, 97]))
    cell = cells.TanhRNN(inst.params, w.D, Dx)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s, info = _solve(lib, inst, "native" if compose == "f32" else "bf16", tol=1e-6)
    assert all(i["converged"] for i in info), info
    assert _rel(s, ref) < 1e-5
    if compose == "f32":
        _, oinfo = newton.newton_batch(cell, inst.x, inst.s0, inst.offsets, mode="dense", tol=1e-6)
        for gi, oi in zip(info, oinfo):
            assert abs(gi["iters"] - oi["iters"]) <= 1, (gi, oi["iters"])


def test_f32_iterates_match_oracle(lib):
    w = workloads.TANH32_DENSE_BF16.scaled(B=2, T=300)
    inst = workloads.make_instance(w, seed=22)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    for k in (1, 2, 3):
        s, info = _solve(lib, inst, "native", tol=1e-12, max_iters=k)
        for b in range(2):
            a, e = inst.offsets[b], inst.offsets[b + 1]
            out = newton.newton(cell, inst.x[a:e], inst.s0[b], mode="dense", tol=1e-12,
                                max_iters=k)
            assert np.abs(s[a:e] - out["s"]).max() < 1e-5


@pytest.mark.parametrize("compose", ["bf16", "native"])
def test_full_size(lib, compose):
    w = workloads.TANH32_DENSE_BF16
    inst = workloads.make_instance(w, seed=0)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    s, info = _solve(lib, inst, compose, tol=1e-6)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    assert all(i["converged"] for i in info)
    assert _rel(s, ref) < 1e-5, _rel(s, ref)


@pytest.mark.parametrize("compose", ["native", "bf16"])
def test_scale_damping(lib, compose):
    """scale-ELK on the dense path: A~_t = (1 - k) A_t (Sec. "Further extensions: scale- and
    clip-ELK"); FP32 iterates equal the oracle loop with the same transition; both composes
    converge to the rollout."""
    w = workloads.TANH32_DENSE_BF16.scaled(B=2, T=300)
    inst = workloads.make_instance(w, seed=23)
    cell = cells.TanhRNN(inst.params, w.D, w.Dx)
    if compose == "native":
        for k in (1, 2, 3):
            s, _ = _solve(lib, inst, compose, tol=1e-12, max_iters=k, damping="scale",
                          damp_k=0.25)
            for b in range(2):
                a, e = inst.offsets[b], inst.offsets[b + 1]
                out = newton.newton(cell, inst.x[a:e], inst.s0[b], mode="scale:0.25",
                                    tol=1e-12, max_iters=k)
                assert np.abs(s[a:e] - out["s"]).max() < 1e-5
    s, info = _solve(lib, inst, compose, tol=1e-6, damping="scale", damp_k=0.25)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    assert all(i["converged"] for i in info)
    assert _rel(s, ref) < 1e-5
