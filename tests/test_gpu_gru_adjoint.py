"""GPU parity: exact quasi adjoint of the GRU (iterated reverse diagonal scans + exact VJP)
and the parameter / input / initial-state gradients, against the FP64 sequential adjoint.

Bar (per gradient tensor): max |g - g*| / max |g*| <= 1e-5 when the forward trajectory is
the oracle's; the full fwd+bwd path (GPU forward then GPU adjoint) is held to the same bar.
"""
import numpy as np
import pytest

from oracle import adjoint, cells, rollout
from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def _split(cell, gp):
    D, Dx = cell.D, cell.Dx
    o = 0
    out = {}
    for name, n in (("W", 3 * D * Dx), ("U", 3 * D * D), ("b", 3 * D), ("bhn", D)):
        out[name] = gp[o:o + n]
        o += n
    return out


def _check_grads(cell, got, want, tol):
    gp, gx, g0 = got
    wp, wx, w0 = want
    gs, ws = _split(cell, gp), _split(cell, wp)
    for k in gs:
        assert _rel(gs[k], ws[k]) < tol, (k, _rel(gs[k], ws[k]))
    assert _rel(gx, wx) < tol, ("gx", _rel(gx, wx))
    assert _rel(g0, w0) < tol, ("gs0", _rel(g0, w0))


@pytest.mark.parametrize("D,Dx", [(64, 32), (48, 24), (16, 8)])
def test_adjoint_on_oracle_trajectory(lib, D, Dx):
    w = workloads.Workload("t", "gru", D=D, Dx=Dx, B=4, tol=1e-5)
    inst = workloads.make_instance(w, seed=7, lengths=np.array([300, 1, 0, 131]))
    cell = cells.GRU(inst.params, D, Dx)
    s = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s32 = s.astype(np.float32).astype(np.float64)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, s32, 2 * s32, inst.offsets)[1:]
    gp, gx, g0, info = lib.deer_adjoint(_t(inst.x), _t(inst.s0), _t(inst.params), _t(s32),
                                        _t(2 * s32), cell="gru", offsets=inst.offsets,
                                        jac="diag", tol=1e-6)
    assert all(i["converged"] for i in info if i is not None)
    got = tuple(v.cpu().double().numpy() for v in (gp, gx, g0))
    _check_grads(cell, got, want, 1e-5)


def test_autograd_function_full_path(lib):
    import torch
    w = workloads.GRU64_QUASI.scaled(T=2000, B=3)
    inst = workloads.make_instance(w, seed=8)
    cell = cells.GRU(inst.params, w.D, w.Dx)
    x = _t(inst.x).requires_grad_(True)
    s0 = _t(inst.s0).requires_grad_(True)
    p = _t(inst.params).requires_grad_(True)
    s = lib.deer(x, s0, p, cell="gru", offsets=inst.offsets, jac="diag", tol=1e-6)
    (s * s).sum().backward()
    sref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, sref, 2 * sref, inst.offsets)[1:]
    got = tuple(v.grad.cpu().double().numpy() for v in (p, x, s0))
    _check_grads(cell, got, want, 1e-5)


@pytest.mark.parametrize("name", ["gru64-quasi-f32", "gru48-ragged-quasi"])
def test_full_size_fwd_bwd(lib, name):
    w = workloads.ALL[name]
    inst = workloads.make_instance(w, seed=0)
    cell = cells.GRU(inst.params, w.D, w.Dx)
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    s, finfo = lib.deer_solve(x, s0, p, cell="gru", offsets=inst.offsets, jac="diag", tol=1e-6)
    gp, gx, g0, binfo = lib.deer_adjoint(x, s0, p, s, 2 * s, cell="gru", offsets=inst.offsets,
                                         jac="diag", tol=1e-6)
    assert all(i["converged"] for i in finfo) and all(i["converged"] for i in binfo)
    sref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, sref, 2 * sref, inst.offsets)[1:]
    got = tuple(v.cpu().double().numpy() for v in (gp, gx, g0))
    _check_grads(cell, got, want, 1e-5)


@pytest.mark.parametrize("damp", [dict(damping="scale", damp_k=0.5), dict(damping="clip", clip=(-0.3, 0.6))])
def test_damped_adjoint_gives_the_same_gradients(lib, damp):
    """The damping changes the reverse scans' transition only; the exact VJP residual fixes
    the result, so the gradients equal the oracle's."""
    import torch
    from oracle import adjoint
    w = workloads.GRU64_QUASI.scaled(B=3, T=0)
    inst = workloads.make_instance(w, seed=44, lengths=np.array([250, 64, 129]))
    cell = cells.GRU(inst.params, w.D, w.Dx)
    sref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    _, wp, wx, w0 = adjoint.adjoint_batch(cell, inst.x, inst.s0, sref, 2 * sref, inst.offsets)
    t = lambda v: torch.tensor(v, dtype=torch.float32, device="cuda")
    gp, gx, g0, info = lib.deer_adjoint(t(inst.x), t(inst.s0), t(inst.params), t(sref),
                                        t(2 * sref), cell="gru", offsets=inst.offsets,
                                        tol=1e-6, **damp)
    assert all(i["converged"] for i in info), info
    rel = lambda a, b: np.abs(a.cpu().double().numpy() - b).max() / np.abs(b).max()
    assert rel(gp, wp) < 1e-5 and rel(gx, wx) < 1e-5 and rel(g0, w0) < 1e-5


@pytest.mark.parametrize("group", [1, 0])
def test_adjoint_freeze_prefix(lib, group):
    """Converged-prefix skipping in the adjoint's scan order (groups from the sequence end):
    the gradients stay within the bar, and the iterations do not grow."""
    w = workloads.GRU48_RAGGED.scaled(B=3, T=0)
    inst = workloads.make_instance(w, seed=82, lengths=np.array([2100, 1, 640]))
    cell = cells.GRU(inst.params, w.D, w.Dx)
    s = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s32 = s.astype(np.float32).astype(np.float64)
    want = adjoint.adjoint_batch(cell, inst.x, inst.s0, s32, 2 * s32, inst.offsets)[1:]
    out = {}
    for fz in (False, True):
        gp, gx, g0, info = lib.deer_adjoint(_t(inst.x), _t(inst.s0), _t(inst.params), _t(s32),
                                            _t(2 * s32), cell="gru", offsets=inst.offsets,
                                            jac="diag", tol=1e-6, freeze_prefix=fz,
                                            group=group)
        assert all(i["converged"] for i in info)
        got = tuple(v.cpu().double().numpy() for v in (gp, gx, g0))
        _check_grads(cell, got, want, 1e-5)
        out[fz] = [i["iters"] for i in info]
    assert all(a <= b + 1 for a, b in zip(out[True], out[False])), out
