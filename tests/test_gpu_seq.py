"""GPU parity of the sequential baselines the benchmark compares against: the rollout
(GRU, tanh) and backpropagation through it (GRU), against the FP64 oracle.

Bars: rollout within 1e-5 relative of the FP64 rollout on contracting instances (the FP32
sequential recurrence accumulates rounding like the parallel solve); gradients within 1e-5
relative of the oracle's sequential adjoint on the same FP32 trajectory.
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


@pytest.mark.parametrize("cell_kind,D,Dx", [("gru", 64, 32), ("gru", 48, 24), ("tanh", 32, 16),
                                            ("tanh", 16, 16)])
def test_seq_rollout(lib, cell_kind, D, Dx):
    w = workloads.Workload("t", cell_kind, D=D, Dx=Dx, B=3, gain=0.9)
    inst = workloads.make_instance(w, seed=50, lengths=np.array([700, 0, 33]))
    cell = cells.make_cell(cell_kind, inst.params, D, Dx)
    s = lib.seq_rollout(_t(inst.x), _t(inst.s0), _t(inst.params), cell=cell_kind,
                        offsets=inst.offsets)
    ref = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    assert _rel(s.cpu().double().numpy(), ref) < 1e-5


@pytest.mark.parametrize("D,Dx", [(64, 32), (16, 8)])
def test_seq_bptt(lib, D, Dx):
    w = workloads.Workload("t", "gru", D=D, Dx=Dx, B=3)
    inst = workloads.make_instance(w, seed=51, lengths=np.array([400, 1, 90]))
    cell = cells.GRU(inst.params, D, Dx)
    s = rollout.rollout_batch(cell, inst.x, inst.s0, inst.offsets)
    s32 = s.astype(np.float32).astype(np.float64)
    _, wp, wx, w0 = adjoint.adjoint_batch(cell, inst.x, inst.s0, s32, 2 * s32, inst.offsets)
    gp, gx, g0 = lib.seq_bptt(_t(inst.x), _t(inst.s0), _t(inst.params), _t(s32), _t(2 * s32),
                              cell="gru", offsets=inst.offsets)
    for got, want in ((gp, wp), (gx, wx), (g0, w0)):
        assert _rel(got.cpu().double().numpy(), want) < 1e-5
