"""Oracle pins for converged-prefix skipping (the causal-convergence argument in the proof of
Prop. global_convergence; sliding-window discussion of Ch. 3).

The frozen-prefix rule is pinned by brute force on hand-made residuals; the restart after
the frozen prefix is pinned against the plain loop run on the sub-problem that starts from
the last frozen state (s_0 := s_{t0}, the remaining inputs), which has no notion of
freezing; the invariants (frozen states never change, the returned iterate still passes the
stop test, a block at least as long as the sequence changes nothing) hold on every run.
"""
import numpy as np
import pytest

from oracle import cells, elk, newton
from paper_2603_16850_amd import workloads


def _inst(seed=36, lengths=(300, 77, 160)):
    w = workloads.TANH16_ELK.scaled(B=len(lengths), T=0)
    inst = workloads.make_instance(w, seed=seed, lengths=np.array(lengths))
    return inst, cells.TanhRNN(inst.params, w.D, w.Dx)


def test_frozen_prefix_brute_force():
    tol = 1e-3
    r = np.zeros((9, 2))
    r[0, 0], r[3, 1], r[4, 0], r[7, 1] = 1e-4, 5e-4, 2e-3, 1e-4
    assert newton.frozen_prefix(r, 2, tol) == 4          # blocks [0,2) [2,4) pass, [4,6) fails
    assert newton.frozen_prefix(r, 3, tol) == 3          # [3,6) holds 2e-3
    assert newton.frozen_prefix(r, 5, tol) == 0
    r[4, 0] = 0.0
    assert newton.frozen_prefix(r, 2, tol) == 9          # all pass; ragged last block
    assert newton.frozen_prefix(r, 100, tol) == 9
    r[1, 1] = np.nan
    assert newton.frozen_prefix(r, 2, tol) == 0          # NaN is not below tol
    r[1, 1] = tol
    assert newton.frozen_prefix(r, 2, tol) == 0          # strict inequality, as the stop test
    assert newton.frozen_prefix(np.zeros((0, 2)), 4, tol) == 0


def _advance(cell, x, s0, lam, mode, iters):
    """An iterate whose leading blocks have converged: `iters` plain updates."""
    return elk.elk(cell, x, s0, lam, mode=mode, tol=0.0, max_iters=iters)["s"]


@pytest.mark.parametrize("lam,mode,block", [(0.0, "dense", 16), (0.05, "dense", 16),
                                            (0.05, "diag", 32), (0.0, "diag", 8)])
def test_restart_equals_subproblem(lam, mode, block):
    """One update with a frozen prefix = the prefix kept, and on the rest exactly one update
    of the sub-problem that starts from the last frozen state."""
    inst, cell = _inst()
    a, e = inst.offsets[0], inst.offsets[1]
    x, s0 = inst.x[a:e], inst.s0[0]
    s = _advance(cell, x, s0, lam, mode, 12 if lam else 7)
    _, r = newton.linearize(cell, x, s0, s)
    bmax = [np.abs(r[j:j + block]).max() for j in range(0, r.shape[0], block)]
    # a tolerance that freezes exactly the first nf blocks (the largest nf with a gap)
    nf = max(n for n in range(1, len(bmax)) if max(bmax[:n]) < bmax[n])
    tol = float(np.sqrt(max(bmax[:nf]) * bmax[nf]))
    assert max(bmax[:nf]) < tol <= bmax[nf]
    t0 = newton.frozen_prefix(r, block, tol)
    assert t0 == nf * block
    one = elk.elk(cell, x, s0, lam, mode=mode, tol=tol, max_iters=1, s_init=s, freeze=block)
    sub = elk.elk(cell, x[t0:], s[t0 - 1], lam, mode=mode, tol=0.0, max_iters=1,
                  s_init=s[t0:])
    assert one["iters"] == 1
    assert np.array_equal(one["s"][:t0], s[:t0])
    np.testing.assert_allclose(one["s"][t0:], sub["s"], rtol=0, atol=1e-12)
    # and the update differs from the unfrozen one (the restart matters)
    full = elk.elk(cell, x, s0, lam, mode=mode, tol=0.0, max_iters=1, s_init=s)
    assert np.abs(full["s"][t0:] - one["s"][t0:]).max() > 0


@pytest.mark.parametrize("lam,mode,block", [(0.0, "dense", 16), (0.05, "dense", 48),
                                            (0.05, "diag", 32)])
def test_frozen_states_never_change(lam, mode, block):
    inst, cell = _inst()
    tol = 1e-3
    work_frozen = work_plain = 0
    for b in range(3):
        a, e = inst.offsets[b], inst.offsets[b + 1]
        x, s0 = inst.x[a:e], inst.s0[b]
        out = elk.elk(cell, x, s0, lam, mode=mode, tol=tol, history=True, freeze=block)
        assert out["converged"]
        hist = out["history"]
        for i in range(len(hist) - 1):
            _, r = newton.linearize(cell, x, s0, hist[i])
            t0 = newton.frozen_prefix(r, block, tol)
            for j in range(i + 1, len(hist)):
                assert np.array_equal(hist[j][:t0], hist[i][:t0]), (b, i, j)
            work_frozen += x.shape[0] - t0
            work_plain += x.shape[0]
        _, r = newton.linearize(cell, x, s0, out["s"])
        assert np.abs(r).max() < tol
    assert work_frozen < work_plain        # the causal front freezes something on this instance


@pytest.mark.parametrize("lam,mode", [(0.0, "dense"), (0.05, "diag")])
def test_block_longer_than_sequence_changes_nothing(lam, mode):
    inst, cell = _inst()
    a, e = inst.offsets[1], inst.offsets[2]
    x, s0 = inst.x[a:e], inst.s0[1]
    plain = elk.elk(cell, x, s0, lam, mode=mode, tol=1e-6, history=True)
    for block in (e - a, 4 * (e - a)):
        fr = elk.elk(cell, x, s0, lam, mode=mode, tol=1e-6, history=True, freeze=block)
        assert fr["iters"] == plain["iters"]
        for u, v in zip(fr["history"], plain["history"]):
            assert np.array_equal(u, v)


def test_deer_freeze_matches_newton_freeze():
    """lambda = 0 ELK with freezing is DEER with freezing (the step callable and the plain
    forward substitution take the same restart)."""
    inst, cell = _inst()
    a, e = inst.offsets[2], inst.offsets[3]
    x, s0 = inst.x[a:e], inst.s0[2]
    u = elk.elk(cell, x, s0, 0.0, tol=1e-3, freeze=16, history=True)
    v = newton.newton(cell, x, s0, mode="dense", tol=1e-3, freeze=16, history=True)
    assert u["iters"] == v["iters"]
    for p, q in zip(u["history"], v["history"]):
        np.testing.assert_allclose(p, q, rtol=0, atol=1e-10)
