"""GPU: the scan-tile autotuner (pn_autotune) and the group-length option it tunes.

The tuner must (1) time every candidate of the route and return the fastest, (2) leave the
caller's iterate as it was, (3) answer a known shape class from its cache without running
anything, also from the JSON cache file, and (4) a solve with tile="auto" must equal the solve
with the returned (tile, group).  The group length only moves rounding: every candidate's
result stays within the usual bars of the sequential rollout.
"""
import json

import numpy as np
import pytest

import paper_2603_16850_amd as pn
from oracle import cells, rollout
from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _gru_inst():
    w = workloads.GRU48_RAGGED.scaled(B=6, T=0)
    return w, workloads.make_instance(w, seed=41, lengths=np.array([700, 64, 1, 2100, 333, 900]))


def test_deer_tuner_times_all_candidates_and_restores_s(lib):
    import torch
    w, inst = _gru_inst()
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    lib.load().pn_autotune_reset()
    s_init = torch.randn(x.shape[0], w.D, device="cuda") * 0.1
    before = s_init.clone()
    t = lib.autotune("deer", x, s0, p, cell="gru", offsets=inst.offsets, s=s_init, jac="diag")
    assert torch.equal(s_init, before)
    assert not t["from_cache"]
    cands = t["candidates"]
    assert len(cands) == 18
    assert {(a, b) for a, b, _ in cands} == {(L, g) for L in (32, 64, 128)
                                            for g in (0, 1, 2, 4, 8, 16)}
    ms = [m for _, _, m in cands if m is not None]
    assert len(ms) == 18 and all(m > 0 for m in ms)
    best = min(cands, key=lambda c: c[2])
    assert (t["tile"], t["group"]) == best[:2]
    assert t["ms_per_iter"] == pytest.approx(best[2], rel=1e-5)
    # known shape class: from the cache, no kernel runs
    with lib.profile():
        t2 = lib.autotune("deer", x, s0, p, cell="gru", offsets=inst.offsets, jac="diag")
        launches = lib.profile.read("gru_quasi_local")[1]
    assert t2["from_cache"] and (t2["tile"], t2["group"]) == (t["tile"], t["group"])
    assert launches == 0
    # tile="auto" is the solve with the returned options
    sa, ia = lib.deer_solve(x, s0, p, cell="gru", offsets=inst.offsets, jac="diag", tile="auto")
    sb, ib = lib.deer_solve(x, s0, p, cell="gru", offsets=inst.offsets, jac="diag",
                            tile=t["tile"], group=t["group"])
    assert torch.equal(sa, sb) and [i["iters"] for i in ia] == [i["iters"] for i in ib]


@pytest.mark.parametrize("tile,group", [(32, 1), (64, 3), (128, 16), (64, 64)])
def test_group_length_moves_rounding_only(lib, tile, group):
    """deer_solve GRU diagonal with explicit group lengths (3 and 64: groups that do not
    divide the sequences, and one group per sequence) converges to the sequential rollout."""
    w, inst = _gru_inst()
    s, info = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="gru",
                             offsets=inst.offsets, jac="diag", tol=1e-6, tile=tile, group=group)
    assert all(i["converged"] for i in info)
    ref = rollout.rollout_batch(cells.GRU(inst.params, w.D, w.Dx), inst.x, inst.s0, inst.offsets)
    s = s.cpu().double().numpy()
    assert np.abs(s - ref).max() / np.abs(ref).max() < 1e-5


def test_adjoint_tuner_and_group_option(lib):
    import torch
    w, inst = _gru_inst()
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    s, _ = lib.deer_solve(x, s0, p, cell="gru", offsets=inst.offsets, jac="diag", tol=1e-6)
    gs = 2 * s
    lib.load().pn_autotune_reset()
    t = lib.autotune("adjoint", x, s0, p, cell="gru", offsets=inst.offsets, s=s, gs=gs,
                     jac="diag")
    assert [(a, b) for a, b, _ in t["candidates"]] == [(0, g) for g in (0, 1, 2, 4, 8, 16)]
    assert all(m is not None and m > 0 for _, _, m in t["candidates"])
    ga = lib.deer_adjoint(x, s0, p, s, gs, cell="gru", offsets=inst.offsets, jac="diag",
                          tile="auto")
    gb = lib.deer_adjoint(x, s0, p, s, gs, cell="gru", offsets=inst.offsets, jac="diag",
                          group=t["group"])
    for a, b in zip(ga[:3], gb[:3]):
        assert torch.equal(a, b)
    # every group length gives the same gradients up to rounding
    g1 = lib.deer_adjoint(x, s0, p, s, gs, cell="gru", offsets=inst.offsets, jac="diag", group=1)
    g16 = lib.deer_adjoint(x, s0, p, s, gs, cell="gru", offsets=inst.offsets, jac="diag",
                           group=16)
    for a, b in zip(g1[:3], g16[:3]):
        a, b = a.cpu().double().numpy(), b.cpu().double().numpy()
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max())


def test_dense_adjoint_tuner_times_whole_calls(lib):
    """The GRU dense adjoint's group candidates are timed as whole calls; the chosen group and
    tile="auto" give the same gradients as an explicit call, every group the same up to
    rounding."""
    import torch
    w, inst = _gru_inst()
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    s, _ = lib.deer_solve(x, s0, p, cell="gru", offsets=inst.offsets, jac="diag", tol=1e-6)
    gs = 2 * s
    kw = dict(cell="gru", offsets=inst.offsets, jac="dense", compose="bf16", tol=1e-6)
    lib.load().pn_autotune_reset()
    t = lib.autotune("adjoint", x, s0, p, s=s, gs=gs, **kw)
    groups = (0, 1, 2, 3, 4, 5, 6, 8, 16)
    assert [(a, b) for a, b, _ in t["candidates"]] == [(0, g) for g in groups]
    assert all(m is not None and m > 0 for _, _, m in t["candidates"])
    assert t["group"] in groups
    ga = lib.deer_adjoint(x, s0, p, s, gs, tile="auto", **kw)
    gb = lib.deer_adjoint(x, s0, p, s, gs, group=t["group"], **kw)
    for a, b in zip(ga[:3], gb[:3]):
        assert torch.equal(a, b)
    g1 = lib.deer_adjoint(x, s0, p, s, gs, group=1, **kw)
    g16 = lib.deer_adjoint(x, s0, p, s, gs, group=16, **kw)
    for a, b in zip(g1[:3], g16[:3]):
        a, b = a.cpu().double().numpy(), b.cpu().double().numpy()
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max())


def test_elk_tuner_and_cache_file(lib, tmp_path, monkeypatch):
    w = workloads.TANH16_ELK.scaled(B=3, T=0)
    inst = workloads.make_instance(w, seed=42, lengths=np.array([900, 50, 1500]))
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PN_AUTOTUNE_CACHE", str(path))
    lib.load().pn_autotune_reset()
    t = lib.autotune("elk", x, s0, p, cell="tanh", offsets=inst.offsets, lam=0.1)
    assert [a for a, _, _ in t["candidates"]] == [0, 16, 32, 64, 128, 256]
    assert t["group"] == 0 and t["tile"] in (0, 16, 32, 64, 128, 256)
    entries = json.loads(path.read_text())
    assert len(entries) == 1
    key = next(iter(entries))
    assert entries[key] == [t["tile"], t["group"]] and "/op1/" in key
    # a fresh process state reads the file; the entry is taken as written
    other = 16 if t["tile"] != 16 else 32
    path.write_text(json.dumps({key: [other, 0]}))
    lib.load().pn_autotune_reset()
    with lib.profile():
        t2 = lib.autotune("elk", x, s0, p, cell="tanh", offsets=inst.offsets, lam=0.1)
        launches = lib.profile.read("elk_local")[1]
    assert t2["from_cache"] and t2["tile"] == other and launches == 0
    # lambda = 0 (the DEER passes) is another shape class
    t3 = lib.autotune("elk", x, s0, p, cell="tanh", offsets=inst.offsets, lam=0.0)
    assert not t3["from_cache"]
    assert len(json.loads(path.read_text())) == 2
    s, info = lib.elk_solve(x, s0, p, 0.1, cell="tanh", offsets=inst.offsets, tile="auto",
                            tol=1e-12, max_iters=3)
    s2, _ = lib.elk_solve(x, s0, p, 0.1, cell="tanh", offsets=inst.offsets, tile=other,
                          tol=1e-12, max_iters=3)
    assert (s.cpu().numpy() == s2.cpu().numpy()).all()
    lib.load().pn_autotune_reset()
