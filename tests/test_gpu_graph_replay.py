"""GPU: replays of the captured iteration graphs against plain launches.

The iteration loop captures `graph_iters` iterations in a hipGraph once per argument set and
replays it for every later batch and call.  Each case calls the C ABI with fixed buffers, so
that the same instantiated graph serves every call, three times with unrelated eager work and
synchronisations between the calls, and checks every result bit for bit against the same call
made with plain launches (use_graph = 0).
"""
import ctypes

import numpy as np
import pytest

from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _eager_noise():
    """Unrelated eager work on the same stream: fills, a product, a reduction."""
    import torch
    a = torch.randn(512, 512, device="cuda")
    b = (a @ a.t()).sum()
    torch.zeros(1 << 20, device="cuda").fill_(3.0)
    torch.cuda.synchronize()
    return float(b)


def _run_fixed(lib, op, cell, inst, w, opts_kw, lam=0.0, s_traj=None):
    """Three graph-replayed calls and one plain-launch call on the same fixed buffers."""
    import torch
    pn = lib
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    sh = pn._shapes(cell, p, x, s0, inst.offsets)
    outs = []
    for use_graph in (True, True, True, False):
        opts = pn.make_opts(use_graph=use_graph, **opts_kw)
        if not outs:
            ws, nb = pn._workspace(op, sh, opts, x.device)
            s = torch.zeros(inst.x.shape[0], w.D, device="cuda")
            gx, g0, gp = torch.empty_like(x), torch.empty_like(s0), torch.empty_like(p)
        info = (pn.SeqInfo * sh.batch.B)()
        L = pn.load()
        if op == pn.OP_DEER:
            s.zero_()
            st = L.deer_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                              pn._ptr(s0), pn._ptr(s), ctypes.byref(opts), pn._aligned(ws), nb,
                              pn._stream(), info)
            res = [s.clone()]
        elif op == pn.OP_ELK:
            s.zero_()
            st = L.elk_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                             pn._ptr(s0), pn._ptr(s), ctypes.c_double(lam), ctypes.byref(opts),
                             pn._aligned(ws), nb, pn._stream(), info)
            res = [s.clone()]
        else:
            gs = 2.0 * s_traj
            st = L.deer_adjoint(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                                pn._ptr(s0), pn._ptr(s_traj), pn._ptr(gs), pn._ptr(gx),
                                pn._ptr(g0), pn._ptr(gp), ctypes.byref(opts), pn._aligned(ws),
                                nb, pn._stream(), info)
            res = [gx.clone(), g0.clone(), gp.clone()]
        assert st >= 0, pn.load().pn_last_error()
        outs.append(([r.cpu().numpy() for r in res], [i.iters for i in info]))
        _eager_noise()
    ref, ref_it = outs[-1]
    for got, it in outs[:-1]:
        assert it == ref_it
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    return ref_it


def test_replay_gru_quasi(lib):
    w = workloads.GRU48_RAGGED.scaled(B=5, T=0)
    inst = workloads.make_instance(w, seed=51, lengths=np.array([900, 64, 1, 2000, 333]))
    _run_fixed(lib, lib.OP_DEER, "gru", inst, w,
               dict(jac="diag", tol=1e-6, graph_iters=3, max_iters=12))


def test_replay_gru_adjoint(lib):
    w = workloads.GRU48_RAGGED.scaled(B=4, T=0)
    inst = workloads.make_instance(w, seed=52, lengths=np.array([700, 1, 1500, 90]))
    s, _ = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="gru",
                          offsets=inst.offsets, jac="diag", tol=1e-6)
    _run_fixed(lib, lib.OP_ADJOINT, "gru", inst, w,
               dict(jac="diag", tol=1e-6, graph_iters=2), s_traj=s)


@pytest.mark.parametrize("compose", ["bf16", "native"])
def test_replay_tanh_adjoint(lib, compose):
    w = workloads.TANH32_DENSE_BF16.scaled(B=3, T=0)
    inst = workloads.make_instance(w, seed=55, lengths=np.array([1000, 37, 2100]))
    s, _ = lib.deer_solve(_t(inst.x), _t(inst.s0), _t(inst.params), cell="tanh",
                          offsets=inst.offsets, jac="dense", tol=1e-6)
    _run_fixed(lib, lib.OP_ADJOINT, "tanh", inst, w,
               dict(jac="dense", compose=compose, tol=1e-6, graph_iters=2, group=2), s_traj=s)


@pytest.mark.parametrize("compose", ["bf16", "native"])
def test_replay_tanh_dense(lib, compose):
    w = workloads.TANH32_DENSE_BF16.scaled(B=3, T=0)
    inst = workloads.make_instance(w, seed=53, lengths=np.array([1000, 37, 2100]))
    _run_fixed(lib, lib.OP_DEER, "tanh", inst, w,
               dict(jac="dense", compose=compose, tol=1e-6, graph_iters=2))


@pytest.mark.parametrize("lam,jac,tile", [(0.1, "dense", 32), (0.1, "diag", 0), (0.0, "dense", 16),
                                          (0.0, "diag", 0)])
def test_replay_elk(lib, lam, jac, tile):
    """ELK (three-phase carry at tile 32), quasi-ELK, DEER with the segmented carry (tile
    16: 94 groups in the longest sequence), quasi-DEER."""
    w = workloads.TANH16_ELK.scaled(B=3, T=0, gain=0.9)
    inst = workloads.make_instance(w, seed=54, lengths=np.array([1500, 20, 700]))
    _run_fixed(lib, lib.OP_ELK, "tanh", inst, w,
               dict(jac=jac, tol=1e-6, graph_iters=4, max_iters=16, tile=tile), lam=lam)


def _solve_fixed(lib, op, cell, x, s0, p, s, ws, offsets, opts_kw, lam=0.0):
    """One solve through the C ABI on caller-held buffers (views of fixed allocations), with
    graph capture on, then the same with plain launches; returns both iterates and counts."""
    import torch
    pn = lib
    sh = pn._shapes(cell, p, x, s0, offsets)
    out = []
    for use_graph in (True, False):
        opts = pn.make_opts(use_graph=use_graph, **opts_kw)
        need = ctypes.c_size_t(0)
        assert pn.load().pn_workspace_bytes(op, ctypes.byref(sh.cell), ctypes.byref(sh.batch),
                                            ctypes.byref(opts), ctypes.byref(need)) == 0
        assert need.value + 256 <= ws.numel()
        info = (pn.SeqInfo * sh.batch.B)()
        s.zero_()
        if op == pn.OP_DEER:
            st = pn.load().deer_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                                      pn._ptr(s0), pn._ptr(s), ctypes.byref(opts),
                                      pn._aligned(ws), need.value, pn._stream(), info)
        else:
            st = pn.load().elk_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                                     pn._ptr(s0), pn._ptr(s), ctypes.c_double(lam),
                                     ctypes.byref(opts), pn._aligned(ws), need.value,
                                     pn._stream(), info)
        assert st >= 0, pn.load().pn_last_error()
        torch.cuda.synchronize()
        out.append((s.cpu().numpy().copy(), [i.iters for i in info]))
        _eager_noise()
    (sg, ig), (sp, ip) = out
    assert ig == ip
    assert np.array_equal(sg, sp)
    return sg


def test_replay_same_buffers_other_length(lib):
    """The same buffers (views at the same addresses, the same workspace pointer) called with
    two lengths that give the same tile and group counts (B = 1, T = 1000 and 1010 at 64-step
    tiles): the workspace offsets of the second call differ, and its graph-launched result
    must still equal its plain launches bit for bit."""
    import torch
    w = workloads.GRU48_RAGGED.scaled(B=1, T=0)
    inst = workloads.make_instance(w, seed=56, lengths=np.array([1010]))
    X, S0, P = _t(inst.x), _t(inst.s0), _t(inst.params)
    S = torch.zeros(1010, w.D, device="cuda")
    WS = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    res = {}
    for T in (1000, 1010, 1000):
        res[T] = _solve_fixed(lib, lib.OP_DEER, "gru", X[:T], S0, P, S[:T], WS,
                              np.array([0, T]), dict(jac="diag", tol=1e-6, graph_iters=3,
                                                     tile=64, group=4))
    assert not np.array_equal(res[1000][:1000], np.zeros((1000, w.D)))


def test_replay_elk_same_tiles_other_longest_sequence(lib):
    """ELK on fixed buffers with two ragged batches of the same total length, chunk count
    and group count but a different longest sequence (10 and 18 groups): the carry plan of
    the second differs, and graph launches must still equal plain launches."""
    import torch
    w = workloads.TANH16_ELK.scaled(B=2, T=0, gain=0.9)
    inst = workloads.make_instance(w, seed=57, lengths=np.array([320, 320]))
    X, S0, P = _t(inst.x), _t(inst.s0), _t(inst.params)
    S = torch.zeros(640, w.D, device="cuda")
    WS = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    for lens in ((320, 320), (64, 576), (320, 320)):
        off = np.concatenate([[0], np.cumsum(lens)])
        _solve_fixed(lib, lib.OP_ELK, "tanh", X, S0, P, S, WS, off,
                     dict(jac="dense", tol=1e-6, graph_iters=4, max_iters=12, tile=32), lam=0.1)


def test_two_threads_evicting_the_graph_cache(lib):
    """Two host threads solve on their own buffers with 40 different lengths each, so that the
    process-wide cache of instantiated iteration graphs (64 entries) evicts while the other
    thread looks up, updates and launches its own executables; every result equals the same
    solve made alone beforehand, bit for bit."""
    import threading
    import torch
    w = workloads.GRU48_RAGGED.scaled(B=1, T=0)
    lens = {0: list(range(100, 140)), 1: list(range(200, 240))}
    kw = dict(cell="gru", jac="diag", tol=1e-6, graph_iters=2, tile=32, group=2)
    inputs = {}
    for k, ls in lens.items():
        for T in ls:
            inst = workloads.make_instance(w, seed=600 + T, lengths=np.array([T]))
            inputs[(k, T)] = (_t(inst.x), _t(inst.s0), _t(inst.params), inst.offsets)
    want = {}
    for key, (x, s0, p, off) in inputs.items():
        s, info = lib.deer_solve(x, s0, p, offsets=off, **kw)
        want[key] = (s.cpu().numpy(), info[0]["iters"])
    torch.cuda.synchronize()
    got, errors = {}, []

    def work(k):
        try:
            for T in lens[k]:
                x, s0, p, off = inputs[(k, T)]
                s, info = lib.deer_solve(x, s0, p, offsets=off, **kw)
                torch.cuda.current_stream().synchronize()
                got[(k, T)] = (s.cpu().numpy(), info[0]["iters"])
        except Exception as e:      # reported by the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(k,)) for k in lens]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    assert set(got) == set(want)
    for key in want:
        assert got[key][1] == want[key][1], key
        assert np.array_equal(got[key][0], want[key][0]), key
