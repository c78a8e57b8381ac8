"""GPU: deer_solve_noalloc (the entry point for callers that cannot allocate) against
deer_solve on the same inputs, through the C ABI: two calls in a row, the second with a
smaller input (the static scratch keeps the first call's contents), each compared with a
deer_solve call bit for bit (the same kernels; deer_solve with plain launches)."""
import ctypes

import numpy as np
import pytest

from paper_2603_16850_amd import workloads

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(a, dtype=torch.float32, device="cuda")


def _call(pn, fn, inst, cell, opts_kw):
    import torch
    x, s0, p = _t(inst.x), _t(inst.s0), _t(inst.params)
    sh = pn._shapes(cell, p, x, s0, inst.offsets)
    opts = pn.make_opts(**opts_kw)
    s = torch.zeros(inst.x.shape[0], s0.shape[1], dtype=torch.float32, device="cuda")
    info = (pn.SeqInfo * sh.batch.B)()
    L = pn.load()
    if fn == "noalloc":
        st = L.deer_solve_noalloc(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                                  pn._ptr(s0), pn._ptr(s), ctypes.byref(opts), pn._stream(), info)
    else:
        ws, nb = pn._workspace(pn.OP_DEER, sh, opts, x.device)
        st = L.deer_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), pn._ptr(x),
                          pn._ptr(s0), pn._ptr(s), ctypes.byref(opts), pn._aligned(ws), nb,
                          pn._stream(), info)
    assert st >= 0, L.pn_last_error()
    torch.cuda.synchronize()
    return s.cpu().numpy(), [(i.iters, i.converged, i.resets) for i in info]


@pytest.mark.parametrize("case", ["gru", "affine_steps"])
def test_noalloc_matches_deer_solve(lib, case):
    if case == "gru":
        w = workloads.GRU48_RAGGED.scaled(B=3, T=0)
        big = workloads.make_instance(w, seed=90, lengths=np.array([1500, 1, 700]))
        small = workloads.make_instance(w, seed=91, lengths=np.array([300, 80]))
        kw = dict(jac="diag", tol=1e-6)
        cell = "gru"
    else:
        rng = np.random.default_rng(92)

        def s5(lens):
            off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
            N = int(off[-1])
            Mt = np.zeros((N, 5, 5))
            for n in range(N):
                Mt[n, np.arange(5), rng.permutation(5)] = 1.0
            wk = workloads.Workload("s5", "affine_steps", D=5, Dx=1, B=len(lens))
            return workloads.Instance(wk, np.concatenate([Mt.ravel(), np.zeros(10)]),
                                      np.zeros((N, 1)), np.tile(np.arange(1.0, 6.0),
                                                                (len(lens), 1)), off)
        big, small = s5([200, 64]), s5([40])
        kw = dict(jac="dense", tol=0.5)
        cell = "affine_steps"
    for inst in (big, small):          # the second, smaller call reuses the dirty scratch
        got, gi = _call(lib, "noalloc", inst, cell, kw)
        want, wi = _call(lib, "ws", inst, cell, dict(kw, use_graph=False))
        assert gi == wi
        assert np.array_equal(got, want)
        assert all(c for _, c, _ in gi)


def test_noalloc_rejects_shapes_beyond_its_scratch(lib):
    import torch
    w = workloads.GRU64_QUASI
    N = 1 << 20                        # needs far more than the static scratch
    f32 = torch.float32      # explicit: another test module changes torch's default dtype
    x = torch.zeros(N, w.Dx, dtype=f32, device="cuda")
    s0 = torch.zeros(16, w.D, dtype=f32, device="cuda")
    p = torch.zeros(lib.param_count("gru", w.D, w.Dx), dtype=f32, device="cuda")
    s = torch.zeros(N, w.D, dtype=f32, device="cuda")
    sh = lib._shapes("gru", p, x, s0, None)
    opts = lib.make_opts(jac="diag")
    st = lib.load().deer_solve_noalloc(ctypes.byref(sh.cell), ctypes.byref(sh.batch),
                                       lib._ptr(x), lib._ptr(s0), lib._ptr(s),
                                       ctypes.byref(opts), lib._stream(), None)
    assert st == -3
    assert b"static scratch" in lib.load().pn_last_error()
