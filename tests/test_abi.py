"""The C ABI on the CPU: the library loads, exports every function pnewton.h declares, and
rejects invalid arguments before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2603_16850_amd as pn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnewton.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pn.LIB_PATH):
        pytest.skip("libpnewton.so not built")
    return pn.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"deer_solve", "elk_solve", "deer_adjoint", "pn_workspace_bytes"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in pn.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


def test_version_and_status_strings(lib):
    assert lib.pn_abi_version() == 1
    assert lib.pn_status_str(0) == b"PN_OK"
    assert lib.pn_status_str(-3) == b"PN_ERR_WORKSPACE"
    assert lib.pn_status_str(99) == b"unknown status"


def _desc(cell="gru", D=64, Dx=32, dtype="f32", params=1 << 20, B=2, N=200, offsets=None):
    c = pn.CellDesc(pn.CELLS.get(cell, 7), D, Dx, pn.DTYPES.get(dtype, 9), params)
    off = None if offsets is None else np.asarray(offsets, np.int64)
    b = pn.Batch(B, 0, N, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if off is not None else None)
    return c, b, off


def _ws(lib, op, c, b, o):
    n = ctypes.c_size_t(0)
    st = lib.pn_workspace_bytes(op, ctypes.byref(c), ctypes.byref(b), ctypes.byref(o), ctypes.byref(n))
    return st, n.value


def test_workspace_query_on_host(lib):
    o = pn.make_opts(jac="diag")
    c, b, _ = _desc()
    st, n = _ws(lib, pn.OP_DEER, c, b, o)
    assert st == 0 and n > 200 * 64 * 4
    st, n2 = _ws(lib, pn.OP_ADJOINT, c, b, o)
    assert st == 0 and n2 > 0
    c, b, _ = _desc(cell="tanh", D=32, Dx=16)
    st, _ = _ws(lib, pn.OP_DEER, c, b, pn.make_opts(jac="dense", compose="bf16"))
    assert st == 0
    # dense tanh adjoint: built undamped with dense Jacobians, FP32 or BF16 maps
    for comp in ("native", "bf16"):
        st, n3 = _ws(lib, pn.OP_ADJOINT, c, b, pn.make_opts(jac="dense", compose=comp))
        assert st == 0 and n3 > 2 * 200 * 32 * 4
    assert _ws(lib, pn.OP_ADJOINT, c, b, pn.make_opts(jac="diag"))[0] == -2
    assert _ws(lib, pn.OP_ADJOINT, c, b, pn.make_opts(jac="dense", damping="scale"))[0] == -2
    c, b, _ = _desc(cell="tanh", D=16, Dx=16)
    st, _ = _ws(lib, pn.OP_ELK, c, b, pn.make_opts(jac="dense"))
    assert st == 0


@pytest.mark.parametrize("kw,expect", [
    (dict(D=0), -1), (dict(Dx=0), -1), (dict(cell="bogus"), -1), (dict(dtype="f16"), -1),
    (dict(params=0), -1), (dict(B=0), -1), (dict(N=201), -1),          # N not divisible by B
    (dict(offsets=[0, 50, 40]), -1), (dict(offsets=[1, 100, 200]), -1),
    (dict(offsets=[0, 100, 150]), -1),                                  # offsets[B] != N
    (dict(D=40), -2), (dict(cell="tanh", D=64), -2),                   # valid but not built
])
def test_invalid_arguments_rejected_before_hip(lib, kw, expect):
    c, b, _keep = _desc(**kw)
    o = pn.make_opts(jac="diag")
    st = lib.deer_solve(ctypes.byref(c), ctypes.byref(b), ctypes.c_void_p(16), ctypes.c_void_p(16),
                        ctypes.c_void_p(16), ctypes.byref(o), None, 0, None, None)
    assert st == expect, (kw, st, lib.pn_last_error())
    assert lib.pn_last_error()


def test_bad_options_and_pointers(lib):
    c, b, _ = _desc()
    o = pn.make_opts(jac="diag")
    o.tol = -1.0
    args = (ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0, None, None) == -1
    o = pn.make_opts(jac="diag")
    o.jac = 5
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0, None, None) == -1
    o = pn.make_opts(jac="diag")
    # NULL and misaligned device pointers
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), None, *args[1:], ctypes.byref(o), None, 0, None, None) == -1
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), ctypes.c_void_p(18), *args[1:], ctypes.byref(o), None, 0, None, None) == -1
    # workspace missing / too small / misaligned
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0, None, None) == -3
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), ctypes.c_void_p(256), 10, None, None) == -3
    _, need = _ws(lib, pn.OP_DEER, c, b, o)
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), ctypes.c_void_p(260), need, None, None) == -3
    # ELK: negative lambda, unsupported shape
    c2, b2, _ = _desc(cell="tanh", D=16, Dx=16)
    assert lib.elk_solve(ctypes.byref(c2), ctypes.byref(b2), *args, ctypes.c_double(-1.0), ctypes.byref(o), None, 0, None, None) == -1
    c3, b3, _ = _desc(cell="tanh", D=32, Dx=16)
    assert lib.elk_solve(ctypes.byref(c3), ctypes.byref(b3), *args, ctypes.c_double(1.0), ctypes.byref(o), None, 0, None, None) == -2
    # adjoint needs gparams
    assert lib.deer_adjoint(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_void_p(16), None, None, None,
                            ctypes.byref(o), None, 0, None, None) == -1


def test_group_option_and_tuner_arguments(lib):
    """The group length option and pn_autotune's argument checks (no HIP call is made)."""
    c, b, _ = _desc()
    args = (ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    for g in (-1, 65):
        o = pn.make_opts(jac="diag", group=g)
        assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0,
                              None, None) == -1
    c2, b2, _ = _desc(cell="tanh", D=16, Dx=16)
    o = pn.make_opts(jac="dense", group=2)
    assert lib.elk_solve(ctypes.byref(c2), ctypes.byref(b2), *args, ctypes.c_double(0.1),
                         ctypes.byref(o), None, 0, None, None) == -1
    assert "tile" in lib.pn_last_error().decode()
    # tuning workspace: the largest candidate's plus a copy of the iterate (deer / elk)
    o = pn.make_opts(jac="diag")
    st, n = _ws(lib, pn.OP_DEER | pn.OP_TUNE, c, b, o)
    _, n1 = _ws(lib, pn.OP_DEER, c, b, o)
    assert st == 0 and n >= n1 + b.N * c.D * 4
    st, _ = _ws(lib, pn.OP_ADJOINT | pn.OP_TUNE, c, b, o)
    assert st == 0
    st, _ = _ws(lib, pn.OP_SEQ | pn.OP_TUNE, c, b, o)
    assert st == -1
    bufs = (ctypes.c_void_p * 7)(16, 16, 16, 16, 16, 16, 16)
    out = pn.Tuned()
    call = lambda op, probe=3, bb=bufs, ob=out: lib.pn_autotune(
        op, ctypes.byref(c), ctypes.byref(b), bb, ctypes.c_double(0.0), ctypes.byref(o), probe,
        None, 0, None, ctypes.byref(ob) if ob is not None else None)
    assert call(pn.OP_SEQ) == -1
    assert call(pn.OP_DEER, probe=65) == -1
    assert call(pn.OP_DEER, ob=None) == -1
    nulls = (ctypes.c_void_p * 7)(16, None, 16, 16, 16, 16, 16)
    assert call(pn.OP_DEER, bb=nulls) == -1


def test_binding_refuses_cpu_tensors():
    import torch
    x = torch.zeros(10, 8)
    with pytest.raises(ValueError):
        pn.deer_solve(x, torch.zeros(1, 16), torch.zeros(10))


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(ImportError):
        pn.load(str(tmp_path / "missing.so"))


def test_struct_sizes_match_header():
    assert ctypes.sizeof(pn.Opts) == 80
    assert ctypes.sizeof(pn.CellDesc) == 24 and ctypes.sizeof(pn.Batch) == 24
    assert ctypes.sizeof(pn.SeqInfo) == 24


@pytest.mark.parametrize("kw,expect", [
    (dict(damping="scale", damp_k=-0.1), -1), (dict(damping="scale", damp_k=1.5), -1),
    (dict(damping="clip", clip=(0.5, 0.2)), -1), (dict(damping="clip", clip=(-2.0, 1.0)), -1),
    (dict(damping="clip", jac="dense"), -1),
])
def test_damping_validation(lib, kw, expect):
    c, b, _ = _desc()
    o = pn.make_opts(**{"jac": "diag", **kw})
    args = (ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0,
                          None, None) == expect
    o = pn.make_opts(jac="diag")
    o.damping = 7
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0,
                          None, None) == -1


def test_damping_routes(lib):
    """Combinations that validate but are not built: clip on the dense tanh path is rejected
    as invalid (clip is diagonal only), damping on the FP64 dense GRU path and on ELK is
    unsupported, ELK with a Picard transition is unsupported."""
    args = (ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    c, b, _ = _desc(D=4, Dx=4, dtype="f64")
    o = pn.make_opts(jac="dense", damping="scale", damp_k=0.2)
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0,
                          None, None) == -2
    c, b, _ = _desc(cell="tanh", D=16, Dx=16)
    o = pn.make_opts(jac="dense", damping="scale", damp_k=0.2)
    assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                         ctypes.byref(o), None, 0, None, None) == -2
    o = pn.make_opts(jac="picard")
    assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                         ctypes.byref(o), None, 0, None, None) == -2
    o = pn.make_opts(jac="diag")
    o.freeze_prefix = 2
    assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                         ctypes.byref(o), None, 0, None, None) == -1
    o = pn.make_opts(jac="diag", freeze_prefix=True, smooth=True)   # not together
    assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                         ctypes.byref(o), None, 0, None, None) == -2
    o = pn.make_opts(jac="diag")
    o.smooth = 3
    assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                         ctypes.byref(o), None, 0, None, None) == -1
    o = pn.make_opts(jac="diag", smooth=True)                       # smoother: ELK only
    c3, b3, _ = _desc(D=64, Dx=32)
    assert lib.deer_solve(ctypes.byref(c3), ctypes.byref(b3), *args, ctypes.byref(o), None, 0,
                          None, None) == -2
    # converged-prefix skipping: ELK and the GRU diagonal path (fails later, on the missing
    # workspace); not on the dense tanh path, not with the update-norm rule
    o = pn.make_opts(jac="diag", freeze_prefix=True)
    c2, b2, _ = _desc(D=64, Dx=32)
    assert lib.deer_solve(ctypes.byref(c2), ctypes.byref(b2), *args, ctypes.byref(o), None, 0,
                          None, None) == -3
    o = pn.make_opts(jac="diag", freeze_prefix=True, stop="delta")
    assert lib.deer_solve(ctypes.byref(c2), ctypes.byref(b2), *args, ctypes.byref(o), None, 0,
                          None, None) == -2
    c4, b4, _ = _desc(cell="tanh", D=32, Dx=16)
    o = pn.make_opts(jac="dense", freeze_prefix=True)
    assert lib.deer_solve(ctypes.byref(c4), ctypes.byref(b4), *args, ctypes.byref(o), None, 0,
                          None, None) == -2
    for tile in (8, 24, 2048):          # ELK groups whole 16-step chunks, at most 64 of them
        o = pn.make_opts(jac="dense", tile=tile)
        assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                             ctypes.byref(o), None, 0, None, None) == -2
    # quasi-ELK and scale damping on the tanh dense path are built: they fail only later,
    # on the missing workspace
    o = pn.make_opts(jac="diag")
    assert lib.elk_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_double(1.0),
                         ctypes.byref(o), None, 0, None, None) == -3
    c, b, _ = _desc(cell="tanh", D=32, Dx=16)
    o = pn.make_opts(jac="dense", damping="scale", damp_k=0.2)
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0,
                          None, None) == -3


def test_stop_rule_and_input_check_options(lib):
    """pn_opts.stop and check_inputs: unknown values are invalid; the update-norm rule is
    built for the GRU diagonal path and the affine cells only; the input scan adds 256 bytes
    to the workspace."""
    args = (ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    c, b, _ = _desc()
    for field, bad in (("stop", 2), ("stop", -1), ("check_inputs", 2)):
        o = pn.make_opts(jac="diag")
        setattr(o, field, bad)
        assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None,
                              0, None, None) == -1
    o = pn.make_opts(jac="diag", stop="delta")            # built: fails on the workspace
    assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None, 0,
                          None, None) == -3
    ct, bt, _ = _desc(cell="tanh", D=32, Dx=16)
    o = pn.make_opts(jac="dense", stop="delta")
    assert lib.deer_solve(ctypes.byref(ct), ctypes.byref(bt), *args, ctypes.byref(o), None, 0,
                          None, None) == -2
    ce, be, _ = _desc(cell="tanh", D=16, Dx=16)
    assert lib.elk_solve(ctypes.byref(ce), ctypes.byref(be), *args, ctypes.c_double(0.1),
                         ctypes.byref(o), None, 0, None, None) == -2
    o = pn.make_opts(jac="diag", stop="delta")
    assert lib.deer_adjoint(ctypes.byref(c), ctypes.byref(b), *args, ctypes.c_void_p(16),
                            None, None, ctypes.c_void_p(16), ctypes.byref(o), None, 0, None,
                            None) == -2
    for op in (pn.OP_DEER, pn.OP_ADJOINT):
        _, n0 = _ws(lib, op, c, b, pn.make_opts(jac="diag"))
        st, n1 = _ws(lib, op, c, b, pn.make_opts(jac="diag", check_inputs=True))
        assert st == 0 and n1 == ((n0 + 255) // 256) * 256 + 256


@pytest.mark.parametrize("cell", ["affine", "affine_steps"])
def test_affine_cells_are_routed(lib, cell):
    """The affine test cells: every transition mode is built for D <= 16 in FP32 (the calls
    fail only on the missing workspace); D > 16, FP64 and damping are not built."""
    args = (ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16))
    for jac in ("dense", "diag", "picard", "jacobi"):
        for D in (1, 5, 16):
            c, b, _ = _desc(cell=cell, D=D, Dx=3)
            o = pn.make_opts(jac=jac)
            st, n = _ws(lib, pn.OP_DEER, c, b, o)
            assert st == 0 and n > 0
            assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o),
                                  None, 0, None, None) == -3
    for kw, mo in ((dict(D=17), {}), (dict(D=4, dtype="f64"), {}),
                   (dict(D=4), dict(damping="scale", damp_k=0.5))):
        c, b, _ = _desc(cell=cell, Dx=3, **kw)
        o = pn.make_opts(jac="dense", **mo)
        assert lib.deer_solve(ctypes.byref(c), ctypes.byref(b), *args, ctypes.byref(o), None,
                              0, None, None) == -2


def test_binding_checks_shapes_before_any_call():
    """The binding checks the tensors against the shapes the C call assumes (the library sees
    only pointers): offsets against x, s0, the packed parameter count, dtypes and devices,
    and the [N, D] arrays."""
    import torch
    f32 = torch.float32       # explicit: another test module changes torch's default dtype
    x = torch.zeros(100, 8, dtype=f32)
    s0 = torch.zeros(2, 16, dtype=f32)
    p = torch.zeros(pn.param_count("gru", 16, 8), dtype=f32)
    sh = pn._shapes("gru", p, x, s0, [0, 40, 100])
    assert sh.batch.B == 2 and sh.batch.N == 100
    bad = [
        dict(offsets=[0, 40, 99]),                    # offsets[-1] != N
        dict(offsets=[0, 100]),                       # B + 1 entries
        dict(offsets=[0, 60, 40, 100]),               # wrong count and decreasing
        dict(offsets=None, x=torch.zeros(101, 8, dtype=f32)),   # N not split into B
        dict(params=torch.zeros(p.numel() - 1, dtype=f32)),     # parameter count
        dict(s0=torch.zeros(2, 16, dtype=torch.float64)),
        dict(cell="bogus"),
        dict(rows=[(torch.zeros(100, 15, dtype=f32), "s", 16)]),
        dict(rows=[(torch.zeros(100, 16, dtype=torch.float64), "gs", 16)]),
    ]
    for kw in bad:
        args = dict(cell="gru", params=p, x=x, s0=s0, offsets=[0, 40, 100])
        args.update(kw)
        rows = args.pop("rows", ())
        with pytest.raises(ValueError):
            pn._shapes(args["cell"], args["params"], args["x"], args["s0"], args["offsets"],
                       rows=rows)
    # the per-step affine cell packs one matrix per row
    assert pn.param_count("affine_steps", 3, 2, N=10) == 10 * 9 + 6 + 3
    assert pn.param_count("affine", 3, 2) == 9 + 6 + 3


def test_copy_probe_rejects_bad_arguments(lib):
    """pn_copy_probe validates before any HIP call: NULL pointers, sizes that are not a positive
    multiple of 16, misaligned pointers and reps < 1 are PN_ERR_INVALID_ARG."""
    out = ctypes.c_double(-1.0)
    ok = ctypes.c_void_p(1 << 20)
    bad = [
        (None, ok, 1024, 1, ctypes.byref(out)),
        (ok, None, 1024, 1, ctypes.byref(out)),
        (ok, ok, 1024, 1, None),
        (ok, ok, 0, 1, ctypes.byref(out)),
        (ok, ok, 1000, 1, ctypes.byref(out)),
        (ctypes.c_void_p((1 << 20) + 4), ok, 1024, 1, ctypes.byref(out)),
        (ok, ctypes.c_void_p((1 << 20) + 8), 1024, 1, ctypes.byref(out)),
        (ok, ok, 1024, 0, ctypes.byref(out)),
    ]
    for src, dst, nbytes, reps, gbs in bad:
        assert lib.pn_copy_probe(src, dst, nbytes, reps, None, gbs) == -1
        assert b"pn_copy_probe" in lib.pn_last_error()
    assert out.value == -1.0
