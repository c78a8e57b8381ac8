"""MI355X parallel Newton methods (DEER, quasi-DEER, ELK) -- Python binding.

Thin ctypes layer over ``libpnewton.so`` (the C ABI declared in ``include/pnewton.h``):
it marshals torch tensors (device memory and streams only) into the C calls, allocates the
workspace the library asks for, and wraps the solve + adjoint in a torch.autograd.Function.
Every step of the method runs in the library's HIP kernels; there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpnewton.so")

PN_OK, PN_NOT_CONVERGED = 0, 1
CELLS = {"gru": 0, "tanh": 1, "meanfield": 2, "affine": 3, "affine_steps": 4}
JACS = {"dense": 0, "diag": 1, "picard": 2, "jacobi": 3}
DTYPES = {"f32": 0, "f64": 1}
COMPOSE = {"native": 0, "bf16": 1}
STOPS = {"resid": 0, "delta": 1}
OP_DEER, OP_ELK, OP_ADJOINT, OP_RESIDUAL64, OP_SEQ, OP_LLE = 0, 1, 2, 3, 4, 5


class CellDesc(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32), ("D", ctypes.c_int32), ("Dx", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("params", ctypes.c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("pad_", ctypes.c_int32), ("N", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int64))]


class Opts(ctypes.Structure):
    _fields_ = [("jac", ctypes.c_int32), ("compose", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iters", ctypes.c_int32), ("graph_iters", ctypes.c_int32),
                ("reset_abs", ctypes.c_double), ("fp64_final_residual", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("damping", ctypes.c_int32), ("damp_k", ctypes.c_float),
                ("clip_lo", ctypes.c_float), ("clip_hi", ctypes.c_float),
                ("freeze_prefix", ctypes.c_int32), ("smooth", ctypes.c_int32),
                ("group", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("check_inputs", ctypes.c_int32)]


TUNE_MAX_CAND = 32
OP_TUNE = 0x100


class Tuned(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("group", ctypes.c_int32),
                ("ms_per_iter", ctypes.c_double), ("from_cache", ctypes.c_int32),
                ("ncand", ctypes.c_int32), ("cand_tile", ctypes.c_int32 * TUNE_MAX_CAND),
                ("cand_group", ctypes.c_int32 * TUNE_MAX_CAND),
                ("cand_ms", ctypes.c_float * TUNE_MAX_CAND)]


class SeqInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("resets", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("max_resid", ctypes.c_double)]


# (name, restype, argtypes) of every symbol the header declares
_P, _V = ctypes.POINTER, ctypes.c_void_p
SIGNATURES = [
    ("pn_default_opts", None, [_P(Opts)]),
    ("pn_workspace_bytes", ctypes.c_int, [ctypes.c_int, _P(CellDesc), _P(Batch), _P(Opts),
                                          _P(ctypes.c_size_t)]),
    ("deer_solve", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _P(Opts), _V,
                                  ctypes.c_size_t, _V, _P(SeqInfo)]),
    ("deer_solve_noalloc", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _P(Opts), _V,
                                          _P(SeqInfo)]),
    ("elk_solve", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, ctypes.c_double,
                                 _P(Opts), _V, ctypes.c_size_t, _V, _P(SeqInfo)]),
    ("deer_adjoint", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _V, _V, _V, _V,
                                    _P(Opts), _V, ctypes.c_size_t, _V, _P(SeqInfo)]),
    ("seq_rollout", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _V, ctypes.c_size_t,
                                   _V]),
    ("seq_bptt", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _V, _V, _V, _V, _V,
                                ctypes.c_size_t, _V]),
    ("pn_residual_f64", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _V,
                                       ctypes.c_size_t, _V, _P(ctypes.c_double)]),
    ("pn_lle_estimate", ctypes.c_int, [_P(CellDesc), _P(Batch), _V, _V, _V, _V, _V,
                                       ctypes.c_size_t, _V, _P(ctypes.c_double)]),
    ("pn_autotune", ctypes.c_int, [ctypes.c_int, _P(CellDesc), _P(Batch), _P(_V),
                                   ctypes.c_double, _P(Opts), ctypes.c_int32, _V,
                                   ctypes.c_size_t, _V, _P(Tuned)]),
    ("pn_autotune_reset", None, []),
    ("pn_copy_probe", ctypes.c_int, [_V, _V, ctypes.c_size_t, ctypes.c_int, _V,
                                     _P(ctypes.c_double)]),
    ("pn_profile_begin", None, []),
    ("pn_profile_end", None, []),
    ("pn_profile_read", ctypes.c_int, [ctypes.c_char_p, _P(ctypes.c_double),
                                       _P(ctypes.c_int64)]),
    ("pn_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("pn_last_error", ctypes.c_char_p, []),
    ("pn_abi_version", ctypes.c_int, []),
]

_lib = None


def load(path=None):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python -m paper_2603_16850_amd.build`")
    lib = ctypes.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.pn_abi_version() != 1:
        raise ImportError("libpnewton ABI version mismatch")
    if path is None:
        _lib = lib
    return lib


class PNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(status):
    if status < 0:
        lib = load()
        raise PNError(status, f"{lib.pn_status_str(status).decode()}: "
                              f"{lib.pn_last_error().decode()}")
    return status


# ---- marshalling helpers ---------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_name(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return "f32"
    if t.dtype == torch.float64:
        return "f64"
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


DAMPING = {"none": 0, "scale": 1, "clip": 2}


def make_opts(jac="diag", compose="native", tol=1e-5, max_iters=0, graph_iters=4,
              reset_abs=1e4, fp64_final_residual=False, use_graph=True, tile=0,
              damping="none", damp_k=0.0, clip=(-1.0, 1.0), freeze_prefix=False,
              smooth=False, group=0, stop="resid", check_inputs=False):
    """pn_opts; damping "scale" (scale-ELK, A~ <- (1 - damp_k) A~) or "clip" (clip-ELK,
    diagonal A~ clipped to `clip`); stop "resid" (max |r| < tol) or "delta" (max update <
    tol); check_inputs scans the inputs for NaN / infinity first."""
    o = Opts()
    load().pn_default_opts(ctypes.byref(o))
    o.damping = DAMPING[damping]
    o.damp_k = float(damp_k)
    o.clip_lo, o.clip_hi = float(clip[0]), float(clip[1])
    o.jac = JACS[jac]
    o.compose = COMPOSE[compose]
    o.tol = float(tol)
    o.max_iters = int(max_iters)
    o.graph_iters = int(graph_iters)
    o.reset_abs = float(reset_abs)
    o.fp64_final_residual = int(bool(fp64_final_residual))
    o.use_graph = int(bool(use_graph))
    o.tile = int(tile)
    o.freeze_prefix = int(bool(freeze_prefix))
    o.smooth = int(bool(smooth))
    o.group = int(group)
    o.stop = STOPS[stop]
    o.check_inputs = int(bool(check_inputs))
    return o


class _Shapes:
    """CellDesc + Batch for one call; keeps the host offsets array alive."""

    def __init__(self, cell, params, D, Dx, dtype, B, N, offsets):
        self.cell = CellDesc(CELLS[cell], int(D), int(Dx), DTYPES[dtype], params.data_ptr())
        self.off = None
        if offsets is not None:
            self.off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
            B = self.off.size - 1
            N = int(self.off[-1])
        self.batch = Batch(int(B), 0, int(N),
                           self.off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                           if self.off is not None else None)


def param_count(cell, D, Dx, N=0):
    """Packed parameter count of a cell (the per-step affine cell holds N matrices)."""
    if cell == "gru":
        return 3 * D * Dx + 3 * D * D + 4 * D
    if cell == "affine_steps":
        return N * D * D + D * Dx + D
    return D * D + D * Dx + D


def _shapes(cell, params, x, s0, offsets, rows=()):
    """Checks every tensor of a call against the shapes the C call will assume (the library
    sees only pointers, so a mismatch here would become an out-of-bounds access there) and
    builds its descriptors.  `rows`: further (tensor, name, columns) of shape [N, columns]."""
    if cell not in CELLS:
        raise ValueError(f"unknown cell {cell!r}")
    if x.dim() != 2 or s0.dim() != 2:
        raise ValueError("x must be [N, Dx] and s0 [B, D]")
    N, Dx = x.shape
    B, D = s0.shape
    if offsets is not None:
        off = np.asarray(offsets)
        if off.ndim != 1 or off.size != B + 1:
            raise ValueError(f"offsets must hold B + 1 = {B + 1} entries, got {off.size}")
        if off[0] != 0 or np.any(np.diff(off) < 0):
            raise ValueError("offsets must start at 0 and be non-decreasing")
        if int(off[-1]) != N:
            raise ValueError(f"offsets[-1] = {int(off[-1])} differs from x.shape[0] = {N}")
    elif B < 1 or N % B:
        raise ValueError(f"N = {N} steps do not split into B = {B} equal sequences")
    want = param_count(cell, D, Dx, N)
    if params.numel() != want:
        raise ValueError(f"params holds {params.numel()} values; the {cell} cell with D = {D}, "
                         f"Dx = {Dx} packs {want}")
    for t, n in ((s0, "s0"), (params, "params")):
        if t.dtype != x.dtype or t.device != x.device:
            raise ValueError(f"{n} must have the dtype and device of x")
    for t, n, cols in rows:
        if t is None:
            continue
        if tuple(t.shape) != (N, cols):
            raise ValueError(f"{n} must be [{N}, {cols}], got {list(t.shape)}")
        if t.dtype != x.dtype or t.device != x.device:
            raise ValueError(f"{n} must have the dtype and device of x")
        _dev(t, n)
    return _Shapes(cell, params, D, Dx, _dtype_name(x), B, N, offsets)


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(op, sh, opts, device):
    torch = _torch()
    nbytes = ctypes.c_size_t(0)
    _check(load().pn_workspace_bytes(op, ctypes.byref(sh.cell), ctypes.byref(sh.batch),
                                     ctypes.byref(opts), ctypes.byref(nbytes)))
    n = max(int(nbytes.value), 1)
    return torch.empty(n + 256, dtype=torch.uint8, device=device), int(nbytes.value)


def _aligned(ws):
    p = ws.data_ptr()
    return ctypes.c_void_p((p + 255) & ~255)


def _infos(arr):
    return [dict(iters=i.iters, converged=bool(i.converged), resets=i.resets,
                 max_resid=i.max_resid) for i in arr]


# ---- public functions (names follow the C ABI) ------------------------------------------------

_OPS = {"deer": OP_DEER, "elk": OP_ELK, "adjoint": OP_ADJOINT}


def autotune(op, x, s0, params, cell="gru", offsets=None, lam=0.0, s=None, gs=None,
             probe_iters=3, **opt_kw):
    """pn_autotune: the fastest (tile, group) of `op` ("deer", "elk" or "adjoint") for these
    inputs and options.  For "deer" / "elk", `s` (default zeros) is the initial guess the
    probes start from and is left unchanged; for "adjoint", `s` is the trajectory and `gs`
    the loss gradient.  Returns dict(tile, group, ms_per_iter, from_cache, candidates =
    [(tile, group, ms per iteration or None if rejected)])."""
    torch = _torch()
    code = _OPS[op]
    for t, n in ((x, "x"), (s0, "s0"), (params, "params")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets)
    if op == "elk":
        opt_kw.setdefault("jac", "dense")
    opts = make_opts(**opt_kw)
    if s is None:
        s = torch.zeros((x.shape[0], s0.shape[1]), dtype=x.dtype, device=x.device)
    _dev(s, "s")
    keep = []
    if op == "adjoint":
        _dev(gs, "gs")
        keep = [torch.empty_like(x), torch.empty_like(s0), torch.empty_like(params)]
        ptrs = [x, s0, s, gs] + keep
    else:
        ptrs = [x, s0, s]
    bufs = (_V * len(ptrs))(*[t.data_ptr() for t in ptrs])
    ws, nb = _workspace(code | OP_TUNE, sh, opts, x.device)
    out = Tuned()
    _check(load().pn_autotune(code, ctypes.byref(sh.cell), ctypes.byref(sh.batch), bufs,
                              ctypes.c_double(lam), ctypes.byref(opts), int(probe_iters),
                              _aligned(ws), nb, _stream(), ctypes.byref(out)))
    cands = [(out.cand_tile[i], out.cand_group[i],
              None if out.cand_ms[i] < 0 else float(out.cand_ms[i])) for i in range(out.ncand)]
    return dict(tile=out.tile, group=out.group, ms_per_iter=out.ms_per_iter,
                from_cache=bool(out.from_cache), candidates=cands)


def _auto_tile(op, opt_kw, x, s0, params, cell, offsets, **extra):
    """tile="auto": the autotuned (tile, group) replace the two options."""
    if opt_kw.get("tile") != "auto":
        return opt_kw
    kw = dict(opt_kw)
    kw.pop("tile")
    kw.pop("group", None)
    t = autotune(op, x, s0, params, cell=cell, offsets=offsets, **extra, **kw)
    kw["tile"], kw["group"] = t["tile"], t["group"]
    return kw

def deer_solve(x, s0, params, cell="gru", offsets=None, s_init=None, **opt_kw):
    """DEER / quasi-DEER solve; returns (s [N, D], per-sequence info list)."""
    torch = _torch()
    for t, n in ((x, "x"), (s0, "s0"), (params, "params")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets, rows=[(s_init, "s_init", s0.shape[1])])
    opts = make_opts(**_auto_tile("deer", opt_kw, x, s0, params, cell, offsets, s=s_init))
    s = (torch.zeros((x.shape[0], s0.shape[1]), dtype=x.dtype, device=x.device)
         if s_init is None else _dev(s_init, "s_init").clone())
    ws, nb = _workspace(OP_DEER, sh, opts, x.device)
    info = (SeqInfo * sh.batch.B)()
    st = _check(load().deer_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x),
                                  _ptr(s0), _ptr(s), ctypes.byref(opts), _aligned(ws), nb,
                                  _stream(), info))
    return s, _infos(info)


def elk_solve(x, s0, params, lam, cell="tanh", offsets=None, s_init=None, **opt_kw):
    torch = _torch()
    for t, n in ((x, "x"), (s0, "s0"), (params, "params")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets, rows=[(s_init, "s_init", s0.shape[1])])
    opt_kw.setdefault("jac", "dense")
    opts = make_opts(**_auto_tile("elk", opt_kw, x, s0, params, cell, offsets, lam=lam,
                                  s=s_init))
    s = (torch.zeros((x.shape[0], s0.shape[1]), dtype=x.dtype, device=x.device)
         if s_init is None else _dev(s_init, "s_init").clone())
    ws, nb = _workspace(OP_ELK, sh, opts, x.device)
    info = (SeqInfo * sh.batch.B)()
    _check(load().elk_solve(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x), _ptr(s0),
                            _ptr(s), ctypes.c_double(lam), ctypes.byref(opts), _aligned(ws), nb,
                            _stream(), info))
    return s, _infos(info)


def deer_adjoint(x, s0, params, s, gs, cell="gru", offsets=None, need_gx=True, need_gs0=True,
                 **opt_kw):
    """Returns (gparams, gx, gs0, info)."""
    torch = _torch()
    for t, n in ((x, "x"), (s0, "s0"), (params, "params"), (s, "s"), (gs, "gs")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets, rows=[(s, "s", s0.shape[1]),
                                                     (gs, "gs", s0.shape[1])])
    opts = make_opts(**_auto_tile("adjoint", opt_kw, x, s0, params, cell, offsets, s=s, gs=gs))
    gp = torch.empty_like(params)
    gx = torch.empty_like(x) if need_gx else None
    g0 = torch.empty_like(s0) if need_gs0 else None
    ws, nb = _workspace(OP_ADJOINT, sh, opts, x.device)
    info = (SeqInfo * sh.batch.B)()
    _check(load().deer_adjoint(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x), _ptr(s0),
                               _ptr(s), _ptr(gs), _ptr(gx), _ptr(g0), _ptr(gp),
                               ctypes.byref(opts), _aligned(ws), nb, _stream(), info))
    return gp, gx, g0, _infos(info)


def seq_rollout(x, s0, params, cell="gru", offsets=None):
    """Sequential GPU baseline of the forward evaluation."""
    torch = _torch()
    for t, n in ((x, "x"), (s0, "s0"), (params, "params")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets)
    s = torch.empty((x.shape[0], s0.shape[1]), dtype=x.dtype, device=x.device)
    ws, nb = _workspace(OP_SEQ, sh, make_opts(), x.device)
    _check(load().seq_rollout(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x), _ptr(s0),
                              _ptr(s), _aligned(ws), nb, _stream()))
    return s


def seq_bptt(x, s0, params, s, gs, cell="gru", offsets=None):
    """Sequential GPU baseline of the backward pass; returns (gparams, gx, gs0)."""
    torch = _torch()
    for t, n in ((x, "x"), (s0, "s0"), (params, "params")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets, rows=[(s, "s", s0.shape[1]),
                                                     (gs, "gs", s0.shape[1])])
    gp = torch.empty_like(params)
    gx = torch.empty_like(x)
    g0 = torch.empty_like(s0)
    ws, nb = _workspace(OP_SEQ, sh, make_opts(), x.device)
    _check(load().seq_bptt(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x), _ptr(s0),
                           _ptr(s), _ptr(gs), _ptr(gx), _ptr(g0), _ptr(gp), _aligned(ws), nb,
                           _stream()))
    return gp, gx, g0


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """pn_copy_probe on two fresh device buffers: GB/s (read + write) of a streaming copy."""
    torch = _torch()
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    out = ctypes.c_double(0.0)
    _check(load().pn_copy_probe(_ptr(a), _ptr(b), int(nbytes), int(reps), _stream(),
                                ctypes.byref(out)))
    return out.value


class profile:
    """Context manager: HIP-event timing of the library's kernel launches on this thread."""

    def __enter__(self):
        load().pn_profile_begin()
        return self

    def __exit__(self, *exc):
        load().pn_profile_end()
        return False

    @staticmethod
    def read(family):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        if not load().pn_profile_read(family.encode(), ctypes.byref(ms), ctypes.byref(n)):
            return 0.0, 0
        return ms.value, n.value


def lle_estimate(x, s0, params, s, u0, cell="meanfield", offsets=None):
    """Largest Lyapunov exponent along the trajectory s per sequence (list of floats)."""
    for t, n in ((x, "x"), (s0, "s0"), (params, "params"), (s, "s"), (u0, "u0")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets, rows=[(s, "s", s0.shape[1])])
    if tuple(u0.shape) != tuple(s0.shape) or u0.dtype != x.dtype:
        raise ValueError(f"u0 must be [B, D] = {list(s0.shape)} of the dtype of x")
    ws, nb = _workspace(OP_LLE, sh, make_opts(), x.device)
    out = (ctypes.c_double * sh.batch.B)()
    _check(load().pn_lle_estimate(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x),
                                  _ptr(s0), _ptr(s), _ptr(u0), _aligned(ws), nb, _stream(), out))
    return list(out)


def residual_f64(x, s0, params, s, cell="tanh", offsets=None):
    for t, n in ((x, "x"), (s0, "s0"), (params, "params"), (s, "s")):
        _dev(t, n)
    sh = _shapes(cell, params, x, s0, offsets, rows=[(s, "s", s0.shape[1])])
    opts = make_opts()
    ws, nb = _workspace(OP_RESIDUAL64, sh, opts, x.device)
    out = (ctypes.c_double * sh.batch.B)()
    _check(load().pn_residual_f64(ctypes.byref(sh.cell), ctypes.byref(sh.batch), _ptr(x),
                                  _ptr(s0), _ptr(s), _aligned(ws), nb, _stream(), out))
    return list(out)


class DeerFunction:
    """torch.autograd.Function: forward = deer_solve, backward = deer_adjoint."""

    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            torch = _torch()

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, x, s0, params, cell, offsets, opt_kw, adj_kw):
                    s, info = deer_solve(x, s0, params, cell=cell, offsets=offsets, **opt_kw)
                    ctx.save_for_backward(x, s0, params, s)
                    ctx.cell, ctx.offsets, ctx.adj_kw = cell, offsets, adj_kw
                    ctx.info = info
                    return s

                @staticmethod
                def backward(ctx, gs):
                    x, s0, params, s = ctx.saved_tensors
                    gp, gx, g0, _ = deer_adjoint(x, s0, params, s, gs.contiguous(),
                                                 cell=ctx.cell, offsets=ctx.offsets,
                                                 **ctx.adj_kw)
                    return gx, g0, gp, None, None, None, None

            cls._cls = _Fn
        return cls._cls


def deer(x, s0, params, cell="gru", offsets=None, adjoint=None, **opt_kw):
    """Differentiable parallel-Newton evaluation of the recurrence (returns s [N, D]).
    The backward pass calls deer_adjoint with the same options, updated by the dict
    `adjoint` (e.g. dict(jac="dense", compose="bf16") for the GRU's dense reverse scan)."""
    adj_kw = dict(opt_kw, **(adjoint or {}))
    return DeerFunction.get().apply(x, s0, params, cell, offsets, opt_kw, adj_kw)
