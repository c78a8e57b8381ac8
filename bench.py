"""Benchmark: forward + backward of the parallel Newton path on one MI355X.

One "step" is the whole hot path over the batch: quasi-DEER solve of the GRU recurrence
(fused linearise + diagonal look-back scan per iteration, hipGraph-captured iterations),
then the exact quasi adjoint for the loss sum_t ||s_t||^2 (iterated reverse scans) and the
parameter / input / initial-state gradients.  Workload: GRU, D=64, Dx=32, B=16 sequences of
T=65536 steps (1,048,576 sequence-steps), weights N(0, 1/D), inputs N(0, 1), s_0 = 0, guess 0.

Printed: one JSON line with the throughput (sequence-steps/s), the sequential GPU baseline on
the same inputs, the dominant kernel's roofline (its duration measured with HIP events on the
library's stream), the CPU oracle baseline and the error of the result against it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--tol 1e-6] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GRAPH_ITERS = 4
METRIC = "fwd+bwd sequence-steps/sec, Newton-scan vs sequential rollout, same GPU, err≤1e-5"
WORKLOAD = "gru64-quasi-f32"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3


# kernel families timed inside the solver calls (HIP events on the library's stream)
FAMILIES = ("gru_quasi_local", "gru_adj_local", "carry_scan", "gru_adj_prep", "gru_adj_grad")


def gate_gemm_flops(D, Dx):
    """Algorithmic MFMA flops per step of the gate GEMM: z, r on [h; x], U_n h, W_n x."""
    return 2 * D * (2 * (D + Dx) + D + Dx)


def vjp_gemm_flops(D):
    """Algorithmic MFMA flops per step of the adjoint VJP [U_z; U_n; U_r]^T (3 D x D)."""
    return 2 * 3 * D * D


def fwd_local_bytes(D, Dx):
    """Algorithmic HBM bytes per step of one forward iteration (FP32): read s^(k-1), the
    previous maps (la, lc) and x; write s^(k) and the new maps."""
    return 4 * D + 8 * D + 4 * Dx + 4 * D + 8 * D


def adj_local_bytes(D):
    """Algorithmic HBM bytes per step of one adjoint iteration after the first (FP32): read
    lambda^(k-1), the step map (la, written once, and lc of the previous iteration), the gate
    values alpha, beta, gamma, the pair (z, diag A) and g; write lambda^(k) and the new lc."""
    return 4 * D + 8 * D + 12 * D + 8 * D + 4 * D + 4 * D + 4 * D


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gru64_hbm_traffic.txt")
SOURCES = {"gru_quasi_local": ["gru_quasi.hip", "gru_common.hpp", "pn_device.hpp"],
           "gru_adj_local": ["gru_adjoint.hip", "gru_common.hpp", "pn_device.hpp"]}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when the kernel's sources changed after the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2603_16850_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha, cur = h.hexdigest()[:16], None
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("kernel:"):
            cur = line.split(":", 1)[1].strip().split("<")[0].replace("_kernel", "")
        elif line.startswith("source_sha:") and cur == kernel:
            if line.split()[1] != sha:
                return None
        elif line.startswith("traffic_bytes:") and cur == kernel:
            return int(line.split()[1])
    return None


def roofline_of(kernel, D, Dx, N, avg_ms):
    """Both ceilings of a launch over N steps; the binding one (longer time at peak) wins."""
    if kernel == "gru_quasi_local":
        flops, nbytes = gate_gemm_flops(D, Dx) * N, fwd_local_bytes(D, Dx) * N
    else:
        flops, nbytes = vjp_gemm_flops(D) * N, adj_local_bytes(D) * N
    t_mfma = flops / (PEAK_FP32_TFLOPS * 1e12)
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    if t_mfma >= t_hbm:
        achieved = flops / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": kernel, "achieved": round(achieved, 2),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "algorithmic_per_launch": flops}
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
            "algorithmic_per_launch": nbytes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-6,
                    help="residual stopping tolerance (1e-6 keeps the error under 1e-5)")
    ap.add_argument("--adj-tol", type=float, default=1e-5,
                    help="stopping tolerance of the adjoint (max |rho| <= tol max(1, max |g|)); "
                         "the workload's stated 1e-5, which keeps the gradients within 1e-5 of "
                         "the FP64 oracle (the forward needs 1e-6 for its trajectory)")
    ap.add_argument("--seq-reps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--rows", action="store_true",
                    help="also measure the other workloads and method variants (adds a 'rows' "
                         "object to the line; a few minutes)")
    ap.add_argument("--rows-sections", type=int, default=0,
                    help="with --rows: measure only the first N sections (0 = all); section 2 is "
                         "the dense tanh D = 32 forward and adjoint")
    ap.add_argument("--graphs", action="store_true",
                    help="also time the step with graph-captured iterations (not the value)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="accepted for older command lines; the 1 GiB copy always runs")
    ap.add_argument("--sweep-lle", action="store_true",
                    help="instead of the step: the mean-field RNN LLE-threshold sweep (one "
                         "JSON line per gain and length)")
    ap.add_argument("--sweep-seeds", type=int, default=3)
    ap.add_argument("--tile", default="auto",
                    help="'auto': the forward and adjoint tile / group lengths chosen by the "
                         "library's autotuner before the warmup (reported, not timed); "
                         "'default': the cost-model choice; 'L,G,GA': forward tile L and group "
                         "G, adjoint group GA as given (e.g. to replay a tuned choice under a "
                         "profiler without the tuning launches)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(sequences would shard by batch with no communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    from paper_2603_16850_amd import workloads
    if args.sweep_lle:
        import torch
        import paper_2603_16850_amd as pn
        sweep_lle(torch, pn, workloads, args.sweep_seeds)
        return
    work = workloads.ALL[WORKLOAD]
    inst = workloads.make_instance(work, seed=0)
    D, Dx, B, N = work.D, work.Dx, work.B, inst.N

    # the CPU oracle runs first, in worker processes forked before anything touches the GPU
    cpu = None if args.no_cpu else cpu_oracle(inst)

    import torch
    import paper_2603_16850_amd as pn

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    pn.load()
    dev = "cuda"
    x = torch.tensor(inst.x, dtype=torch.float32, device=dev)
    s0 = torch.tensor(inst.s0, dtype=torch.float32, device=dev)
    p = torch.tensor(inst.params, dtype=torch.float32, device=dev)
    # The host reads the stopping state every GRAPH_ITERS iterations.  Inside the timed region
    # the iterations of a batch are launched back to back with a HIP event pair around each
    # kernel; launches of iterations after the last sequence stopped return at once and are
    # not counted in the per-kernel averages.
    kw = dict(cell="gru", offsets=inst.offsets, jac="diag", tol=args.tol, graph_iters=GRAPH_ITERS)
    adj_tol = args.adj_tol
    kw_f, kw_b, tuned = dict(kw), dict(kw, tol=adj_tol), None
    if args.tile == "auto":
        # one-time plan: the autotuner times the candidate tile / group lengths of both passes
        # on these inputs (8 iterations each); excluded from the timed region, reported
        torch.cuda.synchronize()
        tt0 = time.perf_counter()
        tf = pn.autotune("deer", x, s0, p, probe_iters=8, **kw)
        s_tr, _ = pn.deer_solve(x, s0, p, tile=tf["tile"], group=tf["group"], **kw)
        tb = pn.autotune("adjoint", x, s0, p, s=s_tr, gs=2.0 * s_tr, probe_iters=8,
                         **dict(kw, tol=adj_tol))
        torch.cuda.synchronize()
        tuned = {"tune_ms": round((time.perf_counter() - tt0) * 1e3, 1),
                 "fwd": {k: tf[k] for k in ("tile", "group", "ms_per_iter", "from_cache")},
                 "adj": {k: tb[k] for k in ("group", "ms_per_iter", "from_cache")},
                 "fwd_candidates": tf["candidates"], "adj_candidates": tb["candidates"]}
        kw_f.update(tile=tf["tile"], group=tf["group"])
        kw_b.update(group=tb["group"])
        del s_tr
    elif args.tile != "default":
        L, G, GA = (int(v) for v in args.tile.split(","))
        kw_f.update(tile=L, group=G)
        kw_b.update(group=GA)
        tuned = {"given": {"fwd_tile": L, "fwd_group": G, "adj_group": GA}}

    def step():
        s, finfo = pn.deer_solve(x, s0, p, **kw_f)
        gp, gx, g0, binfo = pn.deer_adjoint(x, s0, p, s, 2.0 * s, **kw_b)
        return s, gp, gx, g0, finfo, binfo

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K full steps, kernel durations by HIP events on the library stream
    step_ms = []
    with pn.profile():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            out = step()          # the solvers return after their work finished
            step_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fam = {f: pn.profile.read(f) for f in FAMILIES}
    s, gp, gx, g0, finfo, binfo = out
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = N / (ms_per_step * 1e-3)

    # ---- sequential GPU baseline on the same inputs
    torch.cuda.synchronize()
    ts0 = time.perf_counter()
    for _ in range(args.seq_reps):
        s_seq = pn.seq_rollout(x, s0, p, cell="gru", offsets=inst.offsets)
        sg = pn.seq_bptt(x, s0, p, s_seq, 2.0 * s_seq, cell="gru", offsets=inst.offsets)
    torch.cuda.synchronize()
    ts1 = time.perf_counter()
    seq_ms = (ts1 - ts0) * 1e3 / args.seq_reps
    seq_value = N / (seq_ms * 1e-3)

    # device-to-device copy of 1 GiB: the achievable HBM rate on this machine (read + write), and
    # the reference dispatch for the FETCH_SIZE / WRITE_SIZE counter scaling
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    copy_gbs = 3 * 2 * a.numel() * 4 / (time.perf_counter() - tc0) / 1e9
    del a, b

    # ---- roofline of the dominant kernel (largest share of the measured kernel time).
    # Launches that find every sequence stopped return at once; the average is taken over
    # the launches that did an iteration (one per iteration of the longest sequence, plus
    # the one that tests the last iterate).
    it_f = [i["iters"] for i in finfo]
    it_b = [i["iters"] for i in binfo]
    dom = max(("gru_quasi_local", "gru_adj_local"), key=lambda f: fam[f][0])
    dms, dn = fam[dom]
    avg_ms = dms / max(dn, 1)
    roofline = roofline_of(dom, D, Dx, N, avg_ms)
    roofline.update({"traffic": measured_traffic(dom), "avg_launch_ms": round(avg_ms, 4),
                     "launches": dn})
    if roofline["bound"] == "hbm":
        roofline["frac_of_measured_copy"] = round(roofline["achieved"] / copy_gbs, 4)

    # optionally the same step with the library's defaults (iterations captured in HIP graphs,
    # stopping state read every 4 iterations), outside the timed region
    ms_graph = None
    if args.graphs:
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for _ in range(args.steps):
            pn.deer_solve(x, s0, p, **dict(kw_f, graph_iters=4))
            pn.deer_adjoint(x, s0, p, s, 2.0 * s, **dict(kw_b, graph_iters=4))
        torch.cuda.synchronize()
        ms_graph = round((time.perf_counter() - tg0) * 1e3 / args.steps, 3)

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "sequence-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "cell": "gru", "D": D, "Dx": Dx, "B": B,
                   "T": work.T, "N": N, "method": "quasi-DEER fwd + exact quasi adjoint",
                   "tol": args.tol, "adj_tol": adj_tol, "loss": "sum_t ||s_t||^2",
                   "graph_iters": GRAPH_ITERS},
        "iters_fwd": it_f, "iters_bwd": it_b,
        "kernel_ms": {k: {"total": round(v[0], 3), "launches": v[1]} for k, v in fam.items()},
        "sequential_gpu": {"value": round(seq_value, 1), "unit": "sequence-steps/s",
                           "ms_per_step": round(seq_ms, 3)},
        "speedup_vs_sequential": round(value / seq_value, 2),
        "step_ms_median": round(float(np.median(step_ms)), 3),
        "step_ms_iqr": round(float(np.percentile(step_ms, 75) - np.percentile(step_ms, 25)), 3),
        "copy_bandwidth_gbs": round(copy_gbs, 1),
        "ms_per_step_graphs": ms_graph,
        "roofline": roofline,
        "autotune": tuned,
    }

    if cpu is not None:
        rec["cpu_baseline"] = cpu["baseline"]
        rec["cpu_single_core"] = cpu["single_core"]
        rec["err"] = errors(cpu, s, gp, gx, g0, s_seq)
    if args.rows:
        rec["rows"] = measure_rows(torch, pn, workloads, args.rows_sections)
    print(json.dumps(rec), flush=True)


def sweep_lle(torch, pn, workloads, seeds):
    """The LLE-threshold experiment of Ch. 5 on the mean-field RNN (D = 16): for every gain g
    and length T, each seed draws its own W; the sequential GPU rollout gives the trajectory,
    the LLE is estimated along it on the GPU from three random unit vectors (averaged), and
    DEER (ELK with lambda = 0, dense, tol 1e-5) solves the same sequence from s = 0.  Chaotic
    cases are capped at `cap` iterations (reported as not converged)."""
    dev = "cuda"
    gains = [round(0.5 + 0.125 * i, 3) for i in range(13)]
    for T, cap in ((1000, 1000), (10000, 400)):
        for g in gains:
            lles, iters, conv, deer_ms, seq_ms, errs = [], [], [], [], [], []
            for seed in range(seeds):
                w = workloads.MEANFIELD16.scaled(gain=g, T=T)
                inst = workloads.make_instance(w, seed=seed)
                x, s0, p = (torch.tensor(v, dtype=torch.float32, device=dev)
                            for v in (inst.x, inst.s0, inst.params))
                ms, s_seq = _timed(torch, lambda: pn.seq_rollout(x, s0, p, cell="meanfield",
                                                                 offsets=inst.offsets))
                seq_ms.append(ms)
                u = torch.tensor(np.random.default_rng(100 + seed).standard_normal((3, 16)),
                                 dtype=torch.float32, device=dev)
                lles.append(float(np.mean([pn.lle_estimate(x, s0, p, s_seq, u[i:i + 1],
                                                           cell="meanfield",
                                                           offsets=inst.offsets)[0]
                                           for i in range(3)])))
                ms, (s, info) = _timed(torch, lambda: pn.elk_solve(
                    x, s0, p, 0.0, cell="meanfield", offsets=inst.offsets, jac="dense",
                    tol=w.tol, max_iters=cap), reps=1)
                deer_ms.append(ms)
                iters.append(info[0]["iters"])
                conv.append(bool(info[0]["converged"]))
                ref = s_seq.double()
                errs.append(float((s.double() - ref).abs().max() / ref.abs().max()))
            print(json.dumps({
                "sweep": "meanfield16-lle", "T": T, "g": g, "seeds": seeds,
                "lle_mean": round(float(np.mean(lles)), 4),
                "lle_min": round(float(np.min(lles)), 4), "lle_max": round(float(np.max(lles)), 4),
                "deer_iters_mean": round(float(np.mean(iters)), 1), "deer_iters_max": max(iters),
                "converged": sum(conv), "cap": cap,
                "deer_ms_mean": round(float(np.mean(deer_ms)), 3),
                "seq_ms_mean": round(float(np.mean(seq_ms)), 3),
                "speedup_vs_sequential": round(float(np.mean(seq_ms) / np.mean(deer_ms)), 3),
                "err_vs_sequential_max": float(np.max(errs))}), flush=True)


def _timed(torch, fn, reps=3):
    """Median wall time (ms) of fn() over reps calls after one warm-up call."""
    out = fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(ts)), out


class _RowsDone(Exception):
    pass


def measure_rows(torch, pn, workloads, sections=0):
    """The other workloads and method variants: wall time per call, iterations, and the error
    against the sequential GPU rollout of the same FP32 inputs (max |s - s_seq| / max |s_seq|;
    on the chaotic tanh instance two FP32 evaluations differ by ~1e-5, and there the FP64
    residual below tol is the criterion).  Inputs are seed 0 of each workload.  `sections` > 0
    stops after that many sections."""
    rows = {}
    try:
        _measure_rows(torch, pn, workloads, sections, rows)
    except _RowsDone:
        pass
    return rows


def _measure_rows(torch, pn, workloads, sections, rows):
    dev = "cuda"
    count = [0]

    def done(name):
        print(f"rows: {name} done", file=sys.stderr, flush=True)
        count[0] += 1
        if sections and count[0] >= sections:
            raise _RowsDone()

    def tens(inst, dtype=torch.float32):
        return tuple(torch.tensor(v, dtype=dtype, device=dev) for v in (inst.x, inst.s0, inst.params))

    def rel(a, b):
        a, b = a.detach().double(), b.detach().double()
        return float((a - b).abs().max() / b.abs().max().clamp_min(1e-30))

    # dense DEER, GRU D = 4, FP64 (one workgroup per sequence, whole loop on chip)
    w = workloads.GRU4_DENSE_F64
    inst = workloads.make_instance(w, seed=0)
    x, s0, p = tens(inst, torch.float64)
    ms, (s, info) = _timed(torch, lambda: pn.deer_solve(x, s0, p, cell="gru", offsets=inst.offsets,
                                                        jac="dense", tol=w.tol))
    rows[w.name] = {"ms": round(ms, 3), "iters": [i["iters"] for i in info],
                    "max_resid_f64": max(i["max_resid"] for i in info),
                    "steps_per_s": round(inst.N / (ms * 1e-3), 1)}

    done('section 1')
    # dense DEER, tanh D = 32: BF16 and FP32 compose, vs the sequential GPU rollout
    w = workloads.TANH32_DENSE_BF16
    inst = workloads.make_instance(w, seed=0)
    x, s0, p = tens(inst)
    seq_ms, s_seq = _timed(torch, lambda: pn.seq_rollout(x, s0, p, cell="tanh", offsets=inst.offsets))
    r = {"sequential_ms": round(seq_ms, 3)}
    for comp in ("bf16", "native"):
        ms, (s, info) = _timed(torch, lambda: pn.deer_solve(
            x, s0, p, cell="tanh", offsets=inst.offsets, jac="dense", compose=comp, tol=1e-6))
        r[comp] = {"ms": round(ms, 3), "iters_max": max(i["iters"] for i in info),
                   "err_vs_sequential": rel(s, s_seq), "steps_per_s": round(inst.N / (ms * 1e-3), 1),
                   "speedup_vs_sequential": round(seq_ms / ms, 2)}
    ms, (s, info) = _timed(torch, lambda: pn.deer_solve(
        x, s0, p, cell="tanh", offsets=inst.offsets, jac="dense", tol=1e-6, damping="scale",
        damp_k=0.2))
    r["scale_elk_k0.2"] = {"ms": round(ms, 3), "iters_max": max(i["iters"] for i in info),
                           "err_vs_sequential": rel(s, s_seq)}
    # backward of the loss sum_t |s_t|^2 (g = 2 s): reverse dense scans, BF16 and FP32 maps
    s, _ = pn.deer_solve(x, s0, p, cell="tanh", offsets=inst.offsets, jac="dense",
                         compose="bf16", tol=1e-6)
    gs = 2 * s
    seq_bwd_ms, _ = _timed(torch, lambda: pn.seq_bptt(x, s0, p, s, gs, cell="tanh",
                                                       offsets=inst.offsets))
    r["sequential_bwd_ms"] = round(seq_bwd_ms, 3)
    for comp in ("bf16", "native"):
        ms, (gp, gx, g0, info) = _timed(torch, lambda: pn.deer_adjoint(
            x, s0, p, s, gs, cell="tanh", offsets=inst.offsets, jac="dense", compose=comp,
            tol=1e-6))
        r[f"adjoint_{comp}"] = {"ms": round(ms, 3), "iters_max": max(i["iters"] for i in info),
                                "converged": all(i["converged"] for i in info),
                                "fwd_bwd_ms": round(ms + r["bf16"]["ms"], 3),
                                "speedup_vs_sequential": round(seq_bwd_ms / ms, 2),
                                "steps_per_s": round(inst.N / (ms * 1e-3), 1)}
    rows[w.name] = r

    done('section 2')
    # ELK, quasi-ELK, DEER, converged-prefix skipping: tanh D = 16, FP64 stopping residual
    w = workloads.TANH16_ELK
    inst = workloads.make_instance(w, seed=0)
    x, s0, p = tens(inst)
    seq_ms, s_seq = _timed(torch, lambda: pn.seq_rollout(x, s0, p, cell="tanh", offsets=inst.offsets))
    r = {"sequential_ms": round(seq_ms, 3)}

    def elk_row(lam, **kw):
        ms, (s, info) = _timed(torch, lambda: pn.elk_solve(
            x, s0, p, lam, cell="tanh", offsets=inst.offsets, tol=w.tol,
            fp64_final_residual=True, **kw), reps=1)
        return {"ms": round(ms, 3), "iters_max": max(i["iters"] for i in info),
                "converged": all(i["converged"] for i in info),
                "max_resid_f64": max(i["max_resid"] for i in info),
                "err_vs_sequential": rel(s, s_seq)}
    for jac, name in (("dense", "elk"), ("diag", "quasi_elk")):
        for lam in w.lambdas:
            r[f"{name}_lambda{lam:g}"] = elk_row(lam, jac=jac)
    r["deer_lambda0"] = elk_row(0.0, jac="dense")
    for lam in w.lambdas:
        r[f"elk_lambda{lam:g}_freeze_prefix"] = elk_row(lam, jac="dense", freeze_prefix=True)
    rows[w.name] = r

    done('section 3')
    # ELK filter vs smoother (the exact LM step) on the contracting variant (gain 0.9)
    w9 = w.scaled(gain=0.9)
    inst = workloads.make_instance(w9, seed=0)
    x, s0, p = tens(inst)
    seq_ms, s_seq = _timed(torch, lambda: pn.seq_rollout(x, s0, p, cell="tanh", offsets=inst.offsets))
    rows["tanh16 gain 0.9 ELK lambda 0.1"] = {
        "sequential_ms": round(seq_ms, 3), "filter": elk_row(0.1, jac="dense"),
        "smoother": elk_row(0.1, jac="dense", smooth=True)}

    done('section 4')
    # mean-field RNN, DEER (lambda = 0) in the predictable regime, T = 10000
    wm = workloads.MEANFIELD16.scaled(gain=0.5, T=10000)
    inst = workloads.make_instance(wm, seed=0)
    x, s0, p = tens(inst)
    seq_ms, s_seq = _timed(torch, lambda: pn.seq_rollout(x, s0, p, cell="meanfield",
                                                         offsets=inst.offsets))
    ms, (s, info) = _timed(torch, lambda: pn.elk_solve(
        x, s0, p, 0.0, cell="meanfield", offsets=inst.offsets, jac="dense", tol=wm.tol))
    rows["meanfield16 g=0.5 T=10000 DEER"] = {
        "ms": round(ms, 3), "sequential_ms": round(seq_ms, 3),
        "speedup_vs_sequential": round(seq_ms / ms, 2), "iters": info[0]["iters"],
        "err_vs_sequential": rel(s, s_seq)}

    done('section 5')
    # ragged GRU batch: forward + backward as the main line
    w = workloads.GRU48_RAGGED
    inst = workloads.make_instance(w, seed=0)
    x, s0, p = tens(inst)
    kw = dict(cell="gru", offsets=inst.offsets, jac="diag", tol=1e-6)
    # autotuned tile / group lengths of both passes (one-time plan, not timed)
    tt0 = time.perf_counter()
    tf = pn.autotune("deer", x, s0, p, probe_iters=6, **kw)
    kw_f = dict(kw, tile=tf["tile"], group=tf["group"])
    s_tr, _ = pn.deer_solve(x, s0, p, **kw_f)
    kw_adj = dict(kw, tol=1e-5)       # the adjoint at the stated tolerance, as the main line
    tb = pn.autotune("adjoint", x, s0, p, s=s_tr, gs=2.0 * s_tr, probe_iters=6, **kw_adj)
    kw_b = dict(kw_adj, group=tb["group"])
    torch.cuda.synchronize()
    tune_ms = (time.perf_counter() - tt0) * 1e3
    del s_tr

    def fb():
        s, fi = pn.deer_solve(x, s0, p, **kw_f)
        gp, gx, g0, bi = pn.deer_adjoint(x, s0, p, s, 2.0 * s, **kw_b)
        return s, fi, bi
    ms, (s, fi, bi) = _timed(torch, fb, reps=2)

    def fb_default():
        s, fi = pn.deer_solve(x, s0, p, **kw)
        pn.deer_adjoint(x, s0, p, s, 2.0 * s, **kw_adj)
        return s
    ms_default, _ = _timed(torch, fb_default, reps=2)

    def seqfb():
        s = pn.seq_rollout(x, s0, p, cell="gru", offsets=inst.offsets)
        pn.seq_bptt(x, s0, p, s, 2.0 * s, cell="gru", offsets=inst.offsets)
        return s
    seq_ms, s_seq = _timed(torch, seqfb, reps=1)
    rows[w.name] = {"fwd_bwd_ms": round(ms, 3), "steps_per_s": round(inst.N / (ms * 1e-3), 1),
                    "sequential_ms": round(seq_ms, 3), "speedup_vs_sequential": round(seq_ms / ms, 2),
                    "iters_fwd_max": max(i["iters"] for i in fi),
                    "iters_bwd_max": max(i["iters"] for i in bi), "N": int(inst.N),
                    "err_vs_sequential": rel(s, s_seq),
                    "autotuned": {"fwd_tile": tf["tile"], "fwd_group": tf["group"],
                                  "adj_group": tb["group"], "tune_ms": round(tune_ms, 1)},
                    "fwd_bwd_ms_cost_model_tiles": round(ms_default, 3)}

    done('section 6')
    # transition variants on the GRU path (benchmark shapes, forward only)
    w = workloads.GRU64_QUASI
    inst = workloads.make_instance(w, seed=0)
    x, s0, p = tens(inst)
    s_seq = pn.seq_rollout(x, s0, p, cell="gru", offsets=inst.offsets)
    r = {}
    for name, extra in (("quasi", {}), ("scale_k0.2", dict(damping="scale", damp_k=0.2)),
                        ("clip", dict(damping="clip"))):
        ms, (s, info) = _timed(torch, lambda: pn.deer_solve(
            x, s0, p, cell="gru", offsets=inst.offsets, jac="diag", tol=1e-6, **extra), reps=2)
        r[name] = {"ms": round(ms, 3), "iters_max": max(i["iters"] for i in info),
                   "err_vs_sequential": rel(s, s_seq)}
    rows["gru64 transitions"] = r

    done('section 7')
    # Picard / Jacobi / quasi-DEER iteration counts (Table fxd_pt_sum) on a short GRU batch
    w = workloads.GRU64_QUASI.scaled(B=16, T=512)
    inst = workloads.make_instance(w, seed=0)
    x, s0, p = tens(inst)
    s_seq = pn.seq_rollout(x, s0, p, cell="gru", offsets=inst.offsets)
    r = {}
    for jac in ("diag", "picard", "jacobi"):
        ms, (s, info) = _timed(torch, lambda: pn.deer_solve(
            x, s0, p, cell="gru", offsets=inst.offsets, jac=jac, tol=1e-6), reps=1)
        r[jac] = {"ms": round(ms, 3), "iters_max": max(i["iters"] for i in info),
                  "converged": all(i["converged"] for i in info),
                  "err_vs_sequential": rel(s, s_seq)}
    rows["gru64 T=512 fixed-point methods"] = r
    done("last section")
    return rows


def _one_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _oracle_one(job):
    """Forward rollout + sequential adjoint of one sequence in FP64 (one worker, one thread)."""
    cell, x, s0 = job
    from oracle import adjoint, rollout
    s = rollout.rollout(cell, x, s0)
    _, gp, gx, g0 = adjoint.adjoint(cell, x, s0, s, 2.0 * s)
    return s, gp, gx, g0


def cpu_oracle(inst):
    """The oracle (FP64 numpy rollout + sequential adjoint) on the host: one sequence on one
    core, then every sequence over a pool of single-threaded workers (one per core, at most
    16).  Returns the results for the error check and the two rates."""
    import multiprocessing as mp
    from oracle import cells
    try:
        from threadpoolctl import threadpool_limits
    except Exception:
        threadpool_limits = None
    w = inst.work
    cell = cells.GRU(inst.params, w.D, w.Dx)
    off = inst.offsets
    jobs = [(cell, inst.x[off[b]:off[b + 1]], inst.s0[b]) for b in range(w.B)]
    ncores = max(1, min(16, os.cpu_count() or 1))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    if threadpool_limits is not None:
        with threadpool_limits(1):
            t0 = time.perf_counter()
            _oracle_one(jobs[0])
            dt1 = time.perf_counter() - t0
    else:
        t0 = time.perf_counter()
        _oracle_one(jobs[0])
        dt1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(processes=ncores, initializer=_one_thread) as pool:
        res = pool.map(_oracle_one, jobs)
    dt = time.perf_counter() - t0
    s = np.concatenate([r[0] for r in res])
    gp = sum(r[1] for r in res)
    gx = np.concatenate([r[2] for r in res])
    g0 = np.stack([r[3] for r in res])
    t_b = int(off[1] - off[0])
    return {
        "s": s, "gp": gp, "gx": gx, "g0": g0,
        "baseline": {"value": round(inst.N / dt, 1), "unit": "sequence-steps/s",
                     "cores": ncores, "kind": "oracle",
                     "sample": f"whole workload ({w.B} x {w.T} steps): FP64 numpy sequential "
                               f"rollout + sequential adjoint, one sequence per single-threaded "
                               f"worker, {ncores} workers, {dt:.1f} s; CPU {model}"},
        "single_core": {"value": round(t_b / dt1, 1), "unit": "sequence-steps/s", "cores": 1,
                        "sample": f"one sequence ({t_b} steps), {dt1:.1f} s"},
    }


def errors(cpu, s, gp, gx, g0, s_seq):
    """Relative max errors of the GPU results against the oracle's."""
    def rel(a, b):
        a = a.detach().cpu().double().numpy() if hasattr(a, "detach") else a
        return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))

    return {"s": rel(s, cpu["s"]), "gparams": rel(gp, cpu["gp"]), "gx": rel(gx, cpu["gx"]),
            "gs0": rel(g0, cpu["g0"]), "s_sequential_gpu": rel(s_seq, cpu["s"])}


if __name__ == "__main__":
    main()
