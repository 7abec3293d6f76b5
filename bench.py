"""Benchmark of the multi-RHS coarse operator and its block-CG solve on one MI355X.

Default line: the precision workload -- periodic 8^4 coarse lattice (4096
sites), nbasis 64, nrhs 32, the 81-point stencil, Hermitian Gaussian links
with the self-term shift that gives condition number ~1e4. The right-hand side
is B = M X_true for a seeded X_true, computed by one complex128 oracle apply on
the host (the CPU baseline, timed), so each solve states its error against the
FP64 oracle. One step = one defect-correction solve to a true relative
residual of 1e-8 with 16-bit (the faster of BF16 and FP16) inner links: double
outer residual on complex64 links, BlockCGrQ inside (apply, Gram reductions,
small double steps, block updates, graph replays). The FP32 comparison solves
(complex64 inner links, 4M and 3M forms) run with the same warmup and steps.
`value` = time to 1e-8 with the faster FP32 inner form over time with the
faster 16-bit form. `roofline` = the faster complex64 apply against the FP32
MFMA peak (executed flops: the 3M form executes 3/4 of the 4M form's);
`roofline_lowp` = the faster 16-bit apply against 8 TB/s HBM.

Extras on the same line: the FP32 production shape (8^4, nbasis 32, nrhs 16,
9-point, kappa ~1e3) with its HBM roofline, backward kernels, solves and quick
figures of the next rows; oracle timings of the small case and the batching
systems. Other workloads: --workload fp32 | precision | batched | chebyshev |
pbcg | deflation | transfer.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the complex64 apply kernels on the 8^4/32/16 9-point
# workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# `--probe-counters` (FETCH_SIZE x 2 + WRITE_SIZE x 1, the factors each counter
# shows on a copy of known size). Valid for the kernels those runs profiled;
# a kernel not listed reports null.
APPLY_C2_TRAFFIC_BYTES = {
    "apply_mfma_kernel<float, 16, 2, 4, 2, 1>": 374.3e6,
    "apply_mfma_kernel<float, 16, 2, 4, 2, 2>": 373.5e6,
    "apply_mfma_kernel<float, 16, 2, 4, 1, 1>": 374.4e6,
    "apply_3m_kernel<1, 2, 1, false, false>": 376.1e6,
    "apply_3m_kernel<1, 2, 2, false, false>": 374.2e6,
}
# the same for the 8^4/64/32 81-point workload's applies (`--probe-counters
# --c3-apply-iters 5`); the 16-bit rows are the stencil kernel of the two-pass
# apply (its operand pass moves another 101 MB)
APPLY_C3_TRAFFIC_BYTES = {
    "apply_mfma_kernel<float, 32, 4, 8, 1, 1>": 11811.5e6,
    "apply_mfma_kernel<float, 32, 4, 8, 2, 1>": 11813.9e6,
    "apply_3m_kernel<2, 4, 1, false, false>": 11741.7e6,
    "apply_3m_kernel<2, 4, 2, false, false>": 11555.5e6,
    "apply_lowp2_kernel<0, 2, 4, 2>": 5942.3e6,
    "apply_lowp2_kernel<1, 2, 4, 2>": 5947.2e6,
}
# Fraction of cycles the MFMA pipes were busy during the kernel (rocprofv3
# --pmc SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE per XCD x 1024 SIMDs),
# from the same counter runs; the clock under the 81-point MFMA load is
# 2.06-2.28 GHz, so busy x clock / 2.4 GHz is the fraction of the peak rate.
APPLY_MFMA_BUSY = {
    "apply_mfma_kernel<float, 32, 4, 8, 1, 1>": 0.740,
    "apply_mfma_kernel<float, 32, 4, 8, 2, 1>": 0.725,
    "apply_3m_kernel<2, 4, 1, false, false>": 0.802,
    "apply_3m_kernel<2, 4, 2, false, false>": 0.764,
    "apply_lowp2_kernel<0, 2, 4, 2>": 0.191,
    "apply_lowp2_kernel<1, 2, 4, 2>": 0.197,
    "apply_mfma_kernel<float, 16, 2, 4, 2, 1>": 0.413,
    "apply_mfma_kernel<float, 16, 2, 4, 1, 1>": 0.457,
    "apply_3m_kernel<1, 2, 1, false, false>": 0.355,
    "apply_3m_kernel<1, 2, 2, false, false>": 0.356,
}
FP32_MFMA_PEAK_TFLOPS = 157.3
# kernels behind the backward timings of the 8^4/32/16 workload
GRAD_KERNELS = {"adjoint": "adjoint_3m_kernel<1, 2, 1>", "adjoint_4m": "adjoint_mfma_kernel<float, 2, 32>",
                "adjoint_as_forward_3m": "apply_3m_kernel<1, 2, 1, false, false> (adjoint links)",
                "link_grad": "link_grad_3m_kernel<2, 1, true>"}
# their HBM bytes per launch from the same counter runs (the 4M adjoint's
# from the complex64-layout run of the same probe)
GRAD_TRAFFIC_BYTES = {"adjoint": 373.5e6, "adjoint_4m": 390.1e6, "link_grad": 355.7e6,
                      "adjoint_as_forward_3m": 376.1e6}  # the forward 3M kernel's figure
METRIC = "mRHS coarse apply TFLOP/s & %roofline; BCG time-to-1e-8, mixed vs FP32"


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """The host the oracle runs on: cores this process may use, BLAS library and threads."""
    info = {"affinity_cores": len(os.sched_getaffinity(0)), "blas": None, "blas_threads": None}
    try:
        from threadpoolctl import threadpool_info
        pools = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if pools:
            info["blas"] = ", ".join(sorted({f"{i.get('internal_api')} {i.get('version')} "
                                             f"({i.get('threading_layer', '?')})" for i in pools}))
            info["blas_threads"] = max(int(i.get("num_threads", 1)) for i in pools)
    except Exception:  # pragma: no cover
        pass
    return info


def timed_oracle(fn):
    """(result, wall seconds, process CPU seconds) of one oracle call."""
    c0, t0 = time.process_time(), time.perf_counter()
    r = fn()
    return r, time.perf_counter() - t0, time.process_time() - c0


def cpu_record(flops, wall, cpu, sample):
    """The cpu_baseline object: the oracle's rate, and the threads it kept busy on
    average (process CPU time over wall time, rounded up) as `cores`."""
    h = host_info()
    busy = cpu / wall if wall > 0 else 0.0
    return {"value": flops / wall / 1e12, "unit": "TFLOP/s",
            "cores": int(min(max(1, math.ceil(busy - 0.05)), h["affinity_cores"])), "kind": "oracle",
            "sample": sample, "wall_s": round(wall, 2), "cpu_s": round(cpu, 2), "busy_threads": round(busy, 2),
            "affinity_cores": h["affinity_cores"], "blas": h["blas"], "blas_threads": h["blas_threads"]}


def oracle_small_timings(budget_s=20.0):
    """Oracle timings of the small parity case (4^4, nbasis 8, nrhs 4, 9-point):
    one apply, the dense LU solve and BlockCGrQ to 1e-10; and of each of the six
    batching systems' applies (links generated here, then freed), within about
    budget_s of CPU work in total."""
    import oracle as O
    import workloads as W
    out = {}
    s = W.C1
    links, offs, b = W.make_system(s)
    _, w, c = timed_oracle(lambda: O.apply(links, offs, s.dims, b))
    out["c1_apply"] = {"seconds": round(w, 5), "gflops": round(s.apply_flops() / w / 1e9, 3)}
    _, w, c = timed_oracle(lambda: O.solve_dense(links, offs, s.dims, b))
    out["c1_dense_lu_solve"] = {"seconds": round(w, 4)}
    op = lambda v: O.flatten(O.apply(links, offs, s.dims, v.reshape(s.volume, s.nbasis, -1)))
    (xs, info), w, c = timed_oracle(lambda: O.bcgrq(op, O.flatten(b), tol=s.tol, maxiter=500))
    rr = O.true_relres(op, O.flatten(b), xs)
    out["c1_bcgrq_solve"] = {"seconds": round(w, 4), "iterations": int(info.iterations),
                             "true_relres": float(np.max(rr))}
    t_start = time.perf_counter()
    c4 = []
    for sysd in W.C4:
        if time.perf_counter() - t_start > budget_s:
            c4.append({"system": sysd.name, "skipped": "time budget"})
            continue
        links, offs, b = W.make_system(sysd)
        _, w, c = timed_oracle(lambda: O.apply(links, offs, sysd.dims, b))
        c4.append({"system": sysd.name, "seconds": round(w, 4), "gflops": round(sysd.apply_flops() / w / 1e9, 3)})
        del links, b
    out["c4_applies"] = c4
    return out


def _time_apply(coarse, torch, op, x, y, iters, reps=5, workspace=None):
    """Median seconds per launch over reps bursts of iters back-to-back applies
    (HIP events recorded on the stream the kernels are launched on)."""
    for _ in range(3):
        coarse.apply(op, x, out=y, workspace=workspace)
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            coarse.apply(op, x, out=y, workspace=workspace)
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) * 1e-3 / iters)
    return float(np.median(out))


def apply_kernel_names(coarse, s, variant, variant3m):
    """Kernel names (as rocprofv3 prints them) of the tuned apply of each link form."""
    mv = coarse.max_apply_variant(s.nbasis)
    ps, pd = (1, 1) if variant == mv else (1 << min(variant, mv - 1), 2)
    nt = (2 * s.nrhs + 15) // 16
    nst = s.nbasis // 16
    return {"c64": f"apply_mfma_kernel<float, {s.nrhs}, {nt}, {s.nbasis // 8}, {pd}, {ps}>",
            "c64_3m": f"apply_3m_kernel<{(s.nrhs + 15) // 16}, {nst}, {1 + variant3m}, false, false>",
            "bf16": f"apply_lowp2_kernel<0, {(s.nrhs + 15) // 16}, {nst}, 2>",
            "fp16": f"apply_lowp2_kernel<1, {(s.nrhs + 15) // 16}, {nst}, 2>"}


def timed_solves(torch, fn, warmup, steps):
    """Run fn (one solve) warmup times untimed, then steps times between two
    device synchronisations; returns (seconds per solve, last result)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = None
    for _ in range(steps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1), r


def solve_errors(x, x_true):
    """Max over columns of ||x_j - x_true_j|| / ||x_true_j|| (complex128 on the device)."""
    d = (x - x_true).reshape(-1, x.shape[-1])
    t = x_true.reshape(-1, x.shape[-1])
    return float((d.abs().pow(2).sum(0).sqrt() / t.abs().pow(2).sum(0).sqrt()).max().item())


def precision_section(a, with_cpu=True):
    """8^4 lattice, nbasis 64, nrhs 32, 81-point stencil, kappa ~1e4.

    A manufactured solution X_true (CN(0,1), drawn after the operator) gives
    the right-hand side B = M X_true by one complete complex128 oracle apply on
    the host (the CPU baseline, timed), so every solve states its error against
    the FP64 oracle. Then, on the GPU: the apply per link form (complex64 4M and
    3M, BF16 and FP16 with per-block scales; HIP events on the launch stream),
    and the defect-correction solve to a 1e-8 true residual with each form as
    the inner operator (the outer residual always takes the complex64 links in
    the 3M layout, double accumulation in the 3M form), every form with the same
    warmup and steps.
    Returns (record, kernel names)."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    s = W.C3
    _log(f"[bench] generating {s.name}: dims {s.dims} nbasis {s.nbasis} nrhs {s.nrhs} {s.stencil}")
    links, offs, rng = W.make_operator(s)
    x_true = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs, dtype=np.complex128)
    flops = s.apply_flops()
    cpu = None
    if with_cpu:
        import oracle as O
        _log("[bench] CPU oracle: B = M X_true (one complete complex128 apply)")
        b, wall, cput = timed_oracle(lambda: O.apply(links, offs, s.dims, x_true))
        cpu = cpu_record(flops, wall, cput,
                         f"one complete complex128 oracle apply of the 8^4/64/32 81-point operator (the "
                         f"manufactured right-hand side B = M X_true of the solves), {wall:.1f} s")
        _log(f"[bench] oracle apply {wall:.1f} s")
    else:
        b = None
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    dev = torch.device("cuda:0")
    lt = torch.from_numpy(links).to(dev)
    del links
    xt = torch.from_numpy(x_true).to(dev)
    x = torch.from_numpy(x_true.astype(np.complex64)).to(dev)
    y = torch.empty_like(x)
    ops = {k: coarse.pack(lt, geom, k) for k in ("c64", "c64_3m", "bf16", "fp16")}
    del lt
    if b is None:  # no oracle: the right-hand side from the library's double apply (errors then not stated)
        bd = torch.empty_like(xt)
        coarse.apply(ops["c64"], xt, out=bd)
    else:
        bd = torch.from_numpy(b).to(dev)
    variant, _ = coarse.tune_apply(ops["c64"], x, reps=5)
    variant3m, _ = coarse.tune_apply(ops["c64_3m"], x, reps=5)
    names = apply_kernel_names(coarse, s, variant, variant3m)
    vec = 2 * s.vector_bytes_c64()
    applies = {}
    ws16 = torch.empty(max(coarse.apply_workspace_bytes(ops["bf16"], s.nrhs), 1), dtype=torch.uint8, device=dev)
    for k, op in ops.items():
        _log(f"[bench] apply {k}")
        t = _time_apply(coarse, torch, op, x, y, a.c3_apply_iters, workspace=ws16)
        nbytes = (s.link_bytes_c64() if k.startswith("c64") else s.link_bytes_lowp()) + vec
        ex = flops * (0.75 if k == "c64_3m" else 1.0)
        applies[k] = {"us": round(t * 1e6, 1), "tflops_useful": round(flops / t / 1e12, 2),
                      "tflops_executed": round(ex / t / 1e12, 2), "gbs": round(nbytes / t / 1e9, 1),
                      "algorithmic_bytes": nbytes, "kernel": names[k]}
        if k.startswith("c64"):  # f32 MFMA (3M: three real products per complex one, 3/4 of the 4M flops)
            applies[k]["mfma_frac"] = round(ex / t / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4)
            applies[k]["hbm_frac"] = round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4)
        else:  # 16-bit links: HBM-bound
            applies[k]["hbm_frac"] = round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4)
    applies["c64"]["variant"] = variant
    applies["c64_3m"]["variant"] = variant3m
    ws = torch.empty(coarse.workspace_bytes(geom, s.nrhs), dtype=torch.uint8, device=dev)
    solves = {}
    # inner tolerances from a sweep on this workload (fastest time-to-1e-8 per precision;
    # complex64 1e-4 among 3e-5..3e-4, FP16 1e-3 among 5e-4..5e-3, BF16 5e-3 among 5e-3..2e-2)
    for k, itol in (("c64_3m", 1e-4), ("fp16", 1e-3), ("c64", 1e-4), ("bf16", 5e-3)):
        kw = dict(tol=s.tol, inner_tol=itol, max_outer=30, max_inner=5000, check_every=16, inner=ops[k],
                  workspace=ws)
        _log(f"[bench] solve {k}: {a.warmup} warmup, {a.steps} timed")
        t, r = timed_solves(torch, lambda: coarse.bcg_solve(ops["c64_3m"], bd, **kw), a.warmup, a.steps)
        solves[k] = {"seconds": round(t, 4), "cycles": r.cycles, "inner_iterations": r.iterations,
                     "relres": r.relres_max, "status": r.status, "inner_tol": itol,
                     "err_vs_oracle": solve_errors(r.x, xt) if b is not None else None}
        _log(f"[bench] solve {k}: {solves[k]}")
    fp32 = min(("c64", "c64_3m"), key=lambda k: solves[k]["seconds"])
    mixed = min(("bf16", "fp16"), key=lambda k: solves[k]["seconds"])
    kf = min(("c64", "c64_3m"), key=lambda k: applies[k]["us"])
    kl = min(("bf16", "fp16"), key=lambda k: applies[k]["us"])
    ex = flops * (0.75 if kf == "c64_3m" else 1.0)
    t_f = applies[kf]["us"] * 1e-6
    t_l = applies[kl]["us"] * 1e-6
    rec = {
        "value": round(solves[fp32]["seconds"] / solves[mixed]["seconds"], 3),
        "unit": f"x (time to a 1e-8 true residual: {fp32} inner / {mixed} inner)",
        "ms_per_step": round(solves[mixed]["seconds"] * 1e3, 2),
        "dtype": f"{mixed}+f32+f64",
        "config": {"workload": "coarse8^4_nb64_nrhs32_81pt_kappa1e4", "lattice": list(s.dims),
                   "nbasis": s.nbasis, "nrhs": s.nrhs, "npoint": s.npoint, "tol": s.tol,
                   "rhs": "B = M X_true (complex128 oracle apply), X_true ~ CN(0,1)",
                   "step": f"one solve with {mixed} inner links", "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": round(ex / t_f / 1e12, 2), "peak": FP32_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(ex / t_f / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4),
                     "traffic": APPLY_C3_TRAFFIC_BYTES.get(names[kf]), "kernel": names[kf],
                     "mfma_busy_counter": APPLY_MFMA_BUSY.get(names[kf]),
                     "executed_flops_per_launch": ex, "useful_flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": applies[kf]["algorithmic_bytes"]},
        "roofline_lowp": {"bound": "hbm", "achieved": round(applies[kl]["algorithmic_bytes"] / t_l / 1e9, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(applies[kl]["algorithmic_bytes"] / t_l / 1e9 / HBM_PEAK_GBS, 4),
                          "traffic": APPLY_C3_TRAFFIC_BYTES.get(names[kl]), "kernel": names[kl],
                          "mfma_busy_counter": APPLY_MFMA_BUSY.get(names[kl]),
                          "algorithmic_bytes_per_launch": applies[kl]["algorithmic_bytes"]},
        "apply": applies,
        "bcg": solves,
        "speedup_mixed_vs_fp32": {"fp32": fp32, "mixed": mixed,
                                  "ratio": round(solves[fp32]["seconds"] / solves[mixed]["seconds"], 3)},
        "cpu_baseline": cpu,
    }
    del ops, ws, ws16
    torch.cuda.empty_cache()
    return rec


def precision_main(a):
    """The 8^4/64/32 81-point workload alone (the default line without the
    8^4/32/16 extras)."""
    rec = precision_section(a, with_cpu=not a.no_cpu_baseline)
    out = {"metric": METRIC, "value": rec.pop("value"), "unit": rec.pop("unit"), "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": rec.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": rec.pop("dtype"), "data": "synthetic", "config": rec.pop("config")}
    out.update(rec)
    print(json.dumps(out), flush=True)
    return 0


def probe_counters(a):
    """A fixed dispatch sequence for hardware-counter runs (no timing).
    8^4/32/16 (`--workload fp32`): the tuned complex64 applies, 4M then 3M form,
    `apply_iters` times each (after the 4M ones as many adjoint applies and
    link gradients, after the 3M ones as many 3M adjoints and Gram-fused 3M
    applies). 8^4/64/32 81-point (`--workload precision`): the tuned 4M
    and 3M applies and the two-pass BF16 and FP16 applies, `c3_apply_iters`
    times each. The default workload runs both. Then three plain
    device-to-device copies of 512 MiB (the calibration of the counters' byte
    totals against a kernel of known traffic)."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    info = {"probe": "counters"}
    if a.workload in ("default", "precision"):
        s = W.C3
        links, offs, _ = W.make_operator(s)
        geom = coarse.Geometry(s.dims, s.nbasis, offs)
        lt = torch.from_numpy(links).cuda()
        del links
        x = torch.from_numpy(W.gaussian_vectors(np.random.default_rng(3), s.dims, s.nbasis, s.nrhs)).cuda()
        y = torch.empty_like(x)
        for form in ("c64", "c64_3m", "bf16", "fp16"):
            op = coarse.pack(lt, geom, form)
            ws = None
            if form.startswith("c64"):
                coarse.tune_apply(op, x, reps=3)
            else:
                ws = torch.empty(coarse.apply_workspace_bytes(op, s.nrhs), dtype=torch.uint8, device="cuda")
            for _ in range(a.c3_apply_iters):
                coarse.apply(op, x, out=y, workspace=ws)
            torch.cuda.synchronize()
            del op, ws
        del lt
        info["c3_applies"] = a.c3_apply_iters
        info["c3_apply_algorithmic_bytes"] = {"c64": s.link_bytes_c64() + 2 * s.vector_bytes_c64(),
                                              "lowp": s.link_bytes_lowp() + 2 * s.vector_bytes_c64()}
        torch.cuda.empty_cache()
    if a.workload in ("default", "fp32"):
        s = W.C2
        links, offs, b = W.make_system(s)
        geom = coarse.Geometry(s.dims, s.nbasis, offs)
        lt = torch.from_numpy(links).cuda()
        x = torch.from_numpy(b.astype(np.complex64)).cuda()
        y = torch.empty_like(x)
        for form in ("c64", "c64_3m"):
            op = coarse.pack(lt, geom, form)
            coarse.tune_apply(op, x, reps=5)
            for _ in range(a.apply_iters):
                coarse.apply(op, x, out=y)
            if form == "c64":  # the backward kernels on the same shapes
                dl = torch.empty(geom.link_shape(), dtype=torch.complex64, device="cuda")
                for _ in range(a.apply_iters):
                    coarse.apply_adjoint(op, x, out=y)
                    coarse.link_grad(geom, x, x, out=dl, accumulate=False)
                del dl
            else:  # the 3M adjoint, then the Gram-fused 3M apply (y = M x and x^H y)
                for _ in range(a.apply_iters):
                    coarse.apply_adjoint(op, x, out=y)
                wsg = torch.empty(coarse.apply_gram_workspace_bytes(op, s.nrhs), dtype=torch.uint8, device="cuda")
                for _ in range(a.apply_iters):
                    coarse.apply_gram(op, x, out=y, workspace=wsg)
                del wsg
            del op
        info["c2_applies"] = a.apply_iters
        info["c2_apply_algorithmic_bytes"] = s.link_bytes_c64() + 2 * s.vector_bytes_c64()
    src = torch.ones(512 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    info.update({"copy_bytes_read": src.numel(), "copy_bytes_written": dst.numel()})
    print(json.dumps(info), flush=True)
    return 0


def batched_main(a):
    """Six independent systems of uneven size (lattices 4^4 .. 8^3x16, nbasis
    24/32/48, nrhs 4..32, 9-point, kappa ~1e3): one persistent launch over all
    of them against the same six applies as separate (tuned) launches, and the
    block-CG solve of each system to 1e-8."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    ops, xs, ys, bs, nbytes, flops = [], [], [], [], 0, 0
    for sysd in W.C4:
        links, offs, b = W.make_system(sysd)
        geom = coarse.Geometry(sysd.dims, sysd.nbasis, offs)
        ops.append(coarse.pack(torch.from_numpy(links).cuda(), geom, "c64"))
        xs.append(torch.from_numpy(b.astype(np.complex64)).cuda())
        ys.append(torch.empty_like(xs[-1]))
        bs.append(torch.from_numpy(b).cuda())
        nbytes += sysd.link_bytes_c64() + 2 * sysd.vector_bytes_c64()
        flops += sysd.apply_flops()
        del links
    variants = [coarse.tune_apply(op, x, reps=10)[0] for op, x in zip(ops, xs)]

    def timed(fn, iters):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        tt = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(iters):
                fn()
            e1.record()
            torch.cuda.synchronize()
            tt.append(e0.elapsed_time(e1) * 1e-3 / iters)
        return float(np.median(tt))

    def separate():
        for op, x, y in zip(ops, xs, ys):
            coarse.apply(op, x, out=y)

    t_sep = timed(separate, a.apply_iters)
    per = [timed(lambda op=op, x=x, y=y: coarse.apply(op, x, out=y), a.apply_iters) for op, x, y in zip(ops, xs, ys)]
    batch = coarse.BatchedApply(ops, xs, ys)
    occ = batch.tune(reps=10, candidates=(1, 2, 3, 4, 6, 8), compare_separate=False)
    t_b = timed(batch.persistent, a.apply_iters)

    # a batch of eight small systems (lattices of 64 to 256 sites): alone, none
    # of them fills the GPU, which is where one persistent launch pays off
    rng = np.random.default_rng(240903904 + 400)
    small = []
    for i, dims in enumerate([(4, 4, 4, 4), (4, 4, 4, 2), (4, 4, 2, 2), (2, 2, 4, 4), (4, 2, 4, 2), (2, 4, 2, 4),
                              (4, 4, 2, 4), (2, 2, 2, 4)]):
        nb, nr = (24, 32, 48)[i % 3], (4, 8, 16, 32)[i % 4]
        offs9 = W.stencil("9pt")
        sl = W.gaussian_links(rng, dims, nb, offs9.shape[0])
        sx = W.gaussian_vectors(rng, dims, nb, nr)
        sg = coarse.Geometry(dims, nb, offs9)
        small.append((coarse.pack(torch.from_numpy(sl).cuda(), sg, "c64"), torch.from_numpy(sx).cuda(),
                      sl.nbytes + 2 * sx.nbytes))
    sops = [o for o, _, _ in small]
    sxs = [x_ for _, x_, _ in small]
    sys_ = [torch.empty_like(x_) for x_ in sxs]
    for o, x_ in zip(sops, sxs):
        coarse.tune_apply(o, x_, reps=10)
    sb = coarse.BatchedApply(sops, sxs, sys_)
    sb.tune(reps=10, candidates=(2, 4, 8), compare_separate=False)
    t_small_p = timed(sb.persistent, a.apply_iters)
    t_small_s = timed(sb.separate, a.apply_iters)
    small_bytes = sum(nb_ for _, _, nb_ in small)
    solves = []
    kw = dict(tol=1e-8, inner_tol=1e-4, max_outer=30, max_inner=5000, check_every=16)
    t_seq = 0.0
    for sysd, op, bd in zip(W.C4, ops, bs):
        coarse.bcg_solve(op, bd, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = coarse.bcg_solve(op, bd, **kw)
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        solves.append({"system": sysd.name, "seconds": round(time.perf_counter() - t0, 5), "cycles": r.cycles,
                       "inner_iterations": r.iterations, "relres": r.relres_max, "status": r.status})
    # all six in one call: one graph, one branch per system
    coarse.bcg_solve_batched(ops, bs, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = coarse.bcg_solve_batched(ops, bs, **kw)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    batched_solve = {"seconds": round(t_bat, 5), "sequential_seconds": round(t_seq, 5),
                     "speedup": round(t_seq / t_bat, 3),
                     "systems": [{"cycles": r.cycles, "inner_iterations": r.iterations, "relres": r.relres_max,
                                  "status": r.status} for r in rb]}
    out = {
        "metric": "mRHS coarse apply TFLOP/s & %roofline; BCG time-to-1e-8, mixed vs FP32",
        "value": round(flops / t_b / 1e12, 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": a.apply_iters, "warmup": 3, "ms_per_step": round(t_b * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "six_uneven_systems_9pt_kappa1e3",
                   "systems": [[list(sd.dims), sd.nbasis, sd.nrhs] for sd in W.C4], "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / t_b / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(nbytes / t_b / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "apply_batched_kernel", "algorithmic_bytes_per_launch": nbytes},
        "batched": {"persistent_us": round(t_b * 1e6, 1), "separate_launches_us": round(t_sep * 1e6, 1),
                    "sum_of_single_us": round(sum(per) * 1e6, 1), "speedup_vs_separate": round(t_sep / t_b, 3),
                    "occupancy_us": {str(k): round(v, 1) for k, v in occ.items()},
                    "single_us": [round(v * 1e6, 1) for v in per], "single_variants": variants,
                    "tuned_mode_us": round(min(t_b, t_sep) * 1e6, 1),
                    "tuned_mode": "persistent" if t_b <= t_sep else "separate"},
        "batched_small": {"systems": 8, "bytes": small_bytes, "persistent_us": round(t_small_p * 1e6, 2),
                          "separate_launches_us": round(t_small_s * 1e6, 2),
                          "speedup_vs_separate": round(t_small_s / t_small_p, 3),
                          "persistent_gbs": round(small_bytes / t_small_p / 1e9, 1)},
        "bcg": solves,
        "bcg_batched": batched_solve,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def chebyshev_main(a):
    """The stationary Chebyshev approximation to M^{-1} (Sec. 2.3) on the
    8^4/32/16 9-point operator: degree 120 on [lo, hi] with hi = 1.1 lambda_max
    (above the spectrum, as in the paper) and lo = hi / 2000 (the paper's
    [0.02, 40] ratio). One step = one P(M) x; timed per link form with HIP
    events, next to one block-CG iteration of the same workload."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    s = W.C2
    links, offs, b = W.make_system(s)
    sh = W.stored_shifts()["c2"]
    hi = 1.1 * sh["lambda_max"]
    lo = hi / 2000.0
    order = 120
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    lt = torch.from_numpy(links).cuda()
    x = torch.from_numpy(b.astype(np.complex64)).cuda()
    y = torch.empty_like(x)
    flops = s.apply_flops()
    vec = s.vector_bytes_c64()
    forms = {}
    for form in ("c64", "c64_3m", "bf16", "fp16"):
        op = coarse.pack(lt, geom, form)
        if form.startswith("c64"):
            coarse.tune_apply(op, x, reps=5)
        ws = torch.empty(coarse.chebyshev_workspace_bytes(op, s.nrhs), dtype=torch.uint8, device="cuda")
        _log(f"[bench] chebyshev {form}")
        for _ in range(2):
            coarse.chebyshev_apply(op, x, lo, hi, order, out=y, workspace=ws)
        torch.cuda.synchronize()
        tt = []
        for _ in range(max(a.steps, 3)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            coarse.chebyshev_apply(op, x, lo, hi, order, out=y, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            tt.append(e0.elapsed_time(e1) * 1e-3)
        t = float(np.median(tt))
        links_b = s.link_bytes_c64() if form.startswith("c64") else s.link_bytes_lowp()
        # apply (links, t, z) + recurrence pass (z, t, t_prev, y in; t_next, y out); with 3M links the pass
        # is the apply's epilogue (links, t, t_prev, y in; t_next, y out)
        per_degree = links_b + (5 if form == "c64_3m" else 8) * vec
        forms[form] = {"ms": round(t * 1e3, 3), "us_per_degree": round(t / order * 1e6, 2),
                       "tflops": round(order * flops / t / 1e12, 2),
                       "gbs": round(order * per_degree / t / 1e9, 1), "algorithmic_bytes_per_degree": per_degree}
        del op, ws
    best = min(("c64", "c64_3m"), key=lambda k: forms[k]["ms"])
    t = forms[best]["ms"] * 1e-3
    out = {
        "metric": "mRHS coarse apply TFLOP/s & %roofline; BCG time-to-1e-8, mixed vs FP32",
        "value": round(order * flops / t / 1e12, 3), "unit": "TFLOP/s",
        "n_gpus": 1, "steps": max(a.steps, 3), "warmup": 2, "ms_per_step": round(t * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "chebyshev_deg120_coarse8^4_nb32_nrhs16_9pt_kappa1e3", "lattice": list(s.dims),
                   "nbasis": s.nbasis, "nrhs": s.nrhs, "npoint": s.npoint, "order": order, "lo": lo, "hi": hi,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": forms[best]["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(forms[best]["gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"{best} apply + recurrence pass per degree",
                     "algorithmic_bytes_per_degree": forms[best]["algorithmic_bytes_per_degree"]},
        "chebyshev": forms,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def pbcg_main(a):
    """Preconditioned BlockCGrQ with the stationary Chebyshev preconditioner on
    the 8^4/32/16 9-point operator (kappa 1e3): time to a 1e-8 true residual
    against the unpreconditioned solve, both on 3M complex64 inner links, for
    a sweep of polynomial degree n and interval [hi / ratio, hi] with
    hi = 1.1 lambda_max. Applies counted: per cycle the start polynomial (n)
    and per inner iteration 1 + n, plus one outer residual per cycle."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    s = W.C2
    links, offs, b = W.make_system(s)
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    dev = torch.device("cuda:0")
    lt = torch.from_numpy(links).to(dev)
    op = coarse.pack(lt, geom, "c64")
    op3m = coarse.pack(lt, geom, "c64_3m")
    x = torch.from_numpy(b.astype(np.complex64)).to(dev)
    coarse.tune_apply(op, x, reps=20)
    coarse.tune_apply(op3m, x, reps=20)
    bd = torch.from_numpy(b).to(dev)
    flops = s.apply_flops()
    hi = 1.1 * W.stored_shifts()["c2"]["lambda_max"]
    kw = dict(tol=s.tol, inner_tol=1e-4, max_outer=30, max_inner=3000, check_every=16)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        tt, r = [], None
        for _ in range(max(a.steps, 3)):
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t0)
        return float(np.median(tt)), r

    t_plain, rp = timed(lambda: coarse.bcg_solve(op3m, bd, inner=op3m, **kw))
    plain = {"ms": round(t_plain * 1e3, 3), "cycles": rp.cycles, "inner_iterations": rp.iterations,
             "applies": rp.iterations + rp.cycles + 1, "relres": rp.relres_max, "status": rp.status}
    _log(f"[bench] plain: {plain}")
    sweep = []
    configs = ((4, 100.0), (8, 200.0), (16, 500.0), (16, 1000.0), (32, 2000.0), (64, 2000.0))
    if a.pbcg_config:
        o, r = a.pbcg_config.split(",")
        configs = ((int(o), float(r)),)
    for order, ratio in configs:
        lo = hi / ratio
        ws = torch.empty(coarse.pbcg_workspace_bytes(geom, s.nrhs, lo, hi, order), dtype=torch.uint8, device=dev)
        t, r = timed(lambda: coarse.pbcg_solve(op3m, bd, lo, hi, order, inner=op3m, workspace=ws, **kw))
        applies = r.iterations * (1 + order) + r.cycles * order + r.cycles + 1
        row = {"order": order, "hi_over_lo": ratio, "ms": round(t * 1e3, 3), "cycles": r.cycles,
               "inner_iterations": r.iterations, "applies": applies, "relres": r.relres_max, "status": r.status,
               "speedup_vs_plain": round(t_plain / t, 3), "tflops": round(applies * flops / t / 1e12, 2)}
        _log(f"[bench] pbcg: {row}")
        sweep.append(row)
        del ws
    ok = [r for r in sweep if r["status"] == 0]
    best = min(ok, key=lambda r: r["ms"]) if ok else None
    out = {
        "metric": "mRHS coarse apply TFLOP/s & %roofline; BCG time-to-1e-8, mixed vs FP32",
        "value": best["tflops"] if best else None, "unit": "TFLOP/s",
        "n_gpus": 1, "steps": max(a.steps, 3), "warmup": 1, "ms_per_step": best["ms"] if best else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "pbcg_chebyshev_coarse8^4_nb32_nrhs16_9pt_kappa1e3_tol1e-8",
                   "lattice": list(s.dims), "nbasis": s.nbasis, "nrhs": s.nrhs, "npoint": s.npoint, "hi": hi,
                   "inner": "c64_3m", "parallelism": "single-gpu"},
        "plain_bcg": plain, "pbcg": sweep, "best": best, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def deflation_main(a):
    """Multi-RHS deflation on the 8^4/32/16 workload: n_ev = 192 and 1000
    orthonormal vectors (the paper's range), c = V^H x, Defl = V diag(1/lambda) c,
    x_perp = x - V c (V streamed three times), and the deflated degree-120
    Chebyshev coarse solve with 192 vectors (3M links)."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    s = W.C2
    links, offs, b = W.make_system(s)
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(b.astype(np.complex64)).to(dev)
    n = s.volume * s.nbasis
    vec = n * s.nrhs * 8
    res = {}
    for nev in (192, 1000):
        # random columns of unit expected norm, orthonormal to O(sqrt(nev / n)); the
        # timing does not depend on orthonormality (set-up, not timed)
        g = torch.Generator(device=dev)
        g.manual_seed(nev)
        v = (torch.randn(n, nev, dtype=torch.complex64, device=dev, generator=g) / float(np.sqrt(n)))
        v = v.contiguous().reshape(s.volume, s.nbasis, nev)
        lam = torch.linspace(0.0066, 0.066, nev, dtype=torch.float64, device=dev)
        ws = torch.empty(coarse.deflation_workspace_bytes(geom, nev, s.nrhs), dtype=torch.uint8, device=dev)
        for _ in range(3):
            coarse.deflate(v, lam, x, geom, want_perp=True, workspace=ws)
        torch.cuda.synchronize()
        tt = []
        for _ in range(max(a.steps, 5)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                coarse.deflate(v, lam, x, geom, want_perp=True, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            tt.append(e0.elapsed_time(e1) * 1e-3 / 20)
        t = float(np.median(tt))
        vb = n * nev * 8
        alg = 2 * vb + 4 * vec  # V twice (coefficients, then both outputs); x twice, y and x_perp written
        res[nev] = {"us": round(t * 1e6, 1), "gbs": round(alg / t / 1e9, 1),
                    "frac": round(alg / t / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg,
                    "tflops": round(3 * 8 * n * nev * s.nrhs / t / 1e12, 2)}
        _log(f"[bench] deflate nev {nev}: {res[nev]}")
        if nev == 192:
            op = coarse.pack(torch.from_numpy(links).to(dev), geom, "c64_3m")
            coarse.tune_apply(op, x, reps=20)
            hi = 1.1 * W.stored_shifts()["c2"]["lambda_max"]
            lo, order = hi / 2000.0, 120
            y = torch.empty_like(x)
            coarse.deflated_chebyshev_apply(op, v, lam, x, lo, hi, order, out=y)
            torch.cuda.synchronize()
            tt = []
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                coarse.deflated_chebyshev_apply(op, v, lam, x, lo, hi, order, out=y)
                e1.record()
                torch.cuda.synchronize()
                tt.append(e0.elapsed_time(e1) * 1e-3)
            res["deflated_chebyshev_192_deg120_ms"] = round(float(np.median(tt)) * 1e3, 3)
            _log(f"[bench] deflated chebyshev: {res['deflated_chebyshev_192_deg120_ms']} ms")
            # block Lanczos set-up: 16 steps of a 16-vector block (K = 256), 32 Ritz pairs
            x0 = x.clone()
            lz_ws = torch.empty(1, dtype=torch.uint8, device=dev)
            coarse.block_lanczos(op, x0, 16, 32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, lz_lam, lz_res, lz_k = coarse.block_lanczos(op, x0, 16, 32)
            torch.cuda.synchronize()
            res["block_lanczos_16x16_nev32"] = {"seconds": round(time.perf_counter() - t0, 4), "basis": lz_k,
                                                "theta_min": float(lz_lam[0]), "residual_min": float(lz_res[0])}
            _log(f"[bench] block lanczos: {res['block_lanczos_16x16_nev32']}")
            del lz_ws
            del op
        del v, ws
    best = res[1000]
    out = {
        "metric": "mRHS coarse apply TFLOP/s & %roofline; BCG time-to-1e-8, mixed vs FP32",
        "value": best["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": max(a.steps, 5), "warmup": 3,
        "ms_per_step": round(best["us"] * 1e-3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "deflation_nev1000_coarse8^4_nb32_nrhs16", "lattice": list(s.dims),
                   "nbasis": s.nbasis, "nrhs": s.nrhs, "parallelism": "single-gpu"},
        # three complex products of n x nev x nrhs (V^H x, V c, V c_s), four real
        # f32 MFMA products each: against the f32 MFMA peak; HBM fraction beside it
        "roofline": {"bound": "mfma", "achieved": best["tflops"], "peak": 157.3, "unit": "TFLOP/s",
                     "frac": round(best["tflops"] / 157.3, 4), "traffic": None,
                     "kernel": "defl_coef_kernel + defl_reduce_kernel + defl_promote_kernel<true>",
                     "hbm_gbs": best["gbs"], "hbm_frac": best["frac"],
                     "algorithmic_bytes": best["algorithmic_bytes"]},
        "deflation": {str(k): v for k, v in res.items()}, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def transfer_main(a):
    """Block project C = B^H F and promote F = B C, one product per coarse site,
    at the paper's Table 6 shapes (N_basis 64, N_rhs 12, V_block 256, batch
    4096 = an 8^4 coarse lattice), complex64."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    dims, nb, vblock, nr = (8, 8, 8, 8), 64, 256, 12
    V = 4096
    geom = coarse.Geometry(dims, nb, W.stencil("9pt"))
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2409)
    B = torch.randn(V, vblock, nb, dtype=torch.complex64, device=dev, generator=g)
    F = torch.randn(V, vblock, nr, dtype=torch.complex64, device=dev, generator=g)
    C = torch.randn(V, nb, nr, dtype=torch.complex64, device=dev, generator=g)
    Co = torch.empty_like(C)
    Fo = torch.empty_like(F)
    flops = 8 * nb * nr * vblock * V
    bytes_ = (V * vblock * nb + V * vblock * nr + V * nb * nr) * 8
    res = {}
    for name, fn in (("project", lambda: coarse.block_project(B, F, geom, out=Co)),
                     ("promote", lambda: coarse.block_promote(B, C, geom, out=Fo))):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        tt = []
        for _ in range(max(a.steps, 5)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(50):
                fn()
            e1.record()
            torch.cuda.synchronize()
            tt.append(e0.elapsed_time(e1) * 1e-3 / 50)
        t = float(np.median(tt))
        res[name] = {"us": round(t * 1e6, 1), "tflops": round(flops / t / 1e12, 2), "gbs": round(bytes_ / t / 1e9, 1),
                     "frac": round(bytes_ / t / 1e9 / HBM_PEAK_GBS, 4)}
        _log(f"[bench] {name}: {res[name]}")
    worst = min(res.values(), key=lambda r: r["tflops"])
    out = {
        "metric": "mRHS coarse apply TFLOP/s & %roofline; BCG time-to-1e-8, mixed vs FP32",
        "value": worst["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": max(a.steps, 5), "warmup": 5,
        "ms_per_step": round(worst["us"] * 1e-3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "block_project_promote_nb64_nrhs12_vblock256_batch4096", "nbasis": nb, "nrhs": nr,
                   "vblock": vblock, "batch": V, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": worst["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": worst["frac"], "traffic": None, "kernel": "slower of project / promote",
                     "algorithmic_bytes": bytes_},
        "transfer": res, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def next_rows_summary(coarse, torch, W, s, geom, op3m, x):
    """Quick timings of the rows beyond the solve, for the default bench line:
    the degree-120 Chebyshev polynomial (3M links, fused epilogue), deflation
    with 192 vectors (c, Defl x and x_perp), and block project / promote at the
    paper's batched shapes (N_basis 64, N_rhs 12, V_block 256, 4096 sites)."""
    dev = x.device

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    out = {}
    hi = 1.1 * W.stored_shifts()["c2"]["lambda_max"]
    y = torch.empty_like(x)
    cws = torch.empty(coarse.chebyshev_workspace_bytes(op3m, s.nrhs), dtype=torch.uint8, device=dev)
    t = timed(lambda: coarse.chebyshev_apply(op3m, x, hi / 2000.0, hi, 120, out=y, workspace=cws), 3)
    out["chebyshev_deg120_3m_ms"] = round(t * 1e3, 3)
    del cws
    n = s.volume * s.nbasis
    g = torch.Generator(device=dev)
    g.manual_seed(192)
    v = (torch.randn(n, 192, dtype=torch.complex64, device=dev, generator=g) / float(np.sqrt(n)))
    v = v.contiguous().reshape(s.volume, s.nbasis, 192)
    lam = torch.linspace(0.0066, 0.066, 192, dtype=torch.float64, device=dev)
    dws = torch.empty(coarse.deflation_workspace_bytes(geom, 192, s.nrhs), dtype=torch.uint8, device=dev)
    t = timed(lambda: coarse.deflate(v, lam, x, geom, want_perp=True, workspace=dws), 20)
    out["deflation_nev192_us"] = round(t * 1e6, 1)
    del v, dws
    tg = coarse.Geometry((8, 8, 8, 8), 64, W.stencil("9pt"))
    B = torch.randn(4096, 256, 64, dtype=torch.complex64, device=dev, generator=g)
    F = torch.randn(4096, 256, 12, dtype=torch.complex64, device=dev, generator=g)
    C = torch.randn(4096, 64, 12, dtype=torch.complex64, device=dev, generator=g)
    Co, Fo = torch.empty_like(C), torch.empty_like(F)
    out["block_project_us"] = round(timed(lambda: coarse.block_project(B, F, tg, out=Co), 20) * 1e6, 1)
    out["block_promote_us"] = round(timed(lambda: coarse.block_promote(B, C, tg, out=Fo), 20) * 1e6, 1)
    del B, F, C, Co, Fo
    return out


def c2_section(a, with_cpu=True):
    """The FP32 production shape (8^4, nbasis 32, nrhs 16, 9-point, kappa ~1e3):
    the apply kernels against the HBM roofline (4M and 3M forms, tuned), the
    backward kernels, and the defect-correction solve to a 1e-8 true residual
    with 3M / BF16 / FP16 inner links and by Preconditioned BlockCGrQ, each with
    its error against a manufactured solution whose right-hand side the
    complex128 oracle computes (timed as this shape's CPU baseline); quick
    figures of the Chebyshev polynomial, deflation and block project / promote."""
    import torch

    import workloads as W
    from paper_2409_03904_amd import coarse

    s = W.C2
    _log(f"[bench] generating {s.name}: dims {s.dims} nbasis {s.nbasis} nrhs {s.nrhs} {s.stencil}")
    links, offs, rng = W.make_operator(s)
    x_true = W.gaussian_vectors(rng, s.dims, s.nbasis, s.nrhs, dtype=np.complex128)
    flops = s.apply_flops()
    cpu = None
    b = None
    if with_cpu:
        import oracle as O
        _log("[bench] CPU oracle: B = M X_true, then repeated applies for ~8 s")
        b, wall, cput = timed_oracle(lambda: O.apply(links, offs, s.dims, x_true))
        n, t0, c0 = 1, time.perf_counter() - wall, time.process_time() - cput
        while time.perf_counter() - t0 < 8.0:
            O.apply(links, offs, s.dims, x_true)
            n += 1
        wall, cput = time.perf_counter() - t0, time.process_time() - c0
        cpu = cpu_record(flops * n, wall, cput, f"{n} complex128 oracle applies of the 8^4/32/16 9-point operator "
                                                f"in {wall:.1f} s ({wall / n * 1e3:.0f} ms each)")
    geom = coarse.Geometry(s.dims, s.nbasis, offs)
    dev = torch.device("cuda:0")
    lt = torch.from_numpy(links).to(dev)
    op = coarse.pack(lt, geom, "c64")
    op3m = coarse.pack(lt, geom, "c64_3m")
    xt = torch.from_numpy(x_true).to(dev)
    x = torch.from_numpy(x_true.astype(np.complex64)).to(dev)
    y = torch.empty_like(x)
    if b is None:
        bd = torch.empty_like(xt)
        coarse.apply(op, xt, out=bd)
    else:
        bd = torch.from_numpy(b).to(dev)
    alg_bytes = s.link_bytes_c64() + 2 * s.vector_bytes_c64()

    variant, tune_us = coarse.tune_apply(op, x, reps=20)
    variant3m, tune3m_us = coarse.tune_apply(op3m, x, reps=20)
    names = apply_kernel_names(coarse, s, variant, variant3m)
    _log(f"[bench] tuned 4M variant {variant} ({tune_us:.1f} us), 3M variant {variant3m} ({tune3m_us:.1f} us)")
    applies = {}
    for form, o in (("c64", op), ("c64_3m", op3m)):
        t = _time_apply(coarse, torch, o, x, y, a.apply_iters)
        ex = flops * (0.75 if form == "c64_3m" else 1.0)
        applies[form] = {"us": round(t * 1e6, 2), "tflops_useful": round(flops / t / 1e12, 2),
                         "tflops_executed": round(ex / t / 1e12, 2), "gbs": round(alg_bytes / t / 1e9, 1),
                         "hbm_frac": round(alg_bytes / t / 1e9 / HBM_PEAK_GBS, 4),
                         "mfma_frac": round(ex / t / 1e12 / FP32_MFMA_PEAK_TFLOPS, 4), "kernel": names[form],
                         "variant": variant if form == "c64" else variant3m}
    form = min(applies, key=lambda k: applies[k]["us"])
    inner_op = op3m if form == "c64_3m" else op
    t_apply = applies[form]["us"] * 1e-6
    gbs = alg_bytes / t_apply / 1e9

    _log("[bench] backward kernels")
    grad = {}
    dl = torch.empty(geom.link_shape(), dtype=torch.complex64, device=dev)
    op_adj = coarse.pack_adjoint(lt, geom, "c64_3m")
    # adjoint: the 3M kernel on the 3M layout (the layout the autograd apply
    # packs); adjoint_4m: the LDS-transposing kernel on the complex64 layout
    for name, fn in (("adjoint", lambda: coarse.apply_adjoint(op3m, x, out=y)),
                     ("adjoint_4m", lambda: coarse.apply_adjoint(op, x, out=y)),
                     ("adjoint_as_forward_3m", lambda: coarse.apply(op_adj, x, out=y)),
                     ("link_grad", lambda: coarse.link_grad(geom, x, x, out=dl, accumulate=False))):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        tt = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(100):
                fn()
            e1.record()
            torch.cuda.synchronize()
            tt.append(e0.elapsed_time(e1) * 1e-3 / 100)
        t = float(np.median(tt))
        grad[name] = {"us": round(t * 1e6, 2), "gbs": round(alg_bytes / t / 1e9, 1),
                      "frac": round(alg_bytes / t / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg_bytes,
                      "kernel": GRAD_KERNELS[name], "traffic": GRAD_TRAFFIC_BYTES.get(name)}
    del dl, op_adj, lt

    kw = dict(tol=s.tol, inner_tol=1e-4, max_outer=30, max_inner=3000, check_every=16)
    ws = torch.empty(coarse.workspace_bytes(geom, s.nrhs), dtype=torch.uint8, device=dev)

    def solve(inner, **extra):  # outer residual: the 3M-layout links in double
        args = dict(kw)
        args.update(extra)
        return coarse.bcg_solve(op3m, bd, inner=inner, workspace=ws, **args)

    bcg = {}
    _log(f"[bench] 8^4/32/16 solves: {a.warmup} warmup, {a.steps} timed each")
    t, r = timed_solves(torch, lambda: solve(inner_op), a.warmup, a.steps)
    n_applies = r.iterations + r.cycles + 1  # inner applies + outer residuals
    bcg["fp32"] = {"inner": form, "seconds": round(t, 5), "cycles": r.cycles, "inner_iterations": r.iterations,
                   "relres": r.relres_max, "status": r.status,
                   "err_vs_oracle": solve_errors(r.x, xt) if b is not None else None,
                   "applies": n_applies, "tflops_of_applies": round(n_applies * flops / t / 1e12, 3)}
    if not a.no_mixed:
        for kind, itol in (("bf16", 1e-2), ("fp16", 1e-3)):
            inner = coarse.pack(torch.from_numpy(links).to(dev), geom, kind)
            t, r = timed_solves(torch, lambda: solve(inner, inner_tol=itol), a.warmup, a.steps)
            bcg[kind] = {"seconds": round(t, 5), "cycles": r.cycles, "inner_iterations": r.iterations,
                         "relres": r.relres_max, "status": r.status,
                         "err_vs_oracle": solve_errors(r.x, xt) if b is not None else None}
            del inner
        hi = 1.1 * W.stored_shifts()["c2"]["lambda_max"]
        lo, order = hi / 200.0, 8
        pws = torch.empty(coarse.pbcg_workspace_bytes(geom, s.nrhs, lo, hi, order), dtype=torch.uint8, device=dev)
        t, r = timed_solves(torch, lambda: coarse.pbcg_solve(op3m, bd, lo, hi, order, inner=inner_op, workspace=pws,
                                                             **kw), a.warmup, a.steps)
        bcg["pbcg_chebyshev_deg8"] = {"seconds": round(t, 5), "inner": form, "cycles": r.cycles,
                                      "inner_iterations": r.iterations, "relres": r.relres_max,
                                      "status": r.status, "order": order, "hi_over_lo": 200.0,
                                      "err_vs_oracle": solve_errors(r.x, xt) if b is not None else None}
        del pws

    _log("[bench] next rows")
    nxt = next_rows_summary(coarse, torch, W, s, geom, op3m, x)
    rec = {
        "config": {"workload": "coarse8^4_nb32_nrhs16_9pt_kappa1e3", "lattice": list(s.dims), "nbasis": s.nbasis,
                   "nrhs": s.nrhs, "npoint": s.npoint, "tol": s.tol},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": APPLY_C2_TRAFFIC_BYTES.get(names[form]),
                     "kernel": names[form], "algorithmic_bytes_per_launch": alg_bytes},
        "apply": {"form": form, "forms": applies},
        "grad": grad,
        "bcg": bcg,
        "next_rows": nxt,
        "cpu_baseline": cpu,
    }
    del op, op3m, ws
    torch.cuda.empty_cache()
    return rec


def fp32_main(a):
    """The 8^4/32/16 workload alone: one step = one FP32 (best complex64 form)
    solve to 1e-8; value = the useful apply rate of that solve."""
    rec = c2_section(a, with_cpu=not a.no_cpu_baseline)
    f = rec["bcg"]["fp32"]
    out = {"metric": METRIC, "value": f["tflops_of_applies"], "unit": "TFLOP/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(f["seconds"] * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
           "config": dict(rec.pop("config"), parallelism="single-gpu")}
    out.update(rec)
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("default", "fp32", "precision", "batched", "chebyshev", "pbcg",
                                           "deflation", "transfer"),
                    default="default",
                    help="default: the 8^4/64/32 81-point precision workload (mixed vs FP32 time to 1e-8) "
                         "with the 8^4/32/16 figures as extras; fp32: 8^4/32/16 9-point alone; precision: "
                         "8^4/64/32 81-point alone; batched: six uneven systems in one persistent launch; "
                         "chebyshev: degree-120 stationary polynomial on the fp32 workload; pbcg: "
                         "Chebyshev-preconditioned block CG on the fp32 workload; deflation: multi-RHS "
                         "deflation with 192 and 1000 vectors and the deflated Chebyshev solve; transfer: "
                         "block project / promote at the paper's batched-GEMM shapes")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--apply-iters", type=int, default=1000, help="back-to-back applies per timing (8^4/32/16)")
    ap.add_argument("--c3-apply-iters", type=int, default=50, help="back-to-back applies per timing (8^4/64/32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-small-oracle", action="store_true", help="skip the small-case oracle timings")
    ap.add_argument("--pbcg-config", default=None, help="pbcg workload: one 'degree,hi_over_lo' instead of the sweep")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--probe-counters", action="store_true",
                    help="run a fixed apply + copy sequence for rocprofv3 --pmc (no timing)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the coarse systems here fit one MI355X, and the "
              "multi-GPU halo exchange is not part of this build (run with --gpus 1)", file=sys.stderr)
        return 2

    if a.probe_counters:
        return probe_counters(a)
    if a.workload == "fp32":
        return fp32_main(a)
    if a.workload == "precision":
        return precision_main(a)
    if a.workload == "batched":
        return batched_main(a)
    if a.workload == "chebyshev":
        return chebyshev_main(a)
    if a.workload == "pbcg":
        return pbcg_main(a)
    if a.workload == "deflation":
        return deflation_main(a)
    if a.workload == "transfer":
        return transfer_main(a)

    # default: the precision workload is the headline; the 8^4/32/16 figures ride along
    cpu = not a.no_cpu_baseline
    rec = precision_section(a, with_cpu=cpu)
    c2 = c2_section(a, with_cpu=cpu)
    small = None
    if cpu and not a.no_small_oracle:
        _log("[bench] CPU oracle: small case and batching systems")
        small = oracle_small_timings()
    out = {"metric": METRIC, "value": rec.pop("value"), "unit": rec.pop("unit"), "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": rec.pop("ms_per_step"), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": rec.pop("dtype"), "data": "synthetic", "config": rec.pop("config")}
    out.update(rec)
    out["coarse8^4_nb32_nrhs16_9pt"] = c2
    out["cpu_oracle_other"] = small
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
