#!/usr/bin/env python3
"""Throughput of the MMOC particle tracer on one MI355X.

Workload: the 3D swirl -- unit cube of 6 Kuhn macro tetrahedra refined to
level 5, 65^3 = 274625 P2 DoFs = particles, LeVeque's deformation field with
g(t) = cos(pi t / 1.5) sampled at every time level, two Gaussian blobs as the
scalar, dt = T/20 (CFL ~ 5), 4 RK4 sub-steps, a 50-step run.

One timed step is one full MMOC advection step of the time loop: the new
velocity level and the current scalar are copied into the library's block
layout (field ingestion), then every particle is created, traced back with
RK4 and the scalar evaluated at its departure point; the result is the next
step's scalar.  All inputs (every velocity level of the run) are resident in
device memory before timing starts.  value = particles per second of the
float64 tracer (error <= 1e-12 against the CPU oracle); the float32-mixed
tracer (<= 1e-5) and the surrogate step (network + RK4 check + fallback,
<= 1e-4) are measured on the same run and reported beside it, as are the
trace kernels alone on the large workloads (rising plumes, 1.7e7
particles; the spherical shell, 1.7e8 particles, float32 paths) and the
advection-diffusion run of Table 4 with its CG solve.

The roofline entry is for the dominant kernel (the float64 trace): its
algorithmic flops per particle (FMA = 2, see flops_per_particle) over its
mean duration from HIP events recorded around each launch on the stream it
runs on.  cpu_baseline times the CPU oracle (single-threaded float64 C) on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TRACE_SRC = os.path.join(ROOT, "paper_2103_02388_amd", "csrc", "mmoc_trace.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "trace_fp64_swirl3d_traffic.json")


def flops_per_particle(dim, nlev, S):
    """Algorithmic flops of one particle's step (FMA = 2).  Per stage
    evaluation: reference coordinates (offset dim, matrix 2 dim^2, lambda_0
    dim + 1), micro location and P2 basis (Kuhn sums 2(dim - 1), scaling 2 dim,
    fractional parts 2 dim, micro barycentrics dim + 1, vertex shape functions
    3 (dim + 1), edge shape functions 2 per edge), the P2 sums (2 per node,
    component and level), the time interpolation (3 dim) and the stage update
    (4 dim); 2 dim per sub-step for the departure point; the scalar evaluation
    at the end.  The first stage evaluation (at the particle's own DoF) is
    counted as a full one."""
    nn = (dim + 1) * (dim + 2) // 2
    ref = dim + 2 * dim * dim + dim + 1
    micro = (2 * (dim - 1) + 2 * dim + 2 * dim) + (dim + 1) + 3 * (dim + 1) + 2 * (nn - dim - 1)
    gather = 2 * nn * dim * nlev + (3 * dim if nlev == 2 else 0)
    stage = 4 * dim
    per_eval = ref + micro + gather + stage
    scalar = ref + micro + 2 * nn
    return S * (4 * per_eval + 2 * dim) + scalar


def bytes_per_particle(dim, nlev, real_bytes):
    """Compulsory HBM bytes of one particle's step: every unique field value
    read once (velocity levels, scalar), every output written once (chat in
    the path's real type, X in float64)."""
    return dim * nlev * real_bytes + real_bytes + real_bytes + dim * 8


PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12


def counter_summary():
    """The committed rocprofv3 counter summary of the float64 trace kernel,
    if it was taken on the current kernel source (else None)."""
    try:
        d = json.load(open(TRAFFIC))
        sha = hashlib.sha256(open(TRACE_SRC, "rb").read()).hexdigest()
        return d if d.get("source_sha256") == sha else None
    except Exception:
        return None


def traffic_entry():
    """HBM bytes per launch of the float64 trace kernel (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy's counts)."""
    d = counter_summary()
    return d["hbm_bytes_per_launch"] if d else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--substeps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--paths", default="fp64,fp32,fp32f", help="tracer paths to time (fp64 is the headline)")
    ap.add_argument("--no-diffusion", action="store_true")
    ap.add_argument("--no-plume", action="store_true")
    ap.add_argument("--no-shell", action="store_true", help="skip the 1.7e8-particle spherical shell")
    ap.add_argument("--diffusion-only", action="store_true",
                    help="only the advection-diffusion sub-result (for profiling its kernels)")
    ap.add_argument("--spmv-only", action="store_true",
                    help="only the operator apply on the large annulus (for profiling that kernel alone)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (10 times), to scale HBM counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 10}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (particles are independent "
              "and would be sharded by macro ownership). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_02388_amd import workloads as W

    torch.cuda.set_device(0)
    if args.diffusion_only:
        print(json.dumps({"diffusion": time_diffusion()}), flush=True)
        return
    if args.spmv_only:
        print(json.dumps({"spmv": spmv_roofline()}), flush=True)
        return
    wl = W.swirl3d()
    S = args.substeps
    results = {}
    paths = args.paths.split(",")
    if "fp64" not in paths:
        paths = ["fp64"] + paths
    for path in paths:
        results[path] = time_path(wl, path, S, args.steps, args.warmup)
    N = results["fp64"]["N"]
    r = results["fp64"]
    fpp = flops_per_particle(3, 2, S)
    bpp64 = bytes_per_particle(3, 2, 8)
    achieved = fpp * N / (r["kernel_ms"] * 1e-3)
    out = {
        "metric": "particles traced/sec (RK4+locate+P2 interp) at stated error; FP32/MLP vs FP64",
        "value": r["value"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "swirl3d: unit cube, 6 Kuhn macro tets, level 5, 274625 P2 particles, LeVeque swirl "
                               "T=1.5, dt=T/20 (CFL~5), RK4 with %d sub-steps, 50-step run" % S,
                   "particles": N, "substeps": S, "precision": "fp64", "error_bound_vs_oracle": 1e-12},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU,
                     "traffic": traffic_entry(),
                     "kernel": "trace_fp64_kernel<3,2,0>", "kernel_ms": r["kernel_ms"], "flop_per_particle": fpp,
                     "hbm_GBps_algorithmic": bpp64 * N / (r["kernel_ms"] * 1e-3) / 1e9,
                     "hbm_frac_algorithmic": bpp64 * N / (r["kernel_ms"] * 1e-3) / PEAK_HBM,
                     "hbm_GBps_measured": (traffic_entry() / (r["kernel_ms"] * 1e-3) / 1e9
                                           if traffic_entry() is not None else None),
                     "l1_tag_lookups_per_cu_cycle": (counter_summary() or {}).get("l1_tag_lookups_per_cu_cycle")},
        "trace_only_particles_per_s": N / (r["kernel_ms"] * 1e-3),
        "stats": r["stats"],
    }
    if "fp32" in results:
        f = results["fp32"]
        out["fp32_mixed"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "kernel_ms": f["kernel_ms"],
                             "trace_only_particles_per_s": N / (f["kernel_ms"] * 1e-3),
                             "speedup_vs_fp64_step": f["value"] / r["value"],
                             "speedup_vs_fp64_trace": r["kernel_ms"] / f["kernel_ms"],
                             "error_bound_vs_oracle": 1e-5,
                             "tieband_fraction": f["stats"]["n_tieband"] / max(1, f["stats"]["n_particles"])}
    if "fp32f" in results:
        f = results["fp32f"]
        out["fp32_fields"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "kernel_ms": f["kernel_ms"],
                              "trace_only_particles_per_s": N / (f["kernel_ms"] * 1e-3),
                              "speedup_vs_fp64_step": f["value"] / r["value"],
                              "speedup_vs_fp64_trace": r["kernel_ms"] / f["kernel_ms"],
                              "error_bound_vs_oracle": 1e-6,
                              "note": "float32 field records, float64 arithmetic"}
    if not args.no_surrogate:
        out["surrogate"] = time_surrogate(wl, S, min(args.steps, 50), min(args.warmup, 5), results)
    if not args.no_plume:
        out["plume3d"] = time_large(W.plume3d(), 120, ("fp64", "fp32", "fp32f"))
    if not args.no_shell:
        out["shell3d"] = time_large(W.shell3d(), 0, ("fp32", "fp32f"))
    if not args.no_diffusion:
        out["diffusion"] = time_diffusion()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, S)
    print(json.dumps(out), flush=True)


def time_path(wl, path, S, steps, warmup):
    import torch
    from paper_2103_02388_amd import mmoc
    from paper_2103_02388_amd import workloads as W

    prec = {"fp64": mmoc.MMOC_FP64, "fp32": mmoc.MMOC_FP32_MIXED, "fp32f": mmoc.MMOC_FP32_FIELDS}[path]
    tr = mmoc.Tracer.from_workload(wl, precision=prec)
    N = tr.N
    x = tr.dof_coords()
    xt = x.t().contiguous()
    nsteps = wl.steps
    U = torch.stack([W.swirl_velocity(xt, n * wl.dt).t().contiguous() for n in range(nsteps + 1)])
    c0 = W.two_blobs(xt).contiguous()
    cur = c0.clone()
    chat = torch.empty(N, dtype=tr.scalar_dtype, device="cuda")
    same_dtype = chat.dtype == torch.float64  # the result can be handed back as the next scalar
    X = torch.empty((3, N), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    state = {"n": 0}

    def step(ev=None):
        n = state["n"] % nsteps
        if n == 0:
            # the run restarts from the initial condition every 50 steps
            tr.set_velocity(0, U[0])
            cur.copy_(c0)
        else:
            tr.swap_levels()
        # the new velocity level and the scalar of this step (the initial
        # condition, or the last step's result; float32 results are widened
        # to float64 first), in one ingestion pass
        tr.set_fields(1, U[n + 1], cur if (n == 0 or not same_dtype) else chat)
        if ev is not None:
            ev[0].record()
        mmoc.mmoc_trace_step(tr.ctx, wl.dt, S, chat, X)
        if ev is not None:
            ev[1].record()
        if not same_dtype:
            cur.copy_(chat)
        state["n"] += 1

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tr.reset_stats()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(steps):
        step(evs[k])
    e1.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ms = max(wall_ms, e0.elapsed_time(e1)) / steps
    kern = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    st = {k: (int(v) if isinstance(v, (int, np.integer)) else float(v)) for k, v in tr.stats().items()}
    tr.close()
    return {"N": N, "value": N / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": kern, "stats": st}


def time_surrogate(wl, S, steps, warmup, results):
    """Steps 1-10 of the run traced by RK4 and recorded, 2e6 pairs sampled,
    30 epochs of training; then steps 11-20 (cycled) with the surrogate (1%
    check sample, tolerance 1e-4, float32-fields RK4 check and fallback)."""
    import torch
    from paper_2103_02388_amd import mmoc
    from paper_2103_02388_amd import workloads as W

    tr = mmoc.Tracer.from_workload(wl, precision=mmoc.MMOC_FP32_FIELDS)
    N = tr.N
    tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, W.SWIRL_T], 2.0)
    x = tr.dof_coords()
    xt = x.t().contiguous()
    U = torch.stack([W.swirl_velocity(xt, n * wl.dt).t().contiguous() for n in range(21)])
    c0 = W.two_blobs(xt).contiguous()
    tr.set_scalar(c0)
    for n in range(10):
        tr.set_velocity(0, U[n])
        tr.set_velocity(1, U[n + 1])
        _, X = tr.trace_step(wl.dt, S)
        tr.mlp_record((n + 1) * wl.dt, wl.dt, X, 10 * N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = tr.mlp_train(2_000_000, 30, batch=8192, lr=1e-3, seed=5)
    t_train = time.perf_counter() - t0
    chat = torch.empty(N, dtype=torch.float32, device="cuda")
    X = torch.empty((3, N), dtype=torch.float64, device="cuda")
    cur = c0.clone()

    def step(k):
        n = 10 + k % 10
        tr.set_velocity(0, U[n])
        tr.set_velocity(1, U[n + 1])
        tr.set_scalar(cur)
        mmoc.mmoc_trace_step_surrogate(tr.ctx, (n + 1) * wl.dt, wl.dt, S, 0.01, 1e-4, n, chat, X)
        cur.copy_(chat)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    tr.reset_stats()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = tr.stats()
    tr.close()
    fb = (st["n_checked"] + st["n_fallback"]) / (N * steps)
    out = {"value": N / (ms * 1e-3), "ms_per_step": ms, "train_seconds": t_train, "final_loss": loss,
           "rk4_fraction": fb, "max_check_residual": st["max_check_residual"], "tolerance": 1e-4,
           "note": "steps 11-20 (cycled) of the swirl run; the network is trained on steps 1-10; "
                   "check sample and fallback traced by the float32-fields RK4 tracer"}
    if "fp64" in results:
        out["speedup_vs_fp64_step"] = out["value"] / results["fp64"]["value"]
    if "fp32" in results:
        out["speedup_vs_fp32_step"] = out["value"] / results["fp32"]["value"]
    if "fp32f" in results:
        out["speedup_vs_fp32_fields_step"] = out["value"] / results["fp32f"]["value"]
    return out


def time_large(wl, step, paths, reps=3):
    """The trace kernel alone on a large workload (the rising plumes at 1.7e7
    particles, or the 1.7e8-particle shell), per path: step `step` of the
    run, RK4 with the workload's sub-steps, HIP events around each of `reps`
    launches after one warm-up launch."""
    import torch
    from paper_2103_02388_amd import mmoc

    prec = {"fp64": mmoc.MMOC_FP64, "fp32": mmoc.MMOC_FP32_MIXED, "fp32f": mmoc.MMOC_FP32_FIELDS}
    names = {"fp64": "fp64", "fp32": "fp32_mixed", "fp32f": "fp32_fields"}
    out = {"workload": wl.description, "level": wl.level}
    for path in paths:
        tr = mmoc.Tracer.from_workload(wl, precision=prec[path])
        xt = tr.dof_coords().t().contiguous()
        t_n = step * wl.dt
        if wl.stationary:
            tr.set_stationary(True)
            tr.set_velocity(0, wl.velocity(xt, t_n).t().contiguous())
        else:
            tr.set_velocity(0, wl.velocity(xt, t_n).t().contiguous())
            tr.set_velocity(1, wl.velocity(xt, t_n + wl.dt).t().contiguous())
        tr.set_scalar(wl.scalar0(xt).contiguous())
        del xt
        chat = torch.empty(tr.N, dtype=tr.scalar_dtype, device="cuda")
        X = torch.empty((wl.dim, tr.N), dtype=torch.float64, device="cuda")
        mmoc.mmoc_trace_step(tr.ctx, wl.dt, wl.substeps, chat, X)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            mmoc.mmoc_trace_step(tr.ctx, wl.dt, wl.substeps, chat, X)
            b.record()
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out["particles"] = tr.N
        out[names[path]] = {"kernel_ms": ms, "trace_only_particles_per_s": tr.N / (ms * 1e-3)}
        tr.close()
        del chat, X
        torch.cuda.empty_cache()
    if "fp64" in out:
        for k in ("fp32_mixed", "fp32_fields"):
            if k in out:
                out[k]["speedup_vs_fp64"] = out["fp64"]["kernel_ms"] / out[k]["kernel_ms"]
    return out


def spmv_bytes(N, nnz):
    """algorithmic HBM bytes of y = V x in CSR: values and column indices
    once, row pointers, x read once, y written once"""
    return nnz * (8 + 4) + (N + 1) * 4 + N * 8 + N * 8


def time_diffusion():
    """Advection-diffusion on the blended annulus (Sec. 4, Table 4's largest
    mesh: level 6, 197,376 P2 DoFs, kappa = 1e-3, tau = 2 pi / 63, one RK4
    step per tau).  One step = the trace of every DoF and the implicit-Euler
    diffusion solve (Jacobi-preconditioned CG to 1e-12) with the exact
    solution as Dirichlet data, as in Alg. 1; the Dirichlet data of all 63
    steps are resident before timing.  The matrix assembly is timed on its
    own.  The SpMV roofline entry is for the CSR operator apply on a larger
    annulus (level 8, 3,148,800 DoFs) whose matrix does not fit in the
    last-level cache."""
    import math
    import torch
    from paper_2103_02388_amd import mmoc
    from paper_2103_02388_amd import workloads as W

    kappa = 1e-3
    wl = W.annulus2d(level=6, kappa=kappa)
    tr = mmoc.Tracer.from_workload(wl)
    N = tr.N
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nnz = tr.fe_assemble()
    setup_ms = (time.perf_counter() - t0) * 1e3
    x = tr.dof_coords()
    xt = x.t().contiguous()
    hill = wl.extra["hill"]
    tr.set_stationary(True)
    tr.set_velocity(0, wl.velocity(xt).t().contiguous())
    c0 = hill(xt, hill.t0).contiguous()
    G = torch.stack([hill(xt, hill.t0 + (k + 1) * wl.dt) for k in range(wl.steps)]).contiguous()
    ch = torch.empty_like(c0)

    def run(timed):
        c, nxt = c0.clone(), torch.empty_like(c0)
        iters, tr_ms = 0, 0.0
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(wl.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(wl.steps):
            tr.set_scalar(c)
            ev[k][0].record()
            tr.trace_step(wl.dt, wl.substeps, c_hat=ch, want_X=False)
            ev[k][1].record()
            nxt, info = tr.diffusion_step(ch, wl.dt, kappa, 1.0, dirichlet=G[k], out=nxt)
            iters += info["iterations"]
            c, nxt = nxt, c
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        tr_ms = sum(a.elapsed_time(b) for a, b in ev)
        return c, wall, tr_ms, iters

    run(False)
    c, wall, tr_ms, iters = run(True)
    ex = G[-1]
    e = (ex - c).contiguous()
    h0 = math.sqrt(float((e * tr.fe_apply(mmoc.MMOC_MAT_MASS, e)).sum()))
    ep = float(c.max() / ex.max() - 1.0)
    steps = wl.steps
    diff_ms = wall - tr_ms
    small_ms = spmv_time(tr)
    tr.close()
    return {
        "workload": "annulus2d: r in [0.5, 1.5], 6x2 macro triangles, radial blending, level 6, 197376 P2 DoFs; "
                    "rotation (-x2, x1); Gaussian hill kappa 1e-3; tau = 2 pi/63, one RK4 step per tau, 63 steps; "
                    "implicit Euler, Jacobi CG to 1e-12, Dirichlet data from the exact solution",
        "dofs": N, "nnz": nnz, "steps": steps,
        "value": N / (wall / steps * 1e-3), "unit": "DoFs advanced/s (trace + diffusion solve)",
        "ms_per_step": wall / steps, "trace_ms_per_step": tr_ms / steps, "diffusion_ms_per_step": diff_ms / steps,
        "cg_iterations_per_step": iters / steps, "us_per_cg_iteration": diff_ms * 1e3 / max(iters, 1),
        "assembly_ms": setup_ms, "H0_error": h0, "E_peak": ep, "paper_H0": 4.32e-3, "paper_E_peak": 3.98e-3,
        "spmv_table4_mesh_us": small_ms * 1e3,
        "roofline": spmv_roofline(),
    }


def spmv_time(t, reps=50):
    """mean duration (ms) of the mass-matrix apply, HIP events around the
    launches on the stream they run on"""
    import torch
    from paper_2103_02388_amd import mmoc
    v = torch.ones(t.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(v)
    for _ in range(3):
        t.fe_apply(mmoc.MMOC_MAT_MASS, v, y)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        t.fe_apply(mmoc.MMOC_MAT_MASS, v, y)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def spmv_roofline():
    """The CSR operator apply on the level-8 annulus (3,148,800 DoFs, 36M
    entries, 497 MB per apply: beyond the last-level cache)."""
    from paper_2103_02388_amd import mmoc
    from paper_2103_02388_amd import workloads as W
    big = mmoc.Tracer.from_workload(W.annulus2d(level=8))
    bnnz = big.fe_assemble()
    big_ms = spmv_time(big)
    bN = big.N
    big.close()
    achieved = spmv_bytes(bN, bnnz) / (big_ms * 1e-3)
    return {"bound": "hbm", "kernel": "spmv_kernel (CSR, mass matrix)", "mesh": "annulus2d level 8",
            "dofs": bN, "nnz": bnnz, "kernel_ms": big_ms, "bytes_per_launch": spmv_bytes(bN, bnnz),
            "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": achieved / PEAK_HBM,
            "traffic": None}


def cpu_baseline(wl, S):
    """The CPU oracle (unchanged, single-threaded) on the same step's
    particles with its own copy of the same inputs: full steps repeated until
    about 10 s of single-core work."""
    import torch
    from oracle import oracle as O
    from paper_2103_02388_amd import workloads as W

    om = O.Mesh.from_workload(wl)
    xc = om.dof_coords()
    xt = torch.from_numpy(np.ascontiguousarray(xc.T))
    u0 = np.ascontiguousarray(W.swirl_velocity(xt, 7 * wl.dt).numpy().T)
    u1 = np.ascontiguousarray(W.swirl_velocity(xt, 8 * wl.dt).numpy().T)
    c = W.two_blobs(xt).numpy()
    reps, total = 0, 0.0
    while reps == 0 or (total < 10.0 and reps < 40):
        t0 = time.perf_counter()
        om.trace(u0, u1, c, wl.dt, S, threads=1)
        total += time.perf_counter() - t0
        reps += 1
    try:
        cpu = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        cpu = "unknown"
    return {"value": om.N * reps / total, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": "%d x %d particles: the full swirl3d step 7 -> 8 repeated, RK4 %d sub-steps, float64, "
                      "single thread; host CPU: %s (%d logical cores)" % (reps, om.N, S, cpu, os.cpu_count() or 0),
            "seconds": total}


if __name__ == "__main__":
    main()
