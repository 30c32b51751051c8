#!/usr/bin/env python3
"""Throughput of the MMOC particle tracer on one MI355X.

Headline workload: the thick spherical shell r in [0.55, 1] -- an
icosahedral macro mesh of 3840 tetrahedra with radial blending, refined to
level 5, 168,428,034 P2 DoFs = particles; a stationary velocity from 16
seeded toroidal/poloidal spherical-harmonic modes (no normal flow at either
radius), the scalar a step at r = 0.8 plus 1% nodal noise, dt = 5 h_min /
max|u| (CFL 5 on the radial micro edge), 4 RK4 sub-steps; the largest
configuration that fits one GPU.  The tracer runs in float64, the paper's
precision (error <= 1e-12 against the CPU oracle).

One timed step is one full MMOC advection step of the time loop: the
current scalar is copied into the library's block layout (field
ingestion), then every particle is created, traced back with RK4 through
the stationary velocity and the scalar evaluated at its departure point;
the result is the next step's scalar.  The velocity and the initial scalar
are resident in device memory before timing starts.  value = particles per
second of the float64 tracer.  Beside it, on the same shell: the
float32-mixed tracer (float32 stages, location and interpolation, float64
tie-break at macro faces, <= 1e-5) and the float32-fields tracer (float32
records, float64 arithmetic), and the measured error of the first step
against the oracle on a seeded subset of 1e6 particles.  Sub-results: the
3D swirl (274,625 particles, time-dependent velocity, all three tracers),
the trace kernels on the rising plumes (1.7e7 particles), the surrogate
step and the advection-diffusion run of Table 4 with its CG solve.

The roofline entry is for the dominant kernel (the float64 trace on the
shell): its algorithmic flops per particle (FMA = 2, see
flops_per_particle) over its mean duration from HIP events recorded around
each launch on the stream it runs on.  cpu_baseline times the CPU oracle
(float64 C, unchanged) on the seeded 1e6-particle subset of the same step,
on all host cores (one thread per core, disjoint particle ranges) and on
one core.
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
TRAFFIC = os.path.join(ROOT, "profiles", "trace_fp64_shell3d_traffic.json")
SUBSET = 1_000_000  # particles of the oracle's share of the shell step


def flops_per_particle(dim, nlev, S, blend=False):
    """Algorithmic flops of one particle's step (FMA = 2).  Per stage
    evaluation: reference coordinates (offset dim, matrix 2 dim^2, lambda_0
    dim + 1), with blending the inverse map Phi^-1(y) = y c |y| / (n.y) first
    (two dot products 4 dim - 2, a square root, a product and a quotient, and
    dim fused scalings: 6 dim + 1), micro location and P2 basis (Kuhn sums
    2(dim - 1), scaling 2 dim, fractional parts 2 dim, micro barycentrics
    dim + 1, vertex shape functions 3 (dim + 1), edge shape functions 2 per
    edge), the P2 sums (2 per node, component and level), the time
    interpolation (3 dim, two levels only) and the stage update (4 dim);
    2 dim per sub-step for the departure point; the scalar evaluation at the
    end.  The first stage evaluation (at the particle's own DoF) is counted
    as a full one; particle creation is not counted."""
    nn = (dim + 1) * (dim + 2) // 2
    ref = dim + 2 * dim * dim + dim + 1 + ((6 * dim + 1) if blend else 0)
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
    """The committed rocprofv3 counter summary of the float64 trace kernel on
    the shell, if it was taken on the current kernel source (else None)."""
    try:
        d = json.load(open(TRAFFIC))
        sha = hashlib.sha256(open(TRACE_SRC, "rb").read()).hexdigest()
        return d if d.get("source_sha256") == sha else None
    except Exception:
        return None


def traffic_entry():
    """HBM bytes per launch of the float64 trace kernel on the shell
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counts)."""
    d = counter_summary()
    return d["hbm_bytes_per_launch"] if d else None


ELEM_CACHE = 1


def options(path="fp64"):
    from paper_2103_02388_amd import mmoc
    o = mmoc.mmoc_default_options()
    o.elem_cache = ELEM_CACHE
    if path == "fp32m":
        o.eps32_micro = 0.0
    return o


def log(msg):
    """progress line on stderr (the JSON result is the only stdout line)"""
    print("[bench %.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


T0 = time.perf_counter()
# "fp32" is the float32-mixed tracer with its default tie bands (macro and
# micro faces); "fp32m" the same with the micro band off (eps32_micro = 0)
PREC = {"fp64": "MMOC_FP64", "fp32": "MMOC_FP32_MIXED", "fp32f": "MMOC_FP32_FIELDS", "fp32m": "MMOC_FP32_MIXED"}
NAMES = {"fp64": "fp64", "fp32": "fp32_mixed", "fp32f": "fp32_fields", "fp32m": "fp32_mixed_macro_band_only"}
ERR_BOUND = {"fp64": 1e-12, "fp32": 1e-5, "fp32f": 1e-6, "fp32m": 1e-5}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--substeps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--paths", default="fp64,fp32,fp32m,fp32f",
                    help="tracer paths timed on the shell and the swirl (fp64 is the headline)")
    ap.add_argument("--no-swirl", action="store_true")
    ap.add_argument("--no-diffusion", action="store_true")
    ap.add_argument("--no-plume", action="store_true")
    ap.add_argument("--no-elem-cache", action="store_true",
                    help="trace without the per-lane element cache (options.elem_cache = 0)")
    ap.add_argument("--surrogate-only", action="store_true", help="only the surrogate legs")
    ap.add_argument("--shell-only", action="store_true",
                    help="only the shell legs of --paths, no oracle (for profiling their kernels)")
    ap.add_argument("--swirl-only", action="store_true",
                    help="only the swirl legs of --paths (for profiling their kernels)")
    ap.add_argument("--plume-only", action="store_true",
                    help="only the trace kernels on the rising plumes, paths from --paths (for profiling them)")
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
    S = args.substeps
    global ELEM_CACHE
    ELEM_CACHE = 0 if args.no_elem_cache else 1
    if args.surrogate_only:
        print(json.dumps({"surrogate": time_surrogate(S, {})}), flush=True)
        return
    if args.plume_only:
        paths = [p for p in args.paths.split(",") if p in PREC]
        print(json.dumps({"plume3d": time_large(W.plume3d(), 120, paths)}), flush=True)
        return
    paths = args.paths.split(",")
    if "fp64" not in paths:
        paths = ["fp64"] + paths
    if args.swirl_only:
        wl = W.swirl3d()
        print(json.dumps({"swirl3d": {p: time_path(wl, p, S, args.steps, args.warmup) for p in paths}}), flush=True)
        return
    wl3 = W.shell3d()
    shell = time_shell(wl3, paths, S, args.steps, args.warmup,
                       oracle=not (args.no_cpu_baseline or args.shell_only))
    r = shell["fp64"]
    N = shell["particles"]
    if args.shell_only:
        print(json.dumps({"shell3d": shell}), flush=True)
        return
    fpp = flops_per_particle(3, 1, S, blend=True)
    bpp64 = bytes_per_particle(3, 1, 8)
    achieved = fpp * N / (r["kernel_ms"] * 1e-3)
    cs = counter_summary() or {}
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
        "config": {"workload": "shell3d: thick spherical shell r in [0.55,1], 3840 icosahedral macro tets with radial "
                               "blending, level 5, 168428034 P2 particles; stationary velocity of 16 seeded "
                               "toroidal/poloidal modes (l<=8); step at r=0.8 plus 1%% noise; dt = 5 h_min/max|u|; "
                               "RK4 with %d sub-steps; scalar ingestion + trace per step" % S,
                   "particles": N, "substeps": S, "precision": "fp64", "error_bound_vs_oracle": 1e-12},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU,
                     "traffic": traffic_entry(),
                     "kernel": "trace_fp64_kernel<3,1,1,double,false,2> (shell, float64)",
                     "kernel_ms": r["kernel_ms"], "flop_per_particle": fpp, "bytes_per_particle": bpp64,
                     "hbm_GBps_algorithmic": bpp64 * N / (r["kernel_ms"] * 1e-3) / 1e9,
                     "hbm_frac_algorithmic": bpp64 * N / (r["kernel_ms"] * 1e-3) / PEAK_HBM,
                     "hbm_GBps_measured": (traffic_entry() / (r["kernel_ms"] * 1e-3) / 1e9
                                           if traffic_entry() is not None else None),
                     "l1_tag_lookups_per_cu_cycle": cs.get("l1_tag_lookups_per_cu_cycle")},
        "trace_only_particles_per_s": N / (r["kernel_ms"] * 1e-3),
        "stats": r["stats"],
    }
    for path in paths:
        if path != "fp64":
            f = shell[path]
            out[NAMES[path]] = dict(f, speedup_vs_fp64_step=f["value"] / r["value"],
                                    speedup_vs_fp64_trace=r["kernel_ms"] / f["kernel_ms"])
    if "error_vs_oracle" in shell:
        out["error_vs_oracle"] = shell["error_vs_oracle"]
    swirl = {}
    if not args.no_swirl:
        wl = W.swirl3d()
        for path in paths:
            log("swirl3d: %s" % path)
            swirl[path] = time_path(wl, path, S, args.steps, args.warmup)
        out["swirl3d"] = {"workload": "swirl3d: unit cube, 6 Kuhn macro tets, level 5, 274625 P2 particles, LeVeque "
                                      "swirl T=1.5, dt=T/20 (CFL~5), RK4 with %d sub-steps, 50-step run; velocity "
                                      "level + scalar ingestion and trace per step" % S,
                          "particles": swirl["fp64"]["N"],
                          "roofline_fp64_trace": {
                              "flop_per_particle": flops_per_particle(3, 2, S),
                              "frac": flops_per_particle(3, 2, S) * swirl["fp64"]["N"]
                              / (swirl["fp64"]["kernel_ms"] * 1e-3) / PEAK_FP64_VALU}}
        for path in paths:
            f = dict(swirl[path])
            f.pop("N")
            f["trace_only_particles_per_s"] = swirl["fp64"]["N"] / (f["kernel_ms"] * 1e-3)
            f["error_bound_vs_oracle"] = ERR_BOUND[path]
            if path != "fp64":
                f["speedup_vs_fp64_step"] = f["value"] / swirl["fp64"]["value"]
            out["swirl3d"][NAMES[path]] = f
    if not args.no_surrogate:
        log("surrogate")
        out["surrogate"] = time_surrogate(S, swirl)
    if not args.no_plume:
        log("plume3d")
        out["plume3d"] = time_large(W.plume3d(), 120, ("fp64", "fp32", "fp32m", "fp32f"))
    if not args.no_diffusion:
        log("diffusion")
        out["diffusion"] = time_diffusion()
    if "cpu_baseline" in shell:
        out["cpu_baseline"] = shell["cpu_baseline"]
    print(json.dumps(out), flush=True)


def shell_fields(wl):
    """The shell's velocity and initial scalar at the library's DoF positions
    (the seeded generators, evaluated on the GPU), unique order."""
    import torch
    from paper_2103_02388_amd import mmoc
    tr = mmoc.Tracer.from_workload(wl, precision=mmoc.MMOC_FP64)
    xt = tr.dof_coords().t().contiguous()
    tr.close()
    u = wl.velocity(xt).t().contiguous()
    c = wl.scalar0(xt).contiguous()
    del xt
    torch.cuda.empty_cache()
    return u, c


def time_shell(wl, paths, S, steps, warmup, oracle=True):
    """The shell's time loop per tracer path: warm-up steps, then `steps`
    timed steps (scalar ingestion + trace), HIP events around every trace
    launch.  With `oracle`, the first step of every path is compared with
    the CPU oracle on a seeded subset of SUBSET particles, and the oracle's
    time for that subset is the CPU baseline."""
    import torch
    from paper_2103_02388_amd import mmoc

    log("shell: evaluating the fields")
    u, c = shell_fields(wl)
    N = c.numel()
    out = {"workload": wl.description, "level": wl.level, "particles": N}
    ids = np.sort(np.random.default_rng(7).choice(N, SUBSET, replace=False))
    first = {}
    for path in paths:
        log("shell: %s context" % path)
        tr = mmoc.Tracer.from_workload(wl, precision=getattr(mmoc, PREC[path]), options=options(path))
        assert tr.N == N
        tr.set_stationary(True)
        tr.set_velocity(0, u)
        cur = c.clone()
        chat = torch.empty(N, dtype=tr.scalar_dtype, device="cuda")
        X = torch.empty((3, N), dtype=torch.float64, device="cuda")
        same = chat.dtype == torch.float64
        if oracle:
            tr.set_scalar(c)
            mmoc.mmoc_trace_step(tr.ctx, wl.dt, S, chat, X)
            idt = torch.from_numpy(ids).cuda()
            first[path] = (chat[idt].double().cpu().numpy(), X[:, idt].cpu().numpy(),
                           tr.dof_coords()[:, idt].cpu().numpy())
            del idt
        state = {"cur": cur, "chat": chat}

        def step(ev=None):
            tr.set_scalar(state["cur"])
            if ev is not None:
                ev[0].record()
            mmoc.mmoc_trace_step(tr.ctx, wl.dt, S, state["chat"], X)
            if ev is not None:
                ev[1].record()
            if same:
                state["cur"], state["chat"] = state["chat"], state["cur"]
            else:
                state["cur"].copy_(state["chat"])

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
        entry = {"value": N / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": kern,
                 "trace_only_particles_per_s": N / (kern * 1e-3), "error_bound_vs_oracle": ERR_BOUND[path],
                 "stats": st}
        if path in ("fp32", "fp32m"):
            entry["tieband_fraction"] = st["n_tieband"] / max(1, st["n_particles"])
        out[path] = entry
        log("shell: %s %.3f ms per step, trace %.3f ms" % (path, ms, kern))
        tr.close()
        del cur, chat, X, state
        torch.cuda.empty_cache()
    if oracle and "fp64" in first:
        base, err = cpu_baseline_shell(wl, u, c, S, ids, first)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = err
    return out


def cpu_baseline_shell(wl, u, c, S, ids, first):
    """The CPU oracle (float64 C, unchanged) on the seeded subset `ids` of the
    shell's first step, with the same input arrays as the GPU: timed on all
    host cores (disjoint particle ranges, one thread each, at most 16: the
    GPU's share of the host) and on one core; its result also gives every
    path's measured error on the subset."""
    from oracle import oracle as O

    log("oracle: shell mesh")
    t0 = time.perf_counter()
    om = O.Mesh.from_workload(wl)
    xc = om.dof_coords()
    setup_s = time.perf_counter() - t0
    uh = u.cpu().numpy()
    ch = c.cpu().numpy()
    n = len(ids)
    threads = max(1, min(os.cpu_count() or 1, 16))
    reps, tot = 0, 0.0
    while reps == 0 or (tot < 5.0 and reps < 20):
        t0 = time.perf_counter()
        chr_, Xr, st = om.trace(uh, None, ch, wl.dt, S, ids=ids, threads=threads)
        tot += time.perf_counter() - t0
        reps += 1
    multi = n * reps / tot
    log("oracle: %d threads %.3g particles/s" % (threads, multi))
    t0 = time.perf_counter()
    om.trace(uh, None, ch, wl.dt, S, ids=ids, threads=1)
    t1 = time.perf_counter() - t0
    single = n / t1
    try:
        cpu = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        cpu = "unknown"
    base = {"value": multi, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": "seeded subset of %d of the shell's 168428034 particles, first step (RK4 %d sub-steps, "
                      "float64), %d repetitions on %d threads (disjoint ranges); host CPU: %s, %d logical cores"
                      % (n, S, reps, threads, cpu, os.cpu_count() or 0),
            "seconds": tot,
            "one_core": {"value": single, "cores": 1, "sample": "the same %d particles, one thread" % n,
                         "seconds": t1},
            "oracle_mesh_setup_seconds": setup_s}
    err = {"subset": n, "dof_coords_max_abs": float(np.abs(first["fp64"][2] - xc[:, ids]).max())}
    # the step scalar has O(1) jumps at r = 0.8: chat is compared where the
    # departure point is not within 0.02 of the jump (the size of a micro
    # element there), beside the plain maximum
    far = np.abs(np.linalg.norm(Xr, axis=0) - 0.8) > 0.02
    for path, (chg, Xg, _) in first.items():
        err[NAMES[path]] = {"X_rel": float(np.abs(Xg - Xr).max() / max(1.0, np.abs(Xr).max())),
                            "chat_max_abs": float(np.abs(chg - chr_).max()),
                            "chat_max_abs_off_step": float(np.abs(chg - chr_)[far].max())}
    return base, err


def time_path(wl, path, S, steps, warmup):
    import torch
    from paper_2103_02388_amd import mmoc
    from paper_2103_02388_amd import workloads as W

    tr = mmoc.Tracer.from_workload(wl, precision=getattr(mmoc, PREC[path]), options=options(path))
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


def surrogate_run(wl, vel, train, run, box_hi, U, period, prec_name="fp64", S=4, tol=1e-4, pred=1, scale=1e-4,
                  scalar=None):
    """The learned flow-map surrogate in a time loop:
    steps `train` (step n covers [t_{n-1}, t_n]) traced by RK4 with S
    sub-steps and recorded, the network trained on 2e6 pairs drawn from
    them (30 epochs), then steps `run` with the surrogate step (1% check
    sample, tolerance tol, per-tile fallback).  The network corrects the
    RK4 trace with `pred` sub-steps; its time input is the phase t mod
    `period` (0: t).  The velocity levels of every run step are resident in
    device memory before timing; one timed step is the ingestion of the new
    velocity level and the scalar plus the surrogate step.  The plain RK4
    step with S sub-steps of the same context is timed on the same steps."""
    import torch
    from paper_2103_02388_amd import mmoc

    tr = mmoc.Tracer.from_workload(wl, precision=getattr(mmoc, PREC[prec_name]))
    N, dt = tr.N, wl.dt
    tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, box_hi], U)
    tr.mlp_set_predictor(pred, scale, period)
    xt = tr.dof_coords().t().contiguous()
    c0 = (scalar or wl.scalar0)(xt).contiguous()
    levels = {n: vel(xt, n * dt).t().contiguous() for n in range(min(train) - 1, max(run) + 1)}
    del xt
    cur = c0.clone()
    for n in train:
        tr.set_velocity(0, levels[n - 1])
        tr.set_velocity(1, levels[n])
        tr.set_scalar(cur)
        ch, X = tr.trace_step(dt, S)
        tr.mlp_record(n * dt, dt, X, len(train) * N)
        cur = ch.double() if ch.dtype != torch.float64 else ch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = tr.mlp_train(2_000_000, 30, batch=8192, lr=1e-3, seed=5)
    t_train = time.perf_counter() - t0
    chat = torch.empty(N, dtype=tr.scalar_dtype, device="cuda")
    X = torch.empty((3, N), dtype=torch.float64, device="cuda")
    runs = list(run)

    def loop(surrogate):
        c = c0.clone()
        tr.set_velocity(1, levels[runs[0] - 1])
        rk4 = []
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in runs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, n in enumerate(runs):
            tr.swap_levels()
            tr.set_fields(1, levels[n], c)
            if surrogate:
                tr.reset_stats()
            ev[k][0].record()
            if surrogate:
                mmoc.mmoc_trace_step_surrogate(tr.ctx, n * dt, dt, S, 0.01, tol, n, chat, X)
            else:
                mmoc.mmoc_trace_step(tr.ctx, dt, S, chat, X)
            ev[k][1].record()
            if surrogate:
                st = tr.stats()  # synchronises: the per-step fraction traced by RK4
                rk4.append((st["n_checked"] + st["n_fallback"]) / N)
            c.copy_(chat)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / len(runs)
        return float(np.mean([a.elapsed_time(b) for a, b in ev])), wall, rk4

    loop(True)  # warm-up pass
    sur_ms, sur_wall, rk4 = loop(True)
    rk_ms, rk_wall, _ = loop(False)
    tr.close()
    kept = [f for f in rk4 if f < 0.5]
    return {"precision": prec_name, "train_steps": [min(train), max(train)], "run_steps": [min(run), max(run)],
            "tolerance": tol, "predictor_substeps": pred, "correction_scale": scale, "time_period": period,
            "train_seconds": t_train, "final_loss": loss,
            "surrogate_ms": sur_ms, "rk4_ms": rk_ms,
            "speedup_vs_rk4_same_precision": rk_ms / sur_ms,
            "rk4_fraction_mean": float(np.mean(rk4)), "rk4_fraction_max": float(np.max(rk4)),
            "steps_keeping_the_network": len(kept), "steps": len(rk4),
            "rk4_fraction_per_step": [round(f, 4) for f in rk4],
            "note": "ms are HIP-event means of the step call (surrogate: predictor, network, check on a second "
                    "stream, residuals, finish pass); the per-step statistics synchronise, so the loop's wall "
                    "time is not the rate"}


def time_surrogate(S, swirl):
    """The swirl run (level 5, 274,625 particles; trained on steps 1-10,
    steps 11-110) and its full-period variant (trained on steps 1-40, one
    period of the velocity; steps 41-140); the rising plumes (level 7,
    16,974,593 particles; trained on steps 1-10, steps 11-200), with float64
    and with float32 records."""
    from paper_2103_02388_amd import workloads as W
    wl = W.swirl3d(steps=140)
    per = 2.0 * W.SWIRL_T
    out = {"swirl3d_train_1_10_run_11_110": surrogate_run(wl, W.swirl_velocity, range(1, 11), range(11, 111), per, 2.0, per, S=S),
           "swirl3d_full_period": surrogate_run(wl, W.swirl_velocity, range(1, 41), range(41, 141), per, 2.0, per,
                                                S=S)}
    if "fp64" in swirl:
        for k in ("swirl3d_train_1_10_run_11_110", "swirl3d_full_period"):
            out[k]["speedup_vs_fp64_swirl_trace"] = swirl["fp64"]["kernel_ms"] / out[k]["surrogate_ms"]
    pl = W.plume3d()
    out["plume3d_train_1_10_run_11_200"] = surrogate_run(pl, pl.velocity, range(1, 11), range(11, 201), pl.extra["T"],
                                           pl.extra["umax"], 0.0, S=S)
    # the same with float32 records (predictor, check and fallback through
    # the element cache), against the float32-fields and float64 RK4 steps
    f = surrogate_run(pl, pl.velocity, range(1, 11), range(11, 201), pl.extra["T"], pl.extra["umax"], 0.0, S=S,
                      prec_name="fp32f")
    f["speedup_vs_fp64_rk4"] = out["plume3d_train_1_10_run_11_200"]["rk4_ms"] / f["surrogate_ms"]
    out["plume3d_train_1_10_run_11_200_fp32_fields"] = f
    return out


def time_large(wl, step, paths, reps=3):
    """The trace kernel alone on a large workload (the rising plumes at 1.7e7
    particles, or the 1.7e8-particle shell), per path: step `step` of the
    run, RK4 with the workload's sub-steps, HIP events around each of `reps`
    launches after one warm-up launch."""
    import torch
    from paper_2103_02388_amd import mmoc

    out = {"workload": wl.description, "level": wl.level}
    for path in paths:
        tr = mmoc.Tracer.from_workload(wl, precision=getattr(mmoc, PREC[path]), options=options(path))
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
        nb = tr.N * bytes_per_particle(wl.dim, 1 if wl.stationary else 2, 8 if path == "fp64" else 4)
        out[NAMES[path]] = {"kernel_ms": ms, "trace_only_particles_per_s": tr.N / (ms * 1e-3),
                            "algorithmic_bytes": nb, "hbm_GBps_algorithmic": nb / (ms * 1e-3) / 1e9}
        tr.close()
        del chat, X
        torch.cuda.empty_cache()
    if "fp64" in out:
        for k in ("fp32_mixed", "fp32_mixed_macro_band_only", "fp32_fields"):
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


if __name__ == "__main__":
    main()
