#!/usr/bin/env python3
"""Throughput of the MMOC particle tracer on one MI355X.

Workload (default): the 3D swirl -- unit cube of 6 Kuhn macro tetrahedra
refined to level 5, 65^3 = 274625 P2 DoFs = particles, LeVeque's deformation
field with g(t) = cos(pi t / 1.5) sampled at every time level, two Gaussian
blobs as the scalar, dt = T/20 (CFL ~ 5), 4 RK4 sub-steps, 50 time steps.

One timed step is one full MMOC advection step of the time loop: the new
velocity level and the current scalar are copied into the library's block
layout (field ingestion), then every particle is created, traced back with
RK4 and the scalar evaluated at its departure point; the result is the next
step's scalar.  All inputs (every velocity level of the run) are resident in
device memory before timing starts.  value = particles traced per second.

Printed: one JSON line.  The dominant kernel's roofline entry uses its
algorithmic flops per particle (FMA = 2, listed in the design notes) and the
kernel's mean duration from HIP events recorded around each launch inside the
timed loop.  cpu_baseline runs the CPU oracle (single-threaded FP64 C) on a
bounded sample of the same workload.
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

# algorithmic flops per particle of one step (FMA counted as 2), per path:
# per stage evaluation 25 (reference coordinates) + 44 (micro location and
# P2 basis) + 20 per component and level (P2 sums) + 9 (time lerp, 2 levels)
# + 12 (stage update); per sub-step 6 more; the scalar evaluation 89.
def flops_per_particle(dim, nlev, S):
    nn = (dim + 1) * (dim + 2) // 2
    ref = dim + 2 * dim * dim + dim + 1
    micro = (2 * (dim - 1) + 2 * dim + 2 * dim) + (dim + 1) + 3 * (dim + 1) + 2 * (nn - dim - 1)
    gather = 2 * nn * dim * nlev + (3 * dim if nlev == 2 else 0)
    stage = 4 * dim
    per_eval = ref + micro + gather + stage
    scalar = ref + micro + 2 * nn
    return S * (4 * per_eval + 2 * dim) + scalar


# compulsory HBM bytes per particle: every unique field value read once,
# every output written once
def bytes_per_particle(dim, nlev, real_bytes):
    return dim * nlev * real_bytes + real_bytes + real_bytes + dim * 8


PEAK_FP64_VALU = 78.6e12
PEAK_FP32_VALU = 78.6e12  # packed FP32 is not used (157.3 TFLOP/s only with packed math)
PEAK_HBM = 8.0e12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--substeps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="particles in the oracle sample (0: auto)")
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
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(particles are independent; see the sharding notes in DESIGN.md). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_02388_amd import mmoc
    from paper_2103_02388_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = W.swirl3d()
    prec = mmoc.MMOC_FP64 if args.precision == "fp64" else mmoc.MMOC_FP32_MIXED
    S = args.substeps
    tr = mmoc.Tracer.from_workload(wl, precision=prec)
    N = tr.N
    x = tr.dof_coords()
    xt = x.t().contiguous()
    nsteps = wl.steps
    U = torch.stack([W.swirl_velocity(xt, n * wl.dt).t().contiguous() for n in range(nsteps + 1)])
    c0 = W.two_blobs(xt).contiguous()
    torch.cuda.synchronize()

    cur = c0.clone()
    nxt = torch.empty(N, dtype=torch.float64, device=dev)
    chat = torch.empty(N, dtype=tr.scalar_dtype, device=dev)
    X = torch.empty((3, N), dtype=torch.float64, device=dev)
    state = {"n": 0}
    tr.set_velocity(0, U[0])
    tr.set_velocity(1, U[1])

    def step(ev=None):
        n = state["n"] % nsteps
        if n == 0:
            # the run restarts from the initial condition every 50 steps
            tr.set_velocity(0, U[0])
            cur.copy_(c0)
        else:
            tr.swap_levels()
        tr.set_velocity(1, U[n + 1])
        tr.set_scalar(cur)
        if ev is not None:
            ev[0].record()
        mmoc.mmoc_trace_step(tr.ctx, wl.dt, S, chat, X)
        if ev is not None:
            ev[1].record()
        if chat.dtype == torch.float64:
            cur.copy_(chat)
        else:
            cur.copy_(chat.double())
        state["n"] += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    tr.reset_stats()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(args.steps):
        step(evs[k])
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall_ms = (t1 - t0) * 1e3
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = max(wall_ms, gpu_ms) / args.steps
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    st = tr.stats()

    nlev = 2
    fpp = flops_per_particle(3, nlev, S)
    rb = 8 if prec == mmoc.MMOC_FP64 else 4
    bpp = bytes_per_particle(3, nlev, rb)
    achieved = fpp * N / (kern_ms * 1e-3)
    peak = PEAK_FP64_VALU if prec == mmoc.MMOC_FP64 else PEAK_FP32_VALU
    value = N / (ms_per_step * 1e-3)

    out = {
        "metric": "particles traced/sec (RK4+locate+P2 interp) at stated error; FP32/MLP vs FP64",
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == mmoc.MMOC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "swirl3d: unit cube, 6 Kuhn macro tets, level 5, 274625 P2 particles, "
                               "LeVeque swirl T=1.5, dt=T/20 (CFL~5), RK4 with %d sub-steps, 50-step run" % S,
                   "particles": N, "substeps": S, "precision": args.precision,
                   "error_bound_vs_fp64_oracle": 1e-12 if prec == mmoc.MMOC_FP64 else 1e-5},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "trace_%s_kernel<3,2,0>" % ("fp64" if prec == mmoc.MMOC_FP64 else "fp32"),
                     "kernel_ms": kern_ms, "flop_per_particle": fpp,
                     "hbm_GBps_algorithmic": bpp * N / (kern_ms * 1e-3) / 1e9,
                     "hbm_frac_algorithmic": bpp * N / (kern_ms * 1e-3) / PEAK_HBM},
        "trace_only_particles_per_s": N / (kern_ms * 1e-3),
        "stats": {k: (int(v) if isinstance(v, (int, np.integer)) else float(v)) for k, v in st.items()},
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, S, args.cpu_sample)
    print(json.dumps(out), flush=True)


def cpu_baseline(wl, S, sample):
    """The CPU oracle (unchanged, single-threaded) on a seeded sample of the
    same step's particles, with its own copy of the same inputs."""
    import torch
    from oracle import oracle as O
    from paper_2103_02388_amd import workloads as W

    om = O.Mesh.from_workload(wl)
    xc = om.dof_coords()
    xt = torch.from_numpy(np.ascontiguousarray(xc.T))
    u0 = np.ascontiguousarray(W.swirl_velocity(xt, 7 * wl.dt).numpy().T)
    u1 = np.ascontiguousarray(W.swirl_velocity(xt, 8 * wl.dt).numpy().T)
    c = W.two_blobs(xt).numpy()
    # full steps (every particle) repeated until about 10 s of single-core work
    n = sample or om.N
    ids = None if n >= om.N else np.sort(np.random.default_rng(0).choice(om.N, n, replace=False))
    reps, total = 0, 0.0
    while reps == 0 or (total < 10.0 and reps < 40):
        t0 = time.perf_counter()
        om.trace(u0, u1, c, wl.dt, S, ids=ids, threads=1)
        total += time.perf_counter() - t0
        reps += 1
    dt = total
    n_total = n * reps
    try:
        cpu = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        cpu = "unknown"
    return {"value": n_total / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": "%d x %d particles: full swirl3d step 7 -> 8 repeated, RK4 %d sub-steps, FP64, "
                      "single thread; host CPU: %s (%d logical cores)" % (reps, n, S, cpu, os.cpu_count() or 0),
            "seconds": dt}


if __name__ == "__main__":
    main()
