"""The flow-map surrogate on the GPU.

* forward pass and gradients of the bf16-matrix-core kernels against the CPU
  reference with the same bf16 rounding points, and against plain float64;
* training on the tracer's own departure points lowers the loss;
* the check / fallback policy: poisoned weights send every tile to the RK4
  fallback (the step then equals the plain tracer), an infinite tolerance
  keeps the network everywhere except at the checked particles;
* the gain of a trained surrogate over the tracer on the 3D swirl workload,
  with the true error of every particle measured against the CPU oracle.
"""
import math
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

from gpu_helpers import Pair, field_gpu, rel_c, rel_x

pytestmark = pytest.mark.gpu


def init_params(seed):
    rng = np.random.default_rng(seed)
    n = mmoc.mmoc_mlp_nparams()
    p = np.empty(n)
    off = 0
    for (o, i) in ((64, 4), (64, 64), (64, 64), (3, 64)):
        p[off:off + o * i] = rng.normal(size=o * i) * math.sqrt(2.0 / i)
        off += o * i
        p[off:off + o] = rng.normal(size=o) * 0.1
        off += o
    return p


def swirl_tracer(level=2, precision=mmoc.MMOC_FP64):
    wl = W.swirl3d()
    tr = mmoc.Tracer.from_workload(wl, level=level, precision=precision)
    tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, W.SWIRL_T], 2.0)
    return wl, tr


# Element-wise parity of the matrix-core network with the CPU reference that
# rounds to bf16 at the same points (W2, W3, a1, a2 forward; dz2, dz3 and
# the transposed operands backward).  The two differ in
#   * the fp32 arithmetic of the GPU (fp32 layer 1, fp32 accumulation in the
#     matrix cores, the GELU from the hardware exp2 and reciprocal, each
#     good to about 1 ulp): relative differences of order 1e-6 in every
#     pre-activation;
#   * bf16 rounding flips: a pre-activation that lies within that 1e-6 of a
#     bf16 rounding midpoint rounds to the other neighbour on one side.  A
#     flip moves one operand by one bf16 unit (2^-8 of it), which reaches
#     an output through one weight and one GELU slope (both below about 1):
#     about 2^-8 of one product term, a few 1e-3 of the output scale.
# Hence the bounds: every element within 4e-3 (|ref| + s), s the RMS of the
# reference outputs (one or two flips), and at least 95% of the elements
# within 1e-5 (|ref| + s) (no flip: fp32 agreement).  The gradients pass
# through twice as many rounding points (the backward operands) and sum
# over the samples of the batch, which averages the flips: every element
# within 5e-3 (|ref| + s_block), at least 90% within 1e-4.
def elementwise(got, ref, loose, tight, share, what):
    s = np.sqrt(np.mean(ref ** 2))
    rel = np.abs(got - ref) / (np.abs(ref) + s)
    print("%s: max %.2e, p99 %.2e, p50 %.2e, share within %.0e: %.4f"
          % (what, rel.max(), np.percentile(rel, 99), np.percentile(rel, 50), tight, (rel <= tight).mean()))
    assert rel.max() <= loose, what
    assert (rel <= tight).mean() >= share, what


def test_forward_matches_reference():
    wl, tr = swirl_tracer()
    for seed in (1, 5):
        p = init_params(seed)
        mmoc.mmoc_mlp_set_weights(tr.ctx, p.astype(np.float32))
        p32 = p.astype(np.float32).astype(np.float64)
        rng = np.random.default_rng(seed + 1)
        n = 4000
        x = rng.uniform(-1, 1, size=(n, 4))
        xin = torch.tensor(x, dtype=torch.float32, device="cuda")
        out = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        mmoc.mmoc_mlp_forward(tr.ctx, xin, out)
        torch.cuda.synchronize()
        y = out.cpu().numpy().astype(np.float64)
        x32 = xin.cpu().numpy().astype(np.float64)
        ref16 = O.mlp_forward(p32, x32, bf16=True)
        ref64 = O.mlp_forward(p32, x32, bf16=False)
        elementwise(y, ref16, 4e-3, 1e-5, 0.95, "forward vs bf16 reference (seed %d)" % seed)
        # and the bf16 rounding itself: against plain float64 only loosely
        e64 = np.abs(y - ref64).max() / np.abs(ref64).max()
        print("forward vs float64: max relative %.2e" % e64)
        assert e64 <= 3e-2


def test_gradients_match_reference():
    wl, tr = swirl_tracer()
    p = init_params(3)
    mmoc.mmoc_mlp_set_weights(tr.ctx, p.astype(np.float32))
    p32 = p.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(4)
    n = 256
    x = rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)
    t = (rng.normal(size=(n, 3)) * 0.5).astype(np.float32)
    g = torch.empty(mmoc.mmoc_mlp_nparams(), dtype=torch.float32, device="cuda")
    loss = mmoc.mmoc_mlp_loss_grad(tr.ctx, torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"), g)
    g = g.cpu().numpy().astype(np.float64)
    l16, g16 = O.mlp_loss_grad(p32, x.astype(np.float64), t.astype(np.float64), bf16=True)
    assert abs(loss - l16) <= 1e-3 * l16
    # element by element within each parameter block (W1, b1, ..., b4)
    blocks = [(0, 256), (256, 320), (320, 4416), (4416, 4480), (4480, 8576), (8576, 8640), (8640, 8832),
              (8832, 8835)]
    for a, b in blocks:
        elementwise(g[a:b], g16[a:b], 5e-3, 1e-4, 0.9 if b - a > 3 else 0.0, "gradient %d:%d" % (a, b))


def record_swirl(tr, wl, steps, dt=None):
    dt = dt or wl.dt
    x = tr.dof_coords()
    xt = x.t().contiguous()
    cap = steps * tr.N
    tr.set_scalar(W.two_blobs(xt).contiguous())
    for n in range(steps):
        tr.set_velocity(0, W.swirl_velocity(xt, n * dt).t().contiguous())
        tr.set_velocity(1, W.swirl_velocity(xt, (n + 1) * dt).t().contiguous())
        _, X = tr.trace_step(dt, 4)
        tr.mlp_record((n + 1) * dt, dt, X, cap)
    return x


def test_training_lowers_the_loss():
    wl, tr = swirl_tracer(level=3)
    record_swirl(tr, wl, 4)
    l1 = tr.mlp_train(65536, 1, batch=4096, lr=1e-3)
    l2 = tr.mlp_train(65536, 10, batch=4096, lr=1e-3)
    print("loss after 1 epoch %.3e, after 10 more %.3e" % (l1, l2))
    assert l2 < 0.5 * l1


def test_poisoned_weights_fall_back_everywhere():
    wl = W.swirl3d()
    for prec in (mmoc.MMOC_FP64, mmoc.MMOC_FP32_MIXED):
        p = Pair(wl, level=3, precision=prec)
        p.tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, W.SWIRL_T], 2.0)
        bad = init_params(7)
        bad[-3:] = 50.0  # output bias: departure points far off
        mmoc.mmoc_mlp_set_weights(p.tr.ctx, bad.astype(np.float32))
        t_n = 0.3
        p.set_fields(t_n, wl.dt, False)
        p.tr.reset_stats()
        ch_s, X_s = p.tr.trace_step_surrogate(t_n + wl.dt, wl.dt, 4, 0.01, 1e-4, step=3)
        st = p.tr.stats()
        ch, X = p.tr.trace_step(wl.dt, 4)
        torch.cuda.synchronize()
        assert st["n_checked"] + st["n_fallback"] == p.tr.N
        assert np.array_equal(X_s.cpu().numpy(), X.cpu().numpy())
        assert rel_c(ch_s.double().cpu().numpy(), ch.double().cpu().numpy()) <= (1e-14 if prec == 0 else 1e-6)


def test_infinite_tolerance_keeps_the_network():
    wl, tr = swirl_tracer(level=3)
    p = init_params(8)
    mmoc.mmoc_mlp_set_weights(tr.ctx, p.astype(np.float32))
    x = tr.dof_coords()
    xt = x.t().contiguous()
    tr.set_velocity(0, W.swirl_velocity(xt, 0.3).t().contiguous())
    tr.set_velocity(1, W.swirl_velocity(xt, 0.3 + wl.dt).t().contiguous())
    tr.set_scalar(W.two_blobs(xt).contiguous())
    tr.reset_stats()
    ch, X = tr.trace_step_surrogate(0.3 + wl.dt, wl.dt, 4, 0.05, float("inf"), step=1)
    st = tr.stats()
    Xn = tr.mlp_infer(0.3 + wl.dt, wl.dt)
    _, Xr = tr.trace_step(wl.dt, 4)
    torch.cuda.synchronize()
    X, Xn, Xr = X.cpu().numpy(), Xn.cpu().numpy(), Xr.cpu().numpy()
    assert st["n_fallback"] == 0 and 0 < st["n_checked"] < tr.N
    same_net = np.all(X == Xn, axis=0)
    same_rk = np.all(X == Xr, axis=0)
    assert np.all(same_net | same_rk)
    assert same_rk.sum() >= st["n_checked"]



def check_sample(N, step, fraction, tile=128):
    """The surrogate's check sample, from its definition: particle i is
    checked when the murmur3 finaliser of (i * 0x9E3779B1) ^ seed is below
    fraction 2^32 (every particle for fraction 1), seed the 32-bit fold of
    0x243F6A8885A308D3 ^ step * 0x9E3779B97F4A7C15; an aligned tile of
    `tile` particles with no such particle checks the one whose hash is
    smallest in its upper 25 bits (ties: lowest index)."""
    m64 = (1 << 64) - 1
    s64 = 0x243F6A8885A308D3 ^ ((step * 0x9E3779B97F4A7C15) & m64)
    seed = np.uint64((s64 ^ (s64 >> 32)) & 0xFFFFFFFF)
    i = np.arange(N, dtype=np.uint64)
    m32 = np.uint64(0xFFFFFFFF)
    x = ((i * np.uint64(0x9E3779B1)) & m32) ^ seed
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x85EBCA6B)) & m32
    x ^= x >> np.uint64(13)
    x = (x * np.uint64(0xC2B2AE35)) & m32
    x ^= x >> np.uint64(16)
    th = float(np.float32(fraction)) * 4294967296.0
    thresh = 0xFFFFFFFF if th >= 4294967295.0 else int(th)
    sel = np.ones(N, bool) if thresh == 0xFFFFFFFF else x < np.uint64(thresh)
    key = (x & np.uint64(0xFFFFFF80)) | (i % np.uint64(tile))
    for t0 in range(0, N, tile):
        if not sel[t0:t0 + tile].any():
            sel[t0 + int(np.argmin(key[t0:t0 + tile]))] = True
    return sel


@pytest.mark.parametrize("level,fraction", [(5, 0.0), (5, 0.01), (5, 0.3), (5, 1.0), (6, 0.01)])
def test_check_sample_is_the_hash_rule(level, fraction):
    """Bit-exact check sample on the swirl: level 5 (274,625 particles, one
    round of 1,024 per selection block, a ragged last block) and level 6
    (2,146,689 particles, eight rounds per block).  With an infinite
    tolerance no tile falls back, so a particle carries its RK4 departure
    point exactly when it was checked and the network's otherwise."""
    wl, tr = swirl_tracer(level=level)
    mmoc.mmoc_mlp_set_weights(tr.ctx, init_params(8).astype(np.float32))
    xt = tr.dof_coords().t().contiguous()
    tr.set_velocity(0, W.swirl_velocity(xt, 0.3).t().contiguous())
    tr.set_velocity(1, W.swirl_velocity(xt, 0.3 + wl.dt).t().contiguous())
    tr.set_scalar(W.two_blobs(xt).contiguous())
    N = tr.N
    want = check_sample(N, 17, fraction)
    tr.reset_stats()
    _, X = tr.trace_step_surrogate(0.3 + wl.dt, wl.dt, 4, fraction, float("inf"), step=17)
    st = tr.stats()
    Xn = tr.mlp_infer(0.3 + wl.dt, wl.dt)
    _, Xr = tr.trace_step(wl.dt, 4)
    torch.cuda.synchronize()
    X, Xn, Xr = X.cpu().numpy(), Xn.cpu().numpy(), Xr.cpu().numpy()
    rk = np.all(X == Xr, axis=0)
    net = np.all(X == Xn, axis=0)
    assert not np.any(rk & net)
    assert np.all(rk | net)
    print("fraction %g: %d checked of %d (%d tiles)" % (fraction, want.sum(), N, (N + 127) // 128))
    assert st["n_fallback"] == 0 and st["n_checked"] == want.sum()
    assert np.array_equal(rk, want)
    tr.close()

SWIRL_PERIOD = 2.0 * W.SWIRL_T   # g(t) = cos(pi t / T) repeats after 2T


def swirl_surrogate_run(train, run, prec=mmoc.MMOC_FP64, pred=1, scale=1e-4, tol=1e-4, n_check=4000,
                        epochs=30, samples=2_000_000, timing=False):
    """The swirl run with the surrogate: steps `train` (1-based
    step n covers [t_{n-1}, t_n]) traced by RK4 (4 sub-steps) and recorded,
    the network trained on `samples` pairs drawn from them, then steps `run`
    with the surrogate (1% check sample, tolerance tol).  The network learns
    the correction to the RK4 trace with `pred` sub-steps (0: the whole
    displacement), with the time input the phase t mod 2T.  For every run
    step: the fraction of particles traced by RK4 (check + fallback) and the
    true error of a seeded sample of n_check particles against the CPU
    oracle, which is given the same scalar c^n as the GPU (per-step parity
    from identical inputs)."""
    wl = W.swirl3d(steps=max(run) + 1)
    p = Pair(wl, precision=prec)
    tr = p.tr
    tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, SWIRL_PERIOD], 2.0)
    tr.mlp_set_predictor(pred, scale, SWIRL_PERIOD)
    xt = p.xg.t().contiguous()
    xc = torch.from_numpy(p.xc.T.copy())
    N, dt = tr.N, wl.dt

    def vel(n):
        return W.swirl_velocity(xt, n * dt).t().contiguous()

    cur = W.two_blobs(xt).contiguous()
    cap = len(train) * N
    for n in train:
        tr.set_velocity(0, vel(n - 1))
        tr.set_velocity(1, vel(n))
        tr.set_scalar(cur)
        ch, X = tr.trace_step(dt, 4)
        tr.mlp_record(n * dt, dt, X, cap)
        cur = ch.double()
    t0 = time.perf_counter()
    loss = tr.mlp_train(samples, epochs, batch=8192, lr=1e-3, seed=5)
    t_train = time.perf_counter() - t0
    ids = np.sort(np.random.default_rng(11).choice(N, n_check, replace=False))
    idt = torch.from_numpy(ids).cuda()
    owner = p.om.dof_owner()[0][ids]
    rows = []
    for n in run:
        tr.set_velocity(0, vel(n - 1))
        tr.set_velocity(1, vel(n))
        tr.set_scalar(cur)
        tr.reset_stats()
        ch, X = tr.trace_step_surrogate(n * dt, dt, 4, 0.01, tol, step=n)
        st = tr.stats()
        u0c = np.ascontiguousarray(W.swirl_velocity(xc, (n - 1) * dt).numpy().T)
        u1c = np.ascontiguousarray(W.swirl_velocity(xc, n * dt).numpy().T)
        ch_h = cur.cpu().numpy()
        chr_, Xr, _ = p.om.trace(u0c, u1c, ch_h, dt, 4, ids=ids, threads=8)
        Xs = X[:, idt].cpu().numpy()
        ex = np.abs(Xs - Xr).max(axis=0)
        # the scalar step at the surrogate's own departure points: c^n_h
        # evaluated there by the oracle (P2 interpolation, float64), its walk
        # starting in the particle's own macro as the GPU's does (a point that
        # a surrogate error puts just outside the cube is extrapolated from
        # the boundary element that walk reaches)
        cx, _, _ = p.om.eval(ch_h, np.ascontiguousarray(Xs.T), start=owner)
        ec = np.abs(ch[idt].double().cpu().numpy() - cx[:, 0])
        rows.append({"step": n, "rk4": (st["n_checked"] + st["n_fallback"]) / N, "err": float(ex.max()),
                     "above": float((ex > tol).mean()), "err_c": float(ec.max()),
                     "max_res": st["max_check_residual"]})
        cur = ch.double()
    out = {"loss": loss, "train_s": t_train, "rows": rows}
    if timing:
        def timeit(f, k=20):
            f()
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(k):
                f()
            torch.cuda.synchronize()
            return (time.perf_counter() - a) / k
        n = run[0]
        tr.set_velocity(0, vel(n - 1))
        tr.set_velocity(1, vel(n))
        out["t_surrogate"] = timeit(lambda: tr.trace_step_surrogate(n * dt, dt, 4, 0.01, tol, step=n))
        out["t_rk4"] = timeit(lambda: tr.trace_step(dt, 4))
        out["t_rk4_s1"] = timeit(lambda: tr.trace_step(dt, 1))
        out["t_rk4_s2"] = timeit(lambda: tr.trace_step(dt, 2))
        out["t_infer"] = timeit(lambda: tr.mlp_infer(n * dt, dt))
    tr.close()
    return out


def report(tag, out, tol):
    rows = out["rows"]
    kept = [r for r in rows if r["rk4"] < 0.5]
    print("%s: loss %.3e (train %.2fs), steps %d-%d: mean rk4 fraction %.3f, kept steps %d of %d, "
          "max sampled error %.2e (kept steps %.2e), max |chat - c^n(X)| %.2e"
          % (tag, out["loss"], out["train_s"], rows[0]["step"], rows[-1]["step"],
             np.mean([r["rk4"] for r in rows]), len(kept), len(rows), max(r["err"] for r in rows),
             max([r["err"] for r in kept] or [0.0]), max(r["err_c"] for r in rows)))
    for r in rows[:: max(1, len(rows) // 20)]:
        print("  step %3d: rk4 fraction %.3f, sampled error %.2e, share above tol %.4f, max check residual %.2e"
              % (r["step"], r["rk4"], r["err"], r["above"], r["max_res"]))
    if "t_surrogate" in out:
        print("  step times: surrogate %.1f us, rk4 S=4 %.1f us, S=2 %.1f us, S=1 %.1f us, inference %.1f us"
              % tuple(1e6 * out[k] for k in ("t_surrogate", "t_rk4", "t_rk4_s2", "t_rk4_s1", "t_infer")))
    return kept


def test_surrogate_swirl_trained_on_steps_1_to_10_run_11_to_110():
    """The swirl (level 5, 274,625 particles): steps 1-10 traced and recorded, then steps
    11-110 with the 1% check at tol 1e-4.  The network corrects the
    one-sub-step RK4 trace (whose own error against 4 sub-steps is up to
    1.4e-4 on this flow); its time input is the phase of the periodic
    velocity, so steps 41-50 and 81-90 repeat the training phases and the
    others lie outside them.

    The check is a sample (one particle in a hundred, at least one per tile
    of 128), so it bounds the error statistically: a tile is kept when its
    checked particles are within tol/2, and an unchecked particle of a kept
    tile can still exceed tol where the network is poor (outside the
    training phases).  Asserted:
      * steps in the training phases (41-50, 81-90) keep the network on
        nearly every tile and every sampled particle is within tol;
      * on every step the share of sampled particles above tol stays below
        1%, and no sampled particle is off by more than 2 tol;
      * chat is c^n_h at the surrogate's departure points, to 1e-12 (the
        oracle's P2 evaluation there)."""
    tol = 1e-4
    out = swirl_surrogate_run(range(1, 11), range(11, 111), tol=tol)
    report("swirl, train 1-10, run 11-110", out, tol)
    for r in out["rows"]:
        assert r["above"] < 0.01, r
        assert r["err"] <= 2 * tol, r
        assert r["err_c"] <= 1e-12, r
    in_phase = [r for r in out["rows"] if (r["step"] - 1) % 40 < 10 and r["step"] > 40]
    assert len(in_phase) == 20
    for r in in_phase:
        assert r["rk4"] < 0.05 and r["err"] <= tol, r
    assert out["loss"] < 1e-2


def test_surrogate_full_period_variant():
    """The full-period variant (labelled as such): steps 1-40, one period of
    the velocity, traced and recorded; then steps 41-140 with the surrogate.
    Every step keeps the network on nearly every tile and every sampled
    particle is within tol; the step time is reported beside the plain RK4
    steps with 4, 2 and 1 sub-steps (the method without the network)."""
    tol = 1e-4
    out = swirl_surrogate_run(range(1, 41), range(41, 141), tol=tol, timing=True)
    report("full-period variant (train 1-40)", out, tol)
    for r in out["rows"]:
        assert r["err"] <= tol, r
        assert r["rk4"] < 0.1, r
        assert r["err_c"] <= 1e-12, r
