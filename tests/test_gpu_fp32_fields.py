"""Float32 field records with float64 arithmetic (MMOC_FP32_FIELDS) on the
GPU vs the float64 CPU oracle.

On this GPU a float32 vector operation is no faster than a float64 one (the
packed float32 forms are not used), so the only thing float32 buys is memory:
half the bytes per gathered node.  This path stores the velocity levels and
the scalar as float32 and does every operation in float64.  Its only error
against the float64 oracle is the rounding of the stored nodal values
(relative 2^-24): a departure point moves by at most dt * 2^-24 * max|u|
times the flow's growth factor over one step, and chat by the scalar's
rounding plus its gradient times that displacement.  The bounds below, X
within 1e-6 relative and chat within 1e-6 * max(1, L) + 1e-6 (L the
scalar's Lipschitz constant estimated from nodal differences), leave two
orders of magnitude of margin over that estimate on these workloads."""
import numpy as np
import pytest
import torch

from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

from gpu_helpers import Pair, rel_c, rel_x
from test_gpu_fp32 import lipschitz

pytestmark = pytest.mark.gpu
TOL_X = 1e-6
PREC = mmoc.MMOC_FP32_FIELDS


def check(ch, X, chr_, Xr, L):
    ex, ec = rel_x(X, Xr), rel_c(ch, chr_)
    assert ex <= TOL_X, ex
    assert ec <= (TOL_X * max(1.0, L) + 1e-6) / max(np.abs(chr_).max(), 1e-300), (ec, L)
    return ex, ec


@pytest.mark.parametrize("step,S", [(7, 4), (0, 1)])
def test_swirl3d_full_size_fp32_fields(step, S):
    wl = W.swirl3d()
    p = Pair(wl, precision=PREC)
    p.set_fields(step * wl.dt, wl.dt, False)
    p.tr.reset_stats()
    ch, X = p.gpu_step(wl.dt, S)
    chr_, Xr, _ = p.oracle_step(wl.dt, S, threads=8)
    ex, ec = check(ch, X, chr_, Xr, lipschitz(p))
    st = p.tr.stats()
    assert st["n_particles"] == p.tr.N and st["n_nan"] == 0 and st["n_tieband"] == 0
    print("fp32 fields swirl step %d S=%d: X %.2e chat %.2e" % (step, S, ex, ec))


def test_rotation2d_and_small_meshes_fp32_fields():
    wl = W.rotation2d()
    p = Pair(wl, precision=PREC)
    p.set_fields(0.0, wl.dt, True)
    ch, X = p.gpu_step(wl.dt, wl.substeps)
    chr_, Xr, _ = p.oracle_step(wl.dt, wl.substeps)
    check(ch, X, chr_, Xr, lipschitz(p))
    for level in (0, 1, 2):
        for wl in (W.rotation2d(), W.swirl3d()):
            p = Pair(wl, level=level, precision=PREC)
            p.set_fields(0.2, wl.dt * 3, wl.stationary)
            ch, X = p.gpu_step(wl.dt * 3, 3)
            chr_, Xr, _ = p.oracle_step(wl.dt * 3, 3)
            check(ch, X, chr_, Xr, lipschitz(p))


def test_shell_fp32_fields():
    wl = W.shell3d(level=1)
    p = Pair(wl, level=1, precision=PREC)
    p.set_fields(0.0, wl.dt, True)
    ch, X = p.gpu_step(wl.dt, 4)
    chr_, Xr, _ = p.oracle_step(wl.dt, 4)
    assert rel_x(X, Xr) <= TOL_X
    r = np.linalg.norm(Xr, axis=0)
    far = np.abs(r - 0.8) > 0.45 / 4 / 2
    assert np.abs(ch[far] - chr_[far]).max() <= 1e-5


def test_fp32_fields_against_fp64_gpu():
    """Same inputs on the two GPU paths: the departure points differ only by
    the field rounding."""
    wl = W.swirl3d()
    a = Pair(wl, level=4)
    b = Pair(wl, level=4, precision=PREC)
    a.set_fields(0.45, wl.dt, False)
    b.set_fields(0.45, wl.dt, False)
    cha, Xa = a.gpu_step(wl.dt, 4)
    chb, Xb = b.gpu_step(wl.dt, 4)
    assert rel_x(Xb, Xa) <= TOL_X
    assert np.abs(chb - cha).max() <= 1e-5


def test_plume3d_full_size_sampled_fp32_fields():
    wl = W.plume3d()
    p = Pair(wl, precision=PREC)
    p.set_fields(120 * wl.dt, wl.dt, False)
    ch, X = p.gpu_step(wl.dt, 4)
    ids = np.sort(np.random.default_rng(15).choice(p.tr.N, 3000, replace=False))
    chr_, Xr, _ = p.oracle_step(wl.dt, 4, ids=ids, threads=8)
    assert rel_x(X[:, ids], Xr) <= TOL_X
    assert np.abs(ch[ids] - chr_).max() <= TOL_X * 10.0 + 1e-6


def test_shell3d_full_size_sampled_fp32_fields():
    """The spherical shell at full size (168,428,034 particles) in the
    benchmark's launch configuration for this path (element cache on),
    against the float64 oracle on a seeded sample of 3000 particles; the same
    float64 field arrays go to both sides (the library rounds them to its
    float32 records).  X within 1e-6 relative.  chat away from the step at
    r = 0.8 (departure radius more than 0.02 from it) within
    1e-6 * max(1, L) + 1e-6, with L = 0.02 * 6 / (h/2) bounding the slope the
    1% nodal noise gives the P2 interpolant (as for the float32-mixed
    tracer); a smooth scalar (|grad| <= 3) within 1e-6 * 3 + 1e-6."""
    from oracle import oracle as O
    wl = W.shell3d()
    tr = mmoc.Tracer.from_workload(wl, precision=PREC, options=mmoc.mmoc_default_options())
    om = O.Mesh.from_workload(wl)
    N = om.N
    assert tr.N == N == 168_428_034
    ids = np.sort(np.random.default_rng(16).choice(N, 3000, replace=False))
    xc = om.dof_coords()
    idt = torch.from_numpy(ids).cuda()
    xg = tr.dof_coords()
    assert np.abs(xg[:, idt].cpu().numpy() - xc[:, ids]).max() < 1e-14
    del xg
    xt = torch.from_numpy(np.ascontiguousarray(xc.T)).cuda()
    u = wl.velocity(xt).t().contiguous()
    c = wl.scalar0(xt).contiguous()
    smooth = (xt[:, 0] ** 2 + xt[:, 1] * xt[:, 2]).contiguous()
    del xt
    tr.set_stationary(True)
    tr.set_velocity(0, u)
    tr.set_scalar(c)
    tr.reset_stats()
    ch, X = tr.trace_step(wl.dt, 4)
    torch.cuda.synchronize()
    st = tr.stats()
    assert st["n_nan"] == 0 and st["n_particles"] == N
    Xs, chs = X[:, idt].cpu().numpy(), ch[idt].double().cpu().numpy()
    tr.set_scalar(smooth)
    ch2, _ = tr.trace_step(wl.dt, 4, want_X=False)
    ch2s = ch2[idt].double().cpu().numpy()
    uc, cc, sc = u.cpu().numpy(), c.cpu().numpy(), smooth.cpu().numpy()
    del u, c, smooth, X, ch, ch2
    tr.close()
    chr_, Xr, _ = om.trace(uc, None, cc, wl.dt, 4, ids=ids, threads=8)
    ch2r, _, _ = om.trace(uc, None, sc, wl.dt, 4, ids=ids, threads=8)
    ex = rel_x(Xs, Xr)
    assert ex <= TOL_X, ex
    L = 0.02 * 6 / (wl.extra["h_min"] / 2)
    far = np.abs(np.linalg.norm(Xr, axis=0) - 0.8) > 0.02
    ec = np.abs(chs[far] - chr_[far]).max()
    assert ec <= TOL_X * max(1.0, L) + 1e-6, (ec, L)
    es = np.abs(ch2s - ch2r).max()
    assert es <= TOL_X * 3 + 1e-6, es
    print("fp32-fields shell %d particles: X %.2e, chat %.2e (bound %.1e), smooth chat %.2e"
          % (N, ex, ec, TOL_X * max(1.0, L) + 1e-6, es))
