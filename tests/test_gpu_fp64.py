"""FP64 tracer on the GPU vs the CPU oracle, element by element.

Tolerance: 1e-12 relative in departure points and interpolated values (the
relative measures are defined in gpu_helpers).  Sizes: the 2D rotation
(16641 particles) and 3D swirl (274625) workloads at full size, plus small
meshes for edge cases (ragged tails: neither count is a multiple of 256).
"""
import numpy as np
import pytest
import torch

from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

from gpu_helpers import Pair, field_cpu, field_gpu, rel_c, rel_x

pytestmark = pytest.mark.gpu
TOL = 1e-12


def check(pair, ch, X, chr_, Xr):
    ex, ec = rel_x(X, Xr), rel_c(ch, chr_)
    assert ex <= TOL, ex
    assert ec <= TOL, ec
    return ex, ec


def test_rotation2d_full_size():
    wl = W.rotation2d()
    p = Pair(wl)
    assert p.tr.N == 16641
    assert p.coord_err < 1e-15
    p.set_fields(0.0, wl.dt, True)
    p.tr.reset_stats()
    ch, X = p.gpu_step(wl.dt, wl.substeps)
    chr_, Xr, st = p.oracle_step(wl.dt, wl.substeps)
    check(p, ch, X, chr_, Xr)
    gs = p.tr.stats()
    assert gs["n_particles"] == p.tr.N
    assert gs["n_outside"] == st[0] > 0  # rotation leaves the square at the corners
    assert gs["n_nan"] == 0


@pytest.mark.parametrize("step,S", [(7, 4), (0, 1), (13, 2)])
def test_swirl3d_full_size(step, S):
    wl = W.swirl3d()
    p = Pair(wl)
    assert p.tr.N == 274625
    assert p.coord_err < 1e-15
    t_n = step * wl.dt
    p.set_fields(t_n, wl.dt, False)
    p.tr.reset_stats()
    ch, X = p.gpu_step(wl.dt, S)
    chr_, Xr, st = p.oracle_step(wl.dt, S, threads=8)
    check(p, ch, X, chr_, Xr)
    gs = p.tr.stats()
    assert gs["n_particles"] == p.tr.N and gs["n_nan"] == 0
    assert abs(gs["n_multi_hop"] - st[1]) <= 2 and abs(gs["n_outside"] - st[0]) <= 2


def test_large_displacement_many_hops_and_exits():
    """dt = T with 2 sub-steps: stage points cross several macros and leave the cube."""
    wl = W.swirl3d()
    p = Pair(wl, level=2)
    p.set_fields(0.1, 1.5, False)
    p.tr.reset_stats()
    ch, X = p.gpu_step(1.5, 2)
    chr_, Xr, st = p.oracle_step(1.5, 2)
    check(p, ch, X, chr_, Xr)
    gs = p.tr.stats()
    assert gs["n_multi_hop"] > 0 and st[1] > 0


def test_brute_force_location_gives_the_same_step():
    """max_hops = 0 sends every macro change to brute force; the result must not change."""
    wl = W.swirl3d()
    opt = mmoc.mmoc_default_options()
    opt.max_hops = 0
    p = Pair(wl, level=3, options=opt)
    p.set_fields(0.3, wl.dt, False)
    p.tr.reset_stats()
    ch, X = p.gpu_step(wl.dt, 4)
    chr_, Xr, st = p.oracle_step(wl.dt, 4, max_hops=0)
    check(p, ch, X, chr_, Xr)
    chr2, Xr2, _ = p.oracle_step(wl.dt, 4)
    assert rel_x(Xr, Xr2) <= TOL and rel_c(chr_, chr2) <= TOL
    assert p.tr.stats()["n_bruteforce"] > 0


def test_small_meshes_every_level():
    for level in (0, 1, 2, 3):
        for wl in (W.rotation2d(), W.swirl3d()):
            p = Pair(wl, level=level)
            assert p.coord_err < 1e-15
            p.set_fields(0.2, wl.dt * 3, wl.stationary)
            ch, X = p.gpu_step(wl.dt * 3, 3)
            chr_, Xr, _ = p.oracle_step(wl.dt * 3, 3)
            check(p, ch, X, chr_, Xr)


def test_stationary_equals_two_identical_levels():
    wl = W.swirl3d()
    p = Pair(wl, level=3)
    p.set_fields(0.4, wl.dt, True)
    ch1, X1 = p.gpu_step(wl.dt, 4)
    p.tr.set_stationary(False)  # new record layout: every field is set again
    with pytest.raises(mmoc.MMOCError):
        p.tr.trace_step(wl.dt, 4)
    p.tr.set_velocity(0, p.u0g)
    p.tr.set_velocity(1, p.u0g)
    p.tr.set_scalar(p.cg)
    ch2, X2 = p.gpu_step(wl.dt, 4)
    assert rel_x(X1, X2) <= 1e-15 and rel_c(ch1, ch2) <= 1e-15


@pytest.mark.parametrize("precision", [mmoc.MMOC_FP64, mmoc.MMOC_FP32_MIXED])
def test_level_swap_equals_fresh_upload(precision):
    """After a swap the old level 1 acts as level 0: the same step, to the
    last bits (the time weights meet the two sums in the other order), as a
    context whose level 0 was uploaded directly."""
    wl = W.swirl3d()
    a = Pair(wl, level=3, precision=precision)
    b = Pair(wl, level=3, precision=precision)
    t0 = 0.45
    a.set_fields(t0 - wl.dt, wl.dt, False)
    a.gpu_step(wl.dt, 4)
    a.tr.swap_levels()
    u2 = field_gpu(wl.velocity, a.xg, t0 + wl.dt)
    a.tr.set_velocity(1, u2)
    b.set_fields(t0, wl.dt, False)
    A = a.gpu_step(wl.dt, 4)
    B = b.gpu_step(wl.dt, 4)
    tol = 1e-14 if precision == mmoc.MMOC_FP64 else 1e-6
    assert rel_x(A[1], B[1]) <= tol and rel_c(A[0], B[0]) <= tol


def test_multi_step_chain_with_level_swap():
    """Five consecutive steps (levels swapped, chat fed back as the next scalar)
    against the oracle's own chain; the two chains drift only by rounding."""
    wl = W.swirl3d()
    p = Pair(wl, level=3)
    dt, S = wl.dt, 4
    p.set_fields(0.0, dt, False)
    cg, cc = p.cg, p.cc
    u0c = p.u0c
    for n in range(5):
        t_n = n * dt
        if n > 0:
            p.tr.swap_levels()
            u1g = field_gpu(wl.velocity, p.xg, t_n + dt)
            p.tr.set_velocity(1, u1g)
            p.tr.set_scalar(cg)
        u1c = field_cpu(wl.velocity, p.xc, t_n + dt)
        chg, Xg = p.tr.trace_step(dt, S)
        torch.cuda.synchronize()
        chc, Xc, _ = p.om.trace(u0c, u1c, cc, dt, S)
        assert rel_x(Xg.cpu().numpy(), Xc) <= TOL
        assert rel_c(chg.cpu().numpy(), chc) <= 1e-11
        cg, cc, u0c = chg.contiguous(), chc, u1c


def test_shell_blended_fp64():
    wl = W.shell3d(level=1)
    p = Pair(wl, level=1)
    assert p.coord_err < 1e-14
    p.set_fields(0.0, wl.dt, True)
    p.tr.reset_stats()
    ch, X = p.gpu_step(wl.dt, 4)
    chr_, Xr, st = p.oracle_step(wl.dt, 4)
    check(p, ch, X, chr_, Xr)
    assert p.tr.stats()["n_nan"] == 0


def test_shell3d_full_size_sampled_fp64():
    """The headline workload in the launch configuration the benchmark times:
    the spherical shell at full size (3840 macros at level 5, 168,428,034
    particles), stationary seeded flow, float64 with the element cache on
    (the default options), RK4 with 4 sub-steps.  The analytic fields are
    evaluated once at the oracle's DoF positions and the same arrays go to
    both sides; the library's own DoF positions are compared on the sample.
    The oracle traces a seeded sample of 3000 particles.

    X to 1e-12 relative.  chat: the scalar is a step at r = 0.8 plus 1%
    nodal noise, so its P2 interpolant has slopes up to about
    L = 6 / (h/2) (a jump of 1 across half a radial micro edge h, P2
    shape-function gradients at most 3 / height, a factor 2 for the element
    shape); a last-bit difference in X moves chat by up to L times it, so
    chat is held to 1e-12 * L + 1e-14 on the sample, and to 1e-12 (relative)
    away from the step (departure radius more than 0.02 from 0.8).  A smooth
    scalar is traced as well, held to 1e-12 relative everywhere."""
    from oracle import oracle as O
    wl = W.shell3d()
    tr = mmoc.Tracer.from_workload(wl, precision=mmoc.MMOC_FP64, options=mmoc.mmoc_default_options())
    om = O.Mesh.from_workload(wl)
    N = om.N
    assert tr.N == N == 168_428_034
    ids = np.sort(np.random.default_rng(15).choice(N, 3000, replace=False))
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
    assert st["n_cache_lookups"] > 0 and st["n_cache_hits"] > 0.5 * st["n_cache_lookups"]
    Xs, chs = X[:, idt].cpu().numpy(), ch[idt].cpu().numpy()
    tr.set_scalar(smooth)
    ch2, _ = tr.trace_step(wl.dt, 4, want_X=False)
    ch2s = ch2[idt].cpu().numpy()
    uc, cc, sc = u.cpu().numpy(), c.cpu().numpy(), smooth.cpu().numpy()
    del u, c, smooth, X, ch, ch2
    tr.close()
    chr_, Xr, _ = om.trace(uc, None, cc, wl.dt, 4, ids=ids, threads=8)
    ch2r, _, _ = om.trace(uc, None, sc, wl.dt, 4, ids=ids, threads=8)
    ex = rel_x(Xs, Xr)
    assert ex <= TOL, ex
    L = 6.0 / (wl.extra["h_min"] / 2)
    ec_all = np.abs(chs - chr_).max()
    assert ec_all <= TOL * L + 1e-14, ec_all
    far = np.abs(np.linalg.norm(Xr, axis=0) - 0.8) > 0.02
    ec = rel_c(chs[far], chr_[far])
    assert ec <= TOL, ec
    es = rel_c(ch2s, ch2r)
    assert es <= TOL, es
    print("fp64 shell %d particles: X %.2e, chat %.2e (all %.2e, bound %.1e), smooth chat %.2e, cache hits %.3f"
          % (N, ex, ec, ec_all, TOL * L + 1e-14, es, st["n_cache_hits"] / st["n_cache_lookups"]))


def test_nan_velocity_is_counted_and_contained():
    wl = W.swirl3d()
    p = Pair(wl, level=2)
    p.set_fields(0.3, wl.dt, False)
    u = p.u0g.clone()
    u[0, p.tr.N // 2] = float("nan")
    p.tr.set_velocity(0, u)
    p.tr.reset_stats()
    ch, X = p.gpu_step(wl.dt, 4)
    st = p.tr.stats()
    nbad = int(np.isnan(X).any(axis=0).sum())
    assert 0 < nbad < p.tr.N // 4
    assert st["n_nan"] == nbad


def test_two_runs_are_bitwise_identical():
    wl = W.swirl3d()
    p = Pair(wl, level=4)
    p.set_fields(0.5, wl.dt, False)
    a = p.gpu_step(wl.dt, 4)
    b = p.gpu_step(wl.dt, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_plume3d_full_size_sampled():
    """1.7e7 particles on the GPU; the oracle traces a seeded sample of 3000."""
    wl = W.plume3d()
    p = Pair(wl)
    assert p.tr.N == 257 ** 3
    assert p.coord_err < 1e-15
    step = 60
    p.set_fields(step * wl.dt, wl.dt, False)
    ch, X = p.gpu_step(wl.dt, 4)
    ids = np.sort(np.random.default_rng(12).choice(p.tr.N, 3000, replace=False))
    chr_, Xr, _ = p.oracle_step(wl.dt, 4, ids=ids, threads=8)
    ex, ec = rel_x(X[:, ids], Xr), rel_c(ch[ids], chr_)
    assert ex <= TOL and ec <= TOL


@pytest.mark.parametrize("prec", [mmoc.MMOC_FP64, mmoc.MMOC_FP32_FIELDS])
def test_set_fields_equals_separate_calls(prec):
    """mmoc_set_fields (velocity level and scalar in one pass) gives the
    same step, bit for bit, as mmoc_set_velocity + mmoc_set_scalar."""
    wl = W.swirl3d()
    out = []
    for combined in (False, True):
        p = Pair(wl, level=3, precision=prec)
        u0 = field_gpu(wl.velocity, p.xg, 0.4)
        u1 = field_gpu(wl.velocity, p.xg, 0.4 + wl.dt)
        c = field_gpu(wl.scalar0, p.xg)
        p.tr.set_velocity(0, u0)
        if combined:
            p.tr.set_fields(1, u1, c)
        else:
            p.tr.set_velocity(1, u1)
            p.tr.set_scalar(c)
        out.append(p.gpu_step(wl.dt, 4))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    with pytest.raises(mmoc.MMOCError) as e:
        p.tr.set_fields(2, u1, c)
    assert e.value.status == -1


@pytest.mark.parametrize("swap", [False, True])
def test_paired_uz_records_equal_unpaired(swap):
    """A two-level float64 3D context pairs the two levels' u_z per slot (one
    load brings both); a three-level context keeps one u_z array per level.
    The same step through both must agree bit for bit, with the earlier level
    in either ring slot (swap: after a level swap it sits in ring slot 1)."""
    wl = W.swirl3d()
    res = []
    for levels in (2, 3):
        tr = mmoc.Tracer.from_workload(wl, level=3)
        if levels == 3:
            tr.set_level_count(3)
        xt = tr.dof_coords().t().contiguous()
        u0 = wl.velocity(xt, 0.4).t().contiguous()
        u1 = wl.velocity(xt, 0.4 + wl.dt).t().contiguous()
        if swap:
            tr.set_velocity(1, u0)
            tr.swap_levels()  # the ring turns: logical level 0 now sits in ring slot 1
            tr.set_velocity(1, u1)
        else:
            tr.set_velocity(0, u0)
            tr.set_velocity(1, u1)
        tr.set_scalar(wl.scalar0(xt).contiguous())
        ch, X = tr.trace_span(0, 1, wl.dt, 4) if levels == 3 else tr.trace_step(wl.dt, 4)
        tau, umax, _ = mmoc.mmoc_cfl_time_step(tr.ctx, 1.0, 1)
        torch.cuda.synchronize()
        res.append((ch.cpu().numpy(), X.cpu().numpy(), umax))
        tr.close()
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][2] == res[1][2]
