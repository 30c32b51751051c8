"""The largest block arrays the 32-bit gather offsets allow.

The trace kernels address field records with a scalar base plus a 32-bit
unsigned byte offset per lane, and the library rejects meshes whose record
arrays would reach 4 GiB.  One Kuhn tetrahedron refined 9 times (the
deepest 3D level) has 180,007,425 lattice nodes in a single macro: its
(u_x, u_y) records span 2.9 GB (float64) and its (u_x, u_y, u_z) records
2.2 GB (float32).  Gathers of the last quarter of the nodes (float64) and of
the last 1.1 million (float32) use byte offsets above 2^31, where a signed
offset would wrap.

A seeded sample of particles plus the last 2,000 in DoF order (whose nodes
sit at the largest offsets) is traced by the oracle; the GPU traces every
particle.  The fields for the oracle are sampled at the oracle's own DoF
positions (evaluated on the GPU for speed: the generator is the same
function either way).  Tolerances as in the per-precision test files: FP64
1e-12 relative; float32 fields 1e-6 in X and 1e-6 * max(1, L) + 1e-6 in
chat, with L = 10 bounding the gradient of the two Gaussian blobs (sigma
0.1: the largest slope of one blob is e^(-1/2) / sigma = 6.1).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

from gpu_helpers import rel_c, rel_x

pytestmark = pytest.mark.gpu


def one_tet(level):
    v, m = W.cube6()
    return W.Workload("tet", 3, level, v, m[:1].copy(), 0, W.SWIRL_T / 320.0, 1, 1, False,
                      W.swirl_velocity, W.two_blobs, "one Kuhn tetrahedron of the unit cube")


def on_gpu(fn, x_rows, *args):
    """fn at positions [d, N] (any device) -> [d, N] / [N] on the GPU"""
    x = torch.as_tensor(x_rows).to("cuda").t().contiguous()
    v = fn(x, *args)
    return v.t().contiguous() if v.dim() == 2 else v.contiguous()


@pytest.mark.parametrize("prec", [mmoc.MMOC_FP64, mmoc.MMOC_FP32_FIELDS])
def test_offsets_past_2gib_single_tet_level9(prec):
    level = 9
    wl = one_tet(level)
    print("limits: one tet, level %d, precision %d" % (level, prec), flush=True)
    tr = mmoc.Tracer.from_workload(wl, precision=prec, level=level)
    N = tr.N
    assert N == 1025 * 1026 * 1027 // 6
    om = O.Mesh.from_workload(wl, level=level)
    assert om.N == N
    xg = tr.dof_coords()
    xc = om.dof_coords()
    assert float((xg - torch.from_numpy(xc).to("cuda")).abs().max()) < 1e-15
    t_n, dt, S = 0.3, wl.dt, 2
    tr.set_velocity(0, on_gpu(wl.velocity, xg, t_n))
    tr.set_velocity(1, on_gpu(wl.velocity, xg, t_n + dt))
    tr.set_scalar(on_gpu(wl.scalar0, xg))
    del xg
    ch, X = tr.trace_step(dt, S)
    torch.cuda.synchronize()
    st = tr.stats()
    assert st["n_particles"] == N and st["n_nan"] == 0
    rng = np.random.default_rng(9)
    ids = np.unique(np.concatenate([rng.choice(N, 2000, replace=False), np.arange(N - 2000, N)]))
    ch_s = ch[torch.from_numpy(ids).cuda()].double().cpu().numpy()
    X_s = X[:, torch.from_numpy(ids).cuda()].cpu().numpy()
    tr.close()
    del ch, X
    torch.cuda.empty_cache()
    u0 = on_gpu(wl.velocity, xc, t_n).cpu().numpy()
    u1 = on_gpu(wl.velocity, xc, t_n + dt).cpu().numpy()
    cc = on_gpu(wl.scalar0, xc).cpu().numpy()
    del xc
    torch.cuda.empty_cache()
    chr_, Xr, _ = om.trace(u0, u1, cc, dt, S, ids=ids, threads=8)
    ex, ec = rel_x(X_s, Xr), rel_c(ch_s, chr_)
    print("limits: N %d, sample %d, X %.2e, chat %.2e" % (N, ids.size, ex, ec), flush=True)
    if prec == mmoc.MMOC_FP64:
        assert ex <= 1e-12 and ec <= 1e-12
    else:
        assert ex <= 1e-6
        assert ec <= (1e-6 * 10.0 + 1e-6) / max(np.abs(chr_).max(), 1e-300)


@pytest.mark.parametrize("prec,level,ok", [(mmoc.MMOC_FP64, 9, False), (mmoc.MMOC_FP32_FIELDS, 9, False),
                                           (mmoc.MMOC_FP64, 8, True)])
def test_meshes_past_4gib_are_rejected_before_any_work(prec, level, ok):
    """The six-tetrahedron cube at level 9 has 1.08e9 block slots: 17 GB of
    float64 (u_x, u_y) records, 13 GB of float32 triples.  The upload is
    refused with MMOC_E_ARG before any table is built; level 8 (135 million
    slots, 2.2 GB) is accepted."""
    wl = W.swirl3d(level=level)
    print("limits: cube, level %d, precision %d" % (level, prec), flush=True)
    if ok:
        tr = mmoc.Tracer.from_workload(wl, precision=prec, level=level)
        assert tr.N == 513 ** 3
        tr.close()
        return
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.Tracer.from_workload(wl, precision=prec, level=level)
    assert e.value.status == -1 and "4 GiB" in str(e.value)  # MMOC_E_ARG
