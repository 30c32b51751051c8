"""The closed-form shell trace of test_oracle_shell_pin on the GPU path.

A velocity affine in the computational coordinates, u(y) = A Phi^-1(y) with
A antisymmetric (tangent to the spheres), is reproduced exactly by P2 on
every element of the right macro column, so the departure points equal a
mesh-free RK4 of dy/dt = -u(y), and the scalar c = xi_0 gives
chat = Phi^-1(X)_0.  Here the library traces every particle of the shell
at level 3 (2.7e6 particles; element cache on, the default), and a seeded
sample of 8000 DoFs off the inner and outer spheres is compared with the
mesh-free reference: float64 to 1e-12; the float32 paths to their own
bounds (float32-mixed locates and evaluates in float32: 1e-5; float32
fields round the nodal values to float32: 1e-6 relative)."""
import numpy as np
import pytest
import torch

from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

from test_oracle_shell_pin import A0, Columns, rk4_reference

pytestmark = pytest.mark.gpu
LEVEL = 3
_NODES = {}


def nodes(tr):
    """DoF positions, their computational coordinates and the column map
    (the same for every precision: computed once)"""
    if not _NODES:
        v, m = W.shell(4, 4)
        cols = Columns(v, m)
        x = tr.dof_coords().cpu().numpy().T.copy()
        _NODES.update(cols=cols, x=x, xi=cols.phi_inv(x))
    return _NODES["cols"], _NODES["x"], _NODES["xi"]


@pytest.mark.parametrize("prec,tol", [(mmoc.MMOC_FP64, 1e-12), (mmoc.MMOC_FP32_MIXED, 1e-5),
                                      (mmoc.MMOC_FP32_FIELDS, 1e-6)])
def test_gpu_shell_trace_with_velocity_affine_in_the_computational_coordinates(prec, tol):
    wl = W.shell3d(level=LEVEL)
    tr = mmoc.Tracer.from_workload(wl, precision=prec)
    cols, x, xi = nodes(tr)
    u_nodes = xi @ A0.T
    scale = 1.0 / np.abs(u_nodes).max()
    A = A0 * scale
    u_nodes = u_nodes * scale
    r = np.linalg.norm(x, axis=1)
    tr.set_stationary(True)
    tr.set_velocity(0, torch.from_numpy(np.ascontiguousarray(u_nodes.T)).cuda())
    tr.set_scalar(torch.from_numpy(np.ascontiguousarray(xi[:, 0])).cuda())
    tr.reset_stats()
    ch, X = tr.trace_step(wl.dt, 4)
    torch.cuda.synchronize()
    st = tr.stats()
    interior = np.nonzero((r > 0.55 + 1e-9) & (r < 1.0 - 1e-9))[0]
    ids = np.sort(np.random.default_rng(21).choice(interior, 8000, replace=False))
    idt = torch.from_numpy(ids).cuda()
    Xs = X[:, idt].cpu().numpy().T
    chs = ch[idt].double().cpu().numpy()
    tr.close()
    Xr = rk4_reference(cols, A, np.zeros(3), x[ids], wl.dt, 4)
    ex = np.abs(Xs - Xr).max()
    ec = np.abs(chs - cols.phi_inv(Xs)[:, 0]).max()
    print("precision %d: %d particles, walks %d, |X - X_ref| %.2e, |chat - xi0(X)| %.2e"
          % (prec, len(ids), st["n_multi_hop"], ex, ec))
    assert st["n_nan"] == 0
    assert ex <= tol
    assert ec <= tol
