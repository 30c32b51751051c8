"""Shared helpers of the GPU tests: build both sides' inputs from the same
workload generator and compare results with the relative measures

  X:    max_i |X_i - X_i^ref|_inf / max(1, max_i |X_i^ref|_inf)
  chat: max_i |chat_i - chat_i^ref| / max_i |chat_i^ref|

Each side samples the analytic fields at its own DoF positions (the library's
``mmoc_dof_coords``, the oracle's ``dof_coords``); the positions themselves
are compared first, so that both sides see the same input to rounding.
"""
import numpy as np
import torch

from oracle import oracle as O
from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W


def rel_x(X, Xr):
    return float(np.abs(X - Xr).max() / max(1.0, np.abs(Xr).max()))


def rel_c(c, cr):
    return float(np.abs(c - cr).max() / max(np.abs(cr).max(), 1e-300))


def field_gpu(fn, xg, *args):
    """fn(x [N,d] tensor, ...) on GPU coordinates [d,N] -> SoA [d,N] (or [N])"""
    v = fn(xg.t().contiguous(), *args)
    return v.t().contiguous() if v.dim() == 2 else v.contiguous()


def field_cpu(fn, xc, *args):
    v = fn(torch.from_numpy(np.ascontiguousarray(xc.T)), *args)
    return np.ascontiguousarray(v.numpy().T) if v.dim() == 2 else v.numpy()


class Pair:
    """A workload set up on both sides."""

    def __init__(self, wl, level=None, precision=mmoc.MMOC_FP64, options=None, order=None):
        self.wl = wl
        self.level = wl.level if level is None else level
        self.tr = mmoc.Tracer.from_workload(wl, precision=precision, level=self.level, options=options, order=order)
        self.om = O.Mesh.from_workload(wl, level=self.level, order=order or 2)
        assert self.tr.N == self.om.N
        self.xg = self.tr.dof_coords()
        torch.cuda.synchronize()
        self.xc = self.om.dof_coords()
        self.coord_err = float(np.abs(self.xg.cpu().numpy() - self.xc).max())

    def set_fields(self, t_n, dt, stationary, scalar_fn=None, vel_fn=None):
        wl = self.wl
        vel = vel_fn or wl.velocity
        sc = scalar_fn or wl.scalar0
        self.u0g = field_gpu(vel, self.xg, t_n)
        self.u0c = field_cpu(vel, self.xc, t_n)
        if stationary:
            self.u1g, self.u1c = None, None
        else:
            self.u1g = field_gpu(vel, self.xg, t_n + dt)
            self.u1c = field_cpu(vel, self.xc, t_n + dt)
        self.cg = field_gpu(sc, self.xg)
        self.cc = field_cpu(sc, self.xc)
        self.tr.set_stationary(stationary)
        self.tr.set_velocity(0, self.u0g)
        if not stationary:
            self.tr.set_velocity(1, self.u1g)
        self.tr.set_scalar(self.cg)

    def gpu_step(self, dt, S):
        ch, X = self.tr.trace_step(dt, S)
        torch.cuda.synchronize()
        return ch.double().cpu().numpy(), X.cpu().numpy()

    def oracle_step(self, dt, S, ids=None, threads=1, max_hops=64):
        return self.om.trace(self.u0c, self.u1c, self.cc, dt, S, ids=ids, threads=threads, max_hops=max_hops)
