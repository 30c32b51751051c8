"""Checkpoint and resume: the state a run carries from step to step is the
scalar (the caller's array) and, for the surrogate, the network's weights.
Ten steps, the state written to a file and the context closed, a new
context reading it back and ten more steps give bitwise the result of
twenty steps in one context."""
import numpy as np
import pytest
import torch

from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

pytestmark = pytest.mark.gpu


def run_steps(tr, wl, c, first, last):
    """Steps first..last (step n covers [t_{n-1}, t_n]) from scalar c."""
    xt = tr.dof_coords().t().contiguous()
    dt = wl.dt
    tr.set_velocity(1, wl.velocity(xt, (first - 1) * dt).t().contiguous())
    X = None
    for n in range(first, last + 1):
        tr.swap_levels()
        tr.set_fields(1, wl.velocity(xt, n * dt).t().contiguous(), c)
        ch, X = tr.trace_step(dt, wl.substeps)
        c = ch.double() if ch.dtype != torch.float64 else ch.clone()
    return c, X


@pytest.mark.parametrize("prec", [mmoc.MMOC_FP64, mmoc.MMOC_FP32_MIXED, mmoc.MMOC_FP32_FIELDS])
def test_resume_is_bitwise(prec, tmp_path):
    wl = W.swirl3d(steps=20)
    tr = mmoc.Tracer.from_workload(wl, level=4, precision=prec)
    c0 = wl.scalar0(tr.dof_coords().t().contiguous()).contiguous()
    c20, X20 = run_steps(tr, wl, c0, 1, 20)
    c10, _ = run_steps(tr, wl, c0, 1, 10)
    tr.close()
    path = tmp_path / "state.npy"
    np.save(path, c10.cpu().numpy())
    del c10
    tr2 = mmoc.Tracer.from_workload(wl, level=4, precision=prec)
    c10r = torch.from_numpy(np.load(path)).cuda()
    c20r, X20r = run_steps(tr2, wl, c10r, 11, 20)
    tr2.close()
    assert torch.equal(c20r, c20)
    assert torch.equal(X20r, X20)


def test_surrogate_resume_is_bitwise(tmp_path):
    """A network's weights written out and read into a new context give the
    same surrogate step, bit for bit."""
    wl = W.swirl3d()
    period = 2.0 * W.SWIRL_T

    def tracer():
        tr = mmoc.Tracer.from_workload(wl, level=4)
        tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, period], 2.0)
        tr.mlp_set_predictor(1, 1e-4, period)
        return tr

    tr = tracer()
    xt = tr.dof_coords().t().contiguous()
    n, dt = 12, wl.dt
    u0 = W.swirl_velocity(xt, (n - 1) * dt).t().contiguous()
    u1 = W.swirl_velocity(xt, n * dt).t().contiguous()
    c = W.two_blobs(xt).contiguous()
    # a network trained briefly on the tracer's own departure points
    tr.set_velocity(0, u0)
    tr.set_velocity(1, u1)
    tr.set_scalar(c)
    _, X = tr.trace_step(dt, 4)
    tr.mlp_record(n * dt, dt, X, tr.N)
    tr.mlp_train(tr.N, 2, batch=4096, lr=1e-3, seed=3)
    ch, Xs = tr.trace_step_surrogate(n * dt, dt, 4, 0.01, 1e-4, step=n)
    np.save(tmp_path / "w.npy", mmoc.mmoc_mlp_get_weights(tr.ctx))
    tr.close()
    tr2 = tracer()
    mmoc.mmoc_mlp_set_weights(tr2.ctx, np.load(tmp_path / "w.npy"))
    tr2.set_velocity(0, u0)
    tr2.set_velocity(1, u1)
    tr2.set_scalar(c)
    ch2, Xs2 = tr2.trace_step_surrogate(n * dt, dt, 4, 0.01, 1e-4, step=n)
    tr2.close()
    assert torch.equal(ch2, ch)
    assert torch.equal(Xs2, Xs)
