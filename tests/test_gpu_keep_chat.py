"""options.keep_chat: the trace writes chat into the library's next-step
scalar array too, and mmoc_use_last_chat makes it the scalar of the next
step.  A run chained that way equals, bit for bit, the same run that hands
every chat back through mmoc_set_scalar (every precision; two velocity
levels on the swirl cube, one stationary level on the blended shell); the
call is refused when nothing was written."""
import numpy as np
import pytest
import torch

from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

pytestmark = pytest.mark.gpu

PRECS = [mmoc.MMOC_FP64, mmoc.MMOC_FP32_MIXED, mmoc.MMOC_FP32_FIELDS]


def keep_options():
    opt = mmoc.mmoc_default_options()
    opt.keep_chat = 1
    return opt


@pytest.mark.parametrize("prec", PRECS)
def test_chained_scalar_equals_ingested_swirl(prec):
    wl = W.swirl3d(steps=8)
    a = mmoc.Tracer.from_workload(wl, level=4, precision=prec)
    b = mmoc.Tracer.from_workload(wl, level=4, precision=prec, options=keep_options())
    xt = a.dof_coords().t().contiguous()
    dt = wl.dt

    def vel(n):
        return wl.velocity(xt, n * dt).t().contiguous()

    ca = wl.scalar0(xt).contiguous()
    a.set_velocity(1, vel(0))
    b.set_velocity(1, vel(0))
    for n in range(1, 7):
        u = vel(n)
        a.swap_levels()
        a.set_fields(1, u, ca)
        b.swap_levels()
        if n == 1:
            b.set_fields(1, u, ca)
        else:
            b.set_velocity(1, u)
            b.use_last_chat()
        cha, Xa = a.trace_step(dt, 4)
        chb, Xb = b.trace_step(dt, 4)
        torch.cuda.synchronize()
        assert torch.equal(cha, chb), n
        assert torch.equal(Xa, Xb), n
        ca = cha.double()
    a.close()
    b.close()


@pytest.mark.parametrize("prec", PRECS)
def test_chained_scalar_equals_ingested_shell(prec):
    wl = W.shell3d(level=2)
    a = mmoc.Tracer.from_workload(wl, level=2, precision=prec)
    b = mmoc.Tracer.from_workload(wl, level=2, precision=prec, options=keep_options())
    xt = a.dof_coords().t().contiguous()
    u = wl.velocity(xt).t().contiguous()
    ca = wl.scalar0(xt).contiguous()
    for tr in (a, b):
        tr.set_stationary(True)
        tr.set_velocity(0, u)
    b.set_scalar(ca)
    for n in range(3):
        a.set_scalar(ca)
        if n > 0:
            b.use_last_chat()
        cha, Xa = a.trace_step(wl.dt, 4)
        chb, Xb = b.trace_step(wl.dt, 4)
        torch.cuda.synchronize()
        assert torch.equal(cha, chb), n
        assert torch.equal(Xa, Xb), n
        ca = cha.double()
    a.close()
    b.close()


def test_use_last_chat_is_refused_without_a_written_chat():
    wl = W.swirl3d()
    off = mmoc.Tracer.from_workload(wl, level=3)
    with pytest.raises(mmoc.MMOCError) as e:
        off.use_last_chat()  # keep_chat off
    assert e.value.status == -3
    off.close()
    on = mmoc.Tracer.from_workload(wl, level=3, options=keep_options())
    with pytest.raises(mmoc.MMOCError) as e:
        on.use_last_chat()  # no step yet
    assert e.value.status == -3
    xt = on.dof_coords().t().contiguous()
    on.set_stationary(True)
    on.set_velocity(0, W.swirl_velocity(xt, 0.3).t().contiguous())
    on.set_scalar(W.two_blobs(xt).contiguous())
    on.trace_step(wl.dt, 4, want_X=False)
    on.use_last_chat()
    with pytest.raises(mmoc.MMOCError) as e:
        on.use_last_chat()  # already used
    assert e.value.status == -3
    on.close()


@pytest.mark.parametrize("prec", [mmoc.MMOC_FP64, mmoc.MMOC_FP32_MIXED])
def test_chained_scalar_equals_ingested_surrogate(prec):
    """The surrogate step's finish pass writes chat for every particle, kept
    tiles and fallback tiles alike, so its chained scalar equals the
    ingested one too (seeded weights correcting a one-sub-step predictor,
    a tolerance that keeps some tiles and sends others back to RK4)."""
    import math
    wl = W.swirl3d(steps=8)
    a = mmoc.Tracer.from_workload(wl, level=4, precision=prec)
    b = mmoc.Tracer.from_workload(wl, level=4, precision=prec, options=keep_options())
    rng = np.random.default_rng(11)
    w = np.empty(mmoc.mmoc_mlp_nparams())
    off = 0
    for (o, i) in ((64, 4), (64, 64), (64, 64), (3, 64)):
        w[off:off + o * i] = rng.normal(size=o * i) * math.sqrt(2.0 / i)
        off += o * i
        w[off:off + o] = rng.normal(size=o) * 0.1
        off += o
    for tr in (a, b):
        tr.mlp_configure([0, 0, 0, 0], [1, 1, 1, 2.0 * W.SWIRL_T], 2.0)
        tr.mlp_set_predictor(1, 1e-4, 2.0 * W.SWIRL_T)
        mmoc.mmoc_mlp_set_weights(tr.ctx, w.astype(np.float32))
    xt = a.dof_coords().t().contiguous()
    dt = wl.dt

    def vel(n):
        return wl.velocity(xt, n * dt).t().contiguous()

    ca = wl.scalar0(xt).contiguous()
    a.set_velocity(1, vel(0))
    b.set_velocity(1, vel(0))
    kept = fell = 0
    for n in range(1, 5):
        u = vel(n)
        a.swap_levels()
        a.set_fields(1, u, ca)
        b.swap_levels()
        if n == 1:
            b.set_fields(1, u, ca)
        else:
            b.set_velocity(1, u)
            b.use_last_chat()
        a.reset_stats()
        cha, Xa = a.trace_step_surrogate(n * dt, dt, 4, 0.01, 2e-4, step=n)
        st = a.stats()
        chb, Xb = b.trace_step_surrogate(n * dt, dt, 4, 0.01, 2e-4, step=n)
        torch.cuda.synchronize()
        fell += st["n_fallback"]
        kept += a.N - st["n_fallback"] - st["n_checked"]
        assert torch.equal(cha, chb), n
        assert torch.equal(Xa, Xb), n
        ca = cha.double()
    print("particles kept on the network %d, traced by fallback %d" % (kept, fell))
    assert kept > 0 and fell > 0
    a.close()
    b.close()
