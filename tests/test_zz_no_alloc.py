"""The allocation-free entry point mmoc_mass_inner_noalloc, through the
C-ABI: its result equals mmoc_mass_inner's on the same inputs (same kernels,
same summation order: bit for bit), on two calls in a row that share the
GPU's scratch array, the second with a smaller mesh; and a mesh beyond the
array's size is refused before anything is enqueued."""
import pytest
import torch

from paper_2103_02388_amd import mmoc
from paper_2103_02388_amd import workloads as W

pytestmark = pytest.mark.gpu


def fields(tr, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    a = torch.rand(tr.N, generator=g, dtype=torch.float64).cuda()
    b = torch.rand(tr.N, generator=g, dtype=torch.float64).cuda()
    s = torch.rand(tr.N, generator=g, dtype=torch.float64).cuda()
    return a, b, s


def test_noalloc_equals_mass_inner_on_two_calls():
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    results = []
    for k, (level, order) in enumerate(((6, 2), (3, 1))):   # 1,048 then 2 partial sums
        opt = mmoc.mmoc_default_options()
        opt.order = order
        tr = mmoc.Tracer.from_workload(W.swirl3d(), level=level, options=opt)
        a, b, s = fields(tr, 10 + k)
        mmoc.mmoc_mass_inner_noalloc(tr.ctx, a, s, b, None, out[k:k + 1])
        torch.cuda.synchronize()
        ref = tr.mass_inner(a, s, b, None)
        got = out[k].item()
        print("level %d P%d: noalloc %.17g, mass_inner %.17g" % (level, order, got, ref))
        assert got == ref
        # a = b = 1: the volume of the unit cube
        one = torch.ones(tr.N, dtype=torch.float64, device="cuda")
        mmoc.mmoc_mass_inner_noalloc(tr.ctx, one, None, one, None, out[k:k + 1])
        torch.cuda.synchronize()
        assert abs(out[k].item() - 1.0) <= 1e-13
        results.append(got)
        tr.close()
    assert results[0] != results[1]


def test_noalloc_refuses_large_and_blended_meshes():
    opt = mmoc.mmoc_default_options()
    opt.order = 1
    tr = mmoc.Tracer.from_workload(W.swirl3d(), level=8, options=opt)   # 66,306 partial sums
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    one = torch.ones(tr.N, dtype=torch.float64, device="cuda")
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_mass_inner_noalloc(tr.ctx, one, None, one, None, out)
    assert e.value.status == -1 and "allocation-free" in str(e.value)
    tr.close()
    ann = mmoc.Tracer.from_workload(W.annulus2d(level=2))
    one = torch.ones(ann.N, dtype=torch.float64, device="cuda")
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_mass_inner_noalloc(ann.ctx, one, None, one, None, out)
    assert e.value.status == -6
    ann.close()
