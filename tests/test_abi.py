"""The C-ABI: every symbol declared in include/mmoc.h is exported (CPU), and
argument, state and mesh errors come back as the documented codes before any
device work is enqueued (GPU)."""
import os
import re

import numpy as np
import pytest

from paper_2103_02388_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "mmoc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mmoc_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2103_02388_amd import mmoc
    L = mmoc.lib()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(mmoc.EXPORTED)


def test_default_options_and_param_count():
    from paper_2103_02388_amd import mmoc
    o = mmoc.mmoc_default_options()
    assert o.eps_in == 1e-12 and o.max_hops == 64
    assert o.elem_cache == 1 and o.keep_chat == 0
    # float32-mixed: float64 tie-break within a band of both macro and micro faces
    assert o.eps32_macro == pytest.approx(4e-6, rel=1e-6) and o.eps32_micro == 2.0 ** -18
    assert mmoc.mmoc_mlp_nparams() == 4 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 3 + 3


@pytest.mark.gpu
def test_argument_and_state_errors():
    import torch
    from paper_2103_02388_amd import mmoc
    wl = W.swirl3d(level=4)
    tr = mmoc.Tracer.from_workload(wl)
    N = tr.N
    assert 8 * N > 4 * 65536
    dev = tr.device
    c = torch.zeros(N, dtype=torch.float64, device=dev)
    X = torch.zeros((3, N), dtype=torch.float64, device=dev)
    # trace before fields are set
    with pytest.raises(mmoc.MMOCError) as e:
        tr.trace_step(0.1, 4, c, X)
    assert e.value.status == -3
    u = torch.zeros((3, N), dtype=torch.float64, device=dev)
    tr.set_stationary(True)
    tr.set_velocity(0, u)
    with pytest.raises(mmoc.MMOCError) as e:
        tr.trace_step(0.1, 4, c, X)  # scalar missing
    assert e.value.status == -3
    tr.set_scalar(c)
    tr.trace_step(0.1, 4, c, X)
    for bad in ((0.0, 4), (-1.0, 4), (float("nan"), 4), (0.1, 0)):
        with pytest.raises(mmoc.MMOCError) as e:
            tr.trace_step(bad[0], bad[1], c, X)
        assert e.value.status == -1
    # host memory, too-small buffers, misaligned pointers
    host = torch.zeros(N, dtype=torch.float64)
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_trace_step(tr.ctx, 0.1, 4, host, X)
    assert e.value.status == -1
    # a buffer that ends before the data would: the library sees the end of a
    # device allocation (not the sub-allocations of torch's caching allocator),
    # so the test makes its own allocation of exactly 8 N bytes and passes a
    # pointer 64 KiB into it
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    raw_p = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(raw_p), ctypes.c_size_t(8 * N)) == 0
    try:
        late = ctypes.c_void_p(raw_p.value + 65536)
        st = mmoc.lib().mmoc_trace_step(tr.ctx, 0.1, 4, late, ctypes.c_void_p(X.data_ptr()))
        assert st == -1, st
        st = mmoc.lib().mmoc_set_scalar(tr.ctx, late)
        assert st == -1, st
        st = mmoc.lib().mmoc_set_scalar(tr.ctx, raw_p)
        assert st == 0, st
    finally:
        hip.hipDeviceSynchronize()
        hip.hipFree(raw_p)
    raw = torch.zeros(8 * N + 16, dtype=torch.uint8, device=dev)
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_set_scalar(tr.ctx, raw[1:])
    assert e.value.status == -1
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_set_velocity(tr.ctx, 2, u)
    assert e.value.status == -1
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_swap_velocity_levels(tr.ctx)  # level 1 never set
    assert e.value.status == -3
    tr.close()


@pytest.mark.gpu
def test_mesh_errors():
    from paper_2103_02388_amd import mmoc
    v, m = W.cube6()
    # degenerate macro (repeated coordinates)
    v2 = v.copy()
    v2[7] = v2[3]
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.Tracer(3, 1, v2, m)
    assert e.value.status == -2
    # non-conforming vertex order on a shared face
    m2 = m.copy()
    m2[0] = m2[0][[3, 1, 2, 0]]
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.Tracer(3, 1, v, m2)
    assert e.value.status == -2
    # vertex id out of range
    m3 = m.copy()
    m3[1, 2] = 99
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.Tracer(3, 1, v, m3)
    assert e.value.status == -2
    # radial blending needs vertices away from the origin, each macro spanning
    # exactly d radial directions: the unit square has a vertex at the origin
    vs, ms = W.square2()
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.Tracer(2, 1, vs, ms, blend=1)
    assert e.value.status == -2
    # P1 elements are not built for blended meshes
    va, ma = W.annulus()
    opt = mmoc.mmoc_default_options()
    opt.order = 1
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.Tracer(2, 1, va, ma, blend=1, options=opt)
    assert e.value.status == -6


@pytest.mark.gpu
def test_failed_level_ring_leaves_no_levels():
    """A velocity ring that cannot be allocated (65536 levels of a level-6
    cube: about 2.3 TB) fails with MMOC_E_NOMEM and leaves the context with
    no levels: traces and level uploads are refused until the level count is
    set again, after which the context works as before."""
    import torch
    from paper_2103_02388_amd import mmoc
    wl = W.swirl3d(level=6)
    tr = mmoc.Tracer.from_workload(wl)
    N = tr.N
    c = torch.zeros(N, dtype=torch.float64, device=tr.device)
    u = torch.zeros((3, N), dtype=torch.float64, device=tr.device)
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_set_level_count(tr.ctx, 65536)
    assert e.value.status == -5
    tr.set_scalar(c)
    with pytest.raises(mmoc.MMOCError) as e:
        tr.trace_step(0.01, 1)
    assert e.value.status == -3
    with pytest.raises(mmoc.MMOCError) as e:
        mmoc.mmoc_set_velocity(tr.ctx, 0, u)
    assert e.value.status == -1
    mmoc.mmoc_set_level_count(tr.ctx, 2)
    tr.set_velocity(0, u)
    tr.set_velocity(1, u)
    ch, X = tr.trace_step(0.01, 1)
    torch.cuda.synchronize()
    x = tr.dof_coords()
    assert torch.equal(X, x)  # zero velocity: every particle stays at its DoF
    tr.close()
