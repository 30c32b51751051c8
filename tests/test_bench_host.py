"""Host-side logic of bench.py (no GPU): the algorithmic flop and byte
counts the roofline entry divides by, and the one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_flops_per_particle_3d_p2_rk4():
    # per stage evaluation: reference coordinates 25, micro location and P2
    # basis 44, P2 sums 120, time lerp 9, stage update 12 (FMA = 2)
    per_eval = 25 + 44 + 120 + 9 + 12
    scalar = 25 + 44 + 20
    assert bench.flops_per_particle(3, 2, 4) == 4 * (4 * per_eval + 6) + scalar == 3473
    # one level (stationary): no lerp, half the sums
    assert bench.flops_per_particle(3, 1, 4) == 4 * (4 * (per_eval - 60 - 9) + 6) + scalar
    # 2D: 6 nodes, 2 components
    ref2, micro2 = 2 + 8 + 2 + 1, (2 + 4 + 4) + 3 + 9 + 2 * 3
    assert bench.flops_per_particle(2, 2, 1) == 4 * (ref2 + micro2 + 2 * 6 * 2 * 2 + 6 + 8) + 4 + ref2 + micro2 + 12


def test_flops_per_particle_blended_shell():
    # the blended shell adds the inverse map Phi^-1(y) = y c |y| / (n.y) to
    # every location: n.y 5, |y|^2 5, sqrt 1, c r / (n.y) 2, three fused
    # scalings 6 (19 flops); one stationary level
    per_eval = 25 + 19 + 44 + 60 + 12
    scalar = 25 + 19 + 44 + 20
    assert bench.flops_per_particle(3, 1, 4, blend=True) == 4 * (4 * per_eval + 6) + scalar == 2692
    # and the shell's compulsory bytes: u (24) + c (8) in, chat (8) + X (24) out
    assert bench.bytes_per_particle(3, 1, 8) == 64


def test_compulsory_bytes_per_particle():
    # float64, two levels: u^n and u^{n+1} (48), c (8) in; chat (8) and X (24) out
    assert bench.bytes_per_particle(3, 2, 8) == 88
    # float32 records: the velocity levels, c and chat in float32, X in float64
    assert bench.bytes_per_particle(3, 2, 4) == 24 + 4 + 4 + 24


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
