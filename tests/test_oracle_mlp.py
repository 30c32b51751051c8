"""Pins of the surrogate network's CPU reference.

* gradient: central finite differences of the loss in float64 agree with the
  analytic backward pass (relative error <= 1e-6);
* bf16 rounding: values fixed by the bfloat16 format (8 significand bits,
  round to nearest, ties to even);
* GELU: values of the tanh form at points where it is known in closed form
  (0, large |u|) and its symmetry gelu(u) - gelu(-u) = u;
* Adam: one step from zero moments moves every parameter by lr * sign(g)
  (bias correction makes the first step size exactly lr, up to eps);
* training on a smooth target reduces the loss;
* the forward pass, its bf16 emulation and the gradient against an
  independent torch float64 network built from the header's layout.
"""
import math

import numpy as np
import pytest


def init_params(O, seed=0):
    rng = np.random.default_rng(seed)
    n = O.mlp_nparams()
    p = np.empty(n)
    off = 0
    for (o, i) in ((64, 4), (64, 64), (64, 64), (3, 64)):
        p[off:off + o * i] = rng.normal(size=o * i) * math.sqrt(2.0 / i)
        off += o * i
        p[off:off + o] = rng.normal(size=o) * 0.05
        off += o
    assert off == n
    return p


def test_param_count(oracle_mod):
    assert oracle_mod.mlp_nparams() == 8835


def test_finite_difference_gradient(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(1)
    p = init_params(O)
    x = rng.uniform(-1, 1, size=(16, 4))
    t = rng.normal(size=(16, 3))
    loss, g = O.mlp_loss_grad(p, x, t)
    idx = rng.choice(p.shape[0], 300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (O.mlp_loss_grad(p + e, x, t)[0] - O.mlp_loss_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_bf16_rounding_values(oracle_mod):
    r = oracle_mod.bf16_round
    assert r(1.0) == 1.0
    assert r(1.0 + 2.0 ** -8) == 1.0           # tie -> even (1.0)
    assert r(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even (odd neighbour rounds up)
    assert r(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7  # representable
    assert r(1.0 + 1.5 * 2.0 ** -8) == 1.0 + 2.0 ** -7
    assert r(-3.140625) == -3.140625
    assert r(3.14159) == 3.140625


def test_gelu_values(oracle_mod):
    g = oracle_mod.gelu
    assert g(0.0) == 0.0
    assert abs(g(10.0) - 10.0) < 1e-12 and abs(g(-10.0)) < 1e-12
    for u in (0.3, 1.7, -2.2):
        assert abs(g(u) - g(-u) - u) < 1e-15


def test_adam_first_step(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p0 = p.copy()
    O.adam_step(p, g, m, v, 1e-3, 1, eps=1e-12)
    assert np.abs((p0 - p) - 1e-3 * np.sign(g)).max() < 1e-12


def test_training_reduces_loss(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    p = init_params(O, 2)
    x = rng.uniform(-1, 1, size=(256, 4))
    t = np.stack([np.sin(x[:, 0] + x[:, 3]), x[:, 1] * x[:, 2], np.cos(x[:, 2])], axis=1) * 0.5
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = O.mlp_loss_grad(p, x, t)[0]
    for k in range(1, 201):
        loss, g = O.mlp_loss_grad(p, x, t)
        O.adam_step(p, g, m, v, 3e-3, k)
    assert loss < 0.1 * l0


def test_bf16_mode_is_close_to_fp64(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(5)
    p = init_params(O, 3)
    x = rng.uniform(-1, 1, size=(64, 4))
    y64 = O.mlp_forward(p, x)
    y16 = O.mlp_forward(p, x, bf16=True)
    rel = np.abs(y16 - y64).max() / np.abs(y64).max()
    assert 1e-5 < rel < 5e-2


def _torch_net(params, x, bf16=False):
    """The network as the header defines it, written independently of the
    oracle with torch float64 primitives: flat parameters W1[64][4] b1[64]
    W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3] (W[out][in]), tanh
    GELU after each of the three hidden layers, a linear output layer.  With
    bf16, the operands of the two 64 x 64 products (W2, W3, a1, a2) are
    rounded to bfloat16 by torch's own conversion."""
    import torch
    import torch.nn.functional as F
    p = torch.as_tensor(params, dtype=torch.float64)
    sizes = [(64, 4), (64,), (64, 64), (64,), (64, 64), (64,), (3, 64), (3,)]
    parts, off = [], 0
    for s in sizes:
        k = int(np.prod(s))
        parts.append(p[off:off + k].reshape(s))
        off += k
    assert off == p.numel()
    W1, b1, W2, b2, W3, b3, W4, b4 = parts

    def q(t):
        return t.to(torch.bfloat16).to(torch.float64) if bf16 else t

    a = torch.as_tensor(x, dtype=torch.float64)
    a1 = F.gelu(F.linear(a, W1, b1), approximate="tanh")
    a2 = F.gelu(F.linear(q(a1), q(W2), b2), approximate="tanh")
    a3 = F.gelu(F.linear(q(a2), q(W3), b3), approximate="tanh")
    return F.linear(a3, W4, b4)


def test_forward_matches_torch_float64(oracle_mod):
    """Pins orc_mlp_forward: element by element against the torch float64
    network above, on random inputs and parameters (rounding-level bound)."""
    O = oracle_mod
    rng = np.random.default_rng(6)
    for seed in (0, 1):
        p = init_params(O, 10 + seed)
        p[256:320] = rng.normal(size=64)   # non-zero hidden biases
        p[-3:] = rng.normal(size=3)
        x = rng.uniform(-1.5, 1.5, size=(500, 4))
        y = O.mlp_forward(p, x)
        yt = _torch_net(p, x).numpy()
        assert np.abs(y - yt).max() <= 1e-14 * max(1.0, np.abs(yt).max())


def test_bf16_forward_matches_torch(oracle_mod):
    """Pins the bf16 emulation: the oracle's bf16 mode against torch with its
    own bfloat16 conversion at the same operand points.  The sums run in a
    different order, so the bound is rounding-level, not bitwise; a bf16
    operand off by one unit (2^-8 relative) would exceed it."""
    O = oracle_mod
    rng = np.random.default_rng(7)
    p = init_params(O, 12)
    x = rng.uniform(-1, 1, size=(500, 4))
    y = O.mlp_forward(p, x, bf16=True)
    yt = _torch_net(p, x, bf16=True).numpy()
    assert np.abs(y - yt).max() <= 1e-12 * max(1.0, np.abs(yt).max())
    # and the rounding does matter at this bound: plain float64 is far off
    assert np.abs(O.mlp_forward(p, x) - yt).max() > 1e-6


def test_gradient_matches_torch_autograd(oracle_mod):
    """Pins orc_mlp_loss_grad in float64 against torch autograd of the loss
    1/(3B) sum |y - t|^2 of the torch network (independent of the finite
    differences above, which rest on the oracle's own forward pass)."""
    import torch
    O = oracle_mod
    rng = np.random.default_rng(8)
    p = init_params(O, 13)
    x = rng.uniform(-1, 1, size=(32, 4))
    t = rng.normal(size=(32, 3))
    loss, g = O.mlp_loss_grad(p, x, t)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    y = _torch_net(pt, x)
    lt = ((y - torch.as_tensor(t)) ** 2).sum() / (3 * x.shape[0])
    lt.backward()
    gt = pt.grad.numpy()
    assert abs(loss - lt.item()) <= 1e-14 * abs(lt.item())
    assert np.abs(g - gt).max() <= 1e-13 * np.abs(gt).max()
