"""Oracle pins for the RK4 departure-point trace and the scalar evaluation.

Closed forms (exact up to rounding because every field is a polynomial of
degree <= 2 in space, reproduced exactly by P2 including extrapolation):
  * translation u = a:           X = x - dt a
  * time-linear u^n = a, u^{n+1} = b:  X = x - dt (a+b)/2
  * linear autonomous u = A(x - c):    X = c + R4(-h A)^S (x - c), with
    R4(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24 the RK4 stability polynomial;
  * the whole step with a quadratic scalar q: chat = q(X).
Against the exact flow: a non-commuting, time-dependent linear field compared
with a tight ODE solve (pins stage times and the direction of the time
interpolation); the swirl field over [0, T] whose exact flow map is the
identity; and the paper's printed Table 2 rows (b = infinity).
"""
import json
import os

import numpy as np
import pytest
import torch
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from paper_2103_02388_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def R4(Z):
    I = np.eye(Z.shape[0])
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6 + Z @ Z @ Z @ Z / 24


def setup(O, wlf, level):
    wl = wlf()
    m = O.Mesh.from_workload(wl, level=level)
    return wl, m, m.dof_coords()


@pytest.mark.parametrize("wlf", [W.rotation2d, W.swirl3d])
def test_translation_and_time_linear(oracle_mod, wlf):
    rng = np.random.default_rng(0)
    wl, m, x = setup(oracle_mod, wlf, 2)
    d = m.dim
    a, b = rng.normal(size=d) * 0.4, rng.normal(size=d) * 0.4
    A = rng.normal(size=(d, d))
    q = lambda p: np.einsum("ij,ni,nj->n", A, p, p)
    c = q(x.T)
    U0 = np.tile(a[:, None], (1, m.N))
    U1 = np.tile(b[:, None], (1, m.N))
    for S in (1, 3):
        ch, X, _ = m.trace(U0, None, c, 0.2, S)
        assert np.abs(X - (x - 0.2 * a[:, None])).max() < 1e-14
        assert np.abs(ch - q(X.T)).max() < 1e-13
        ch, X, _ = m.trace(U0, U1, c, 0.2, S)
        assert np.abs(X - (x - 0.1 * (a + b)[:, None])).max() < 1e-14
        assert np.abs(ch - q((x - 0.1 * (a + b)[:, None]).T)).max() < 1e-12


@pytest.mark.parametrize("wlf", [W.rotation2d, W.swirl3d])
def test_linear_field_matches_rk4_stability_polynomial(oracle_mod, wlf):
    rng = np.random.default_rng(1)
    wl, m, x = setup(oracle_mod, wlf, 2)
    d = m.dim
    K = rng.normal(size=(d, d))
    A = K - K.T  # skew: solid-body rotation
    cen = np.full(d, 0.5)
    U = A @ (x - cen[:, None])
    dt, S = 0.3, 4
    h = dt / S
    _, X, _ = m.trace(U, None, np.zeros(m.N), dt, S)
    ref = cen[:, None] + np.linalg.matrix_power(R4(-h * A), S) @ (x - cen[:, None])
    assert np.abs(X - ref).max() < 1e-14
    # and RK4 tracks the exact rotation to O(S (h w)^5)
    exact = cen[:, None] + expm(-dt * A) @ (x - cen[:, None])
    w = np.abs(np.linalg.eigvals(A)).max()
    assert np.abs(X - exact).max() < 2 * S * (h * w) ** 5 / 120 + 1e-14


def test_time_dependent_noncommuting_field_converges_at_fourth_order(oracle_mod):
    """u(x, t) = ((1 - s) A0 + s A1) x with s = (t - t_n)/dt and [A0, A1] != 0.
    The departure point of a particle at t_{n+1} is the solution at t_n of the
    backward ODE; a reversed time interpolation converges to a different map."""
    wl, m, x = setup(oracle_mod, W.swirl3d, 1)
    A0 = np.array([[0.0, 1.0, 0.3], [-1.0, 0.0, 0.2], [-0.3, -0.2, 0.0]])
    A1 = np.array([[0.1, 0.0, -0.8], [0.4, -0.3, 0.5], [0.8, -0.5, 0.2]])
    dt = 0.8
    U0, U1 = A0 @ x, A1 @ x
    ids = np.arange(0, m.N, 5)

    def exact(p):
        f = lambda t, y: (((1 - t / dt) * A0 + (t / dt) * A1) @ y)
        return solve_ivp(f, (dt, 0.0), p, rtol=1e-13, atol=1e-14, method="DOP853").y[:, -1]

    ref = np.stack([exact(x[:, i]) for i in ids], axis=1)
    errs = []
    for S in (2, 4, 8):
        _, X, _ = m.trace(U0, U1, np.zeros(m.N), dt, S, ids=ids)
        errs.append(np.abs(X - ref).max())
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12 and errs[2] < 1e-5
    # the same field with the levels swapped is a different flow: the trace must notice
    _, Xs, _ = m.trace(U1, U0, np.zeros(m.N), dt, 8, ids=ids)
    assert np.abs(Xs - ref).max() > 100 * errs[2]


def test_swirl_full_period_is_identity(oracle_mod):
    """With u^n = swirl(t=0), u^{n+1} = swirl(t=T), dt = T, the interpolated
    velocity is g_lin(t) v_h(x) with zero time integral, so the exact flow map
    is the identity; RK4 converges to it (Sec. 3.3: the field reverses)."""
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    xt = torch.from_numpy(x.T.copy())
    U0 = W.swirl_velocity(xt, 0.0).numpy().T.copy()
    U1 = W.swirl_velocity(xt, W.SWIRL_T).numpy().T.copy()
    e = []
    for S in (16, 64):
        _, X, st = m.trace(U0, U1, np.zeros(m.N), W.SWIRL_T, S)
        e.append(np.abs(X - x).max())
    assert e[0] / e[1] > 30 and e[1] < 1e-5


def test_quadratic_scalar_whole_step(oracle_mod):
    rng = np.random.default_rng(9)
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    A = rng.normal(size=(3, 3))
    q = lambda p: np.einsum("ij,ni,nj->n", A, p, p) + p.sum(axis=1)
    a = np.array([0.3, -0.1, 0.2])
    ch, X, _ = m.trace(np.tile(a[:, None], (1, m.N)), None, q(x.T), 0.25, 2)
    assert np.abs(ch - q((x - 0.25 * a[:, None]).T)).max() < 1e-13


@pytest.mark.parametrize("row", [0, 1])
def test_paper_table2_b_infinity(oracle_mod, row):
    """Table 2 (hill only, P2, b = infinity): a stationary velocity traced over
    the whole revolution is one step of dt = 2 pi with `steps` RK4 sub-steps."""
    gold = json.load(open(os.path.join(GOLD, "table2_binf.json")))["rows"][row]
    wl, m, x = setup(oracle_mod, W.rotation2d, 6)
    assert m.N == 16641
    xt = torch.from_numpy(x.T.copy())
    U = W.rotation_velocity(xt).numpy().T.copy()
    c0 = W.hill(xt).numpy()
    ch, X, _ = m.trace(U, None, c0, 2 * np.pi, gold["steps"])
    e = c0 - ch
    h0 = np.sqrt(m.mass_quadform(e, e))
    dm = m.mass_quadform(np.ones(m.N), ch) / m.mass_quadform(np.ones(m.N), c0) - 1
    var = ch.max() - ch.min()
    # printed with three significant digits
    assert abs(h0 / gold["H0"] - 1) < 0.01
    assert abs(dm / gold["dm"] - 1) < 0.01
    assert abs(var - gold["var"]) < 1e-4


def test_mass_matrix_closed_forms(oracle_mod):
    for wl in (W.rotation2d(), W.swirl3d()):
        Mref = oracle_mod.p2_mass_ref(wl.dim)
        assert abs(Mref.sum() - 1.0) < 1e-14  # integral of 1 over T is |T|
        m = oracle_mod.Mesh.from_workload(wl, level=2)
        x = m.dof_coords()
        one = np.ones(m.N)
        assert abs(m.mass_quadform(one, one) - 1.0) < 1e-13
        # integral of x_0^2 over the unit square / cube = 1/3; of x_0 x_1 = 1/4
        assert abs(m.mass_quadform(one, x[0] ** 2) - 1 / 3) < 1e-13
        assert abs(m.mass_quadform(x[0], x[1]) - 1 / 4) < 1e-13


@pytest.mark.parametrize("steps,b", [(62, 1), (62, 10), (628, 1)])
def test_paper_table2_finite_lookback(oracle_mod, steps, b):
    """Table 2 rows with a finite look-back distance (Sec. 2.3.3): every step
    re-interpolates, so the error is the accumulated interpolation error the
    paper attributes to the Eulerian-Lagrangian transfer.  The oracle runs the
    look-back recursion c^n = c^{n-b'}(X_{b'}) step by step; H0 and var must
    match the printed three digits within 5% and 2e-4."""
    rows = json.load(open(os.path.join(GOLD, "table2_lookback.json")))["rows"]
    gold = [r for r in rows if r["steps"] == steps and r["b"] == b][0]
    wl, m, x = setup(oracle_mod, W.rotation2d, 6)
    xt = torch.from_numpy(x.T.copy())
    U = W.rotation_velocity(xt).numpy().T.copy()
    c0 = W.hill(xt).numpy()
    tau = 2 * np.pi / steps
    hist = {0: c0}
    for n in range(1, steps + 1):
        bp = min(b, n)
        hist[n], _, _ = m.trace(U, None, hist[n - bp], bp * tau, bp, threads=4)
        hist.pop(n - b - 1, None)
    c = hist[steps]
    e = c0 - c
    h0 = np.sqrt(m.mass_quadform(e, e))
    assert abs(h0 / gold["H0"] - 1) < 0.05, h0
    assert abs((c.max() - c.min()) - gold["var"]) < 2e-4


def test_paper_table1_b_infinity(oracle_mod):
    """Table 1, P2, b = infinity (three bodies, one revolution in 6283
    steps): tracing the whole revolution back in one go returns every
    particle to its own position up to the RK4 error of the exact rotation,
    so the error and the mass change are at rounding level and var is 1."""
    gold = [r for r in json.load(open(os.path.join(GOLD, "table1_p2.json")))["rows"] if r["b"] == 0][0]
    wl, m, x = setup(oracle_mod, W.rotation2d, 6)
    xt = torch.from_numpy(x.T.copy())
    U = W.rotation_velocity(xt).numpy().T.copy()
    c0 = (W.slotted_cylinder(xt) + W.cone(xt) + W.hill(xt)).numpy()
    ch, X, _ = m.trace(U, None, c0, 2 * np.pi, 6283, threads=8)
    e = c0 - ch
    h0 = np.sqrt(m.mass_quadform(e, e))
    one = np.ones(m.N)
    dm = m.mass_quadform(one, ch) / m.mass_quadform(one, c0) - 1
    assert h0 < 10 * gold["H0"] and abs(dm) < 1e-12
    assert abs((ch.max() - ch.min()) - gold["var"]) < 1e-4


# ---------------------------------------------------------------- general explicit RK (Sec. 3.1)

from rk_tableaux import TABLEAUX, stability_matrix, tableau  # noqa: E402


@pytest.mark.parametrize("name", list(TABLEAUX))
def test_general_rk_linear_field_matches_stability_polynomial(oracle_mod, name):
    """Any explicit RK method applied to u = Om (x - c), Om skew, advances
    x - c by its stability matrix R(-h Om) per sub-step; P2 reproduces the
    linear field exactly, so the traced departure points are that product."""
    rng = np.random.default_rng(31)
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    K = rng.normal(size=(3, 3))
    Om = K - K.T
    cen = np.full(3, 0.5)
    U = Om @ (x - cen[:, None])
    dt, S = 0.3, 3
    h = dt / S
    A, b, c, _ = tableau(name)
    _, X, _ = m.trace(U, None, np.zeros(m.N), dt, S, tableau=(A, b, c))
    ref = cen[:, None] + np.linalg.matrix_power(stability_matrix(name, -h * Om), S) @ (x - cen[:, None])
    assert np.abs(X - ref).max() < 1e-14


@pytest.mark.parametrize("name", list(TABLEAUX))
def test_general_rk_time_linear_translation(oracle_mod, name):
    """u^n = a, u^{n+1} = b' everywhere: every stage sees the constant
    (1 - theta) a + theta b' at its node theta = 1 - (j + c_i)/S, so
    X = x - h sum_j sum_i b_i ((1 - theta_ij) a + theta_ij b')."""
    rng = np.random.default_rng(32)
    wl, m, x = setup(oracle_mod, W.rotation2d, 2)
    a, bb = rng.normal(size=2) * 0.4, rng.normal(size=2) * 0.4
    A, b, c, p = tableau(name)
    dt, S = 0.2, 3
    h = dt / S
    _, X, _ = m.trace(np.tile(a[:, None], (1, m.N)), np.tile(bb[:, None], (1, m.N)), np.zeros(m.N), dt, S,
                      tableau=(A, b, c))
    disp = np.zeros(2)
    for j in range(S):
        for i in range(b.shape[0]):
            th = 1.0 - (j + c[i]) / S
            disp += h * b[i] * ((1 - th) * a + th * bb)
    assert np.abs(X - (x - disp[:, None])).max() < 1e-14
    if p >= 2:  # exact quadrature of a linear integrand
        assert np.abs(X - (x - dt * 0.5 * (a + bb)[:, None])).max() < 1e-14


def test_general_rk_rk4_tableau_equals_rk4(oracle_mod):
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    xt = torch.from_numpy(x.T.copy())
    U0 = W.swirl_velocity(xt, 0.3).numpy().T.copy()
    U1 = W.swirl_velocity(xt, 0.3 + wl.dt).numpy().T.copy()
    c0 = W.two_blobs(xt).numpy()
    ch, X, _ = m.trace(U0, U1, c0, wl.dt, 4)
    A, b, c, _ = tableau("rk4")
    ch2, X2, _ = m.trace(U0, U1, c0, wl.dt, 4, tableau=(A, b, c))
    assert np.abs(X - X2).max() < 1e-14 and np.abs(ch - ch2).max() < 1e-13


@pytest.mark.parametrize("name", ["heun", "midpoint", "rk3", "rk38"])
def test_general_rk_convergence_order(oracle_mod, name):
    """The non-commuting time-dependent linear field of the RK4 test: the
    error of each method falls by 2^p per halving of h."""
    wl, m, x = setup(oracle_mod, W.swirl3d, 1)
    A0 = np.array([[0.0, 1.0, 0.3], [-1.0, 0.0, 0.2], [-0.3, -0.2, 0.0]])
    A1 = np.array([[0.1, 0.0, -0.8], [0.4, -0.3, 0.5], [0.8, -0.5, 0.2]])
    dt = 0.8
    U0, U1 = A0 @ x, A1 @ x
    ids = np.arange(0, m.N, 5)

    def exact(p0):
        f = lambda t, y: (((1 - t / dt) * A0 + (t / dt) * A1) @ y)
        return solve_ivp(f, (dt, 0.0), p0, rtol=1e-13, atol=1e-14, method="DOP853").y[:, -1]

    ref = np.stack([exact(x[:, i]) for i in ids], axis=1)
    A, b, c, p = tableau(name)
    errs = []
    for S in (8, 16, 32):
        _, X, _ = m.trace(U0, U1, np.zeros(m.N), dt, S, ids=ids, tableau=(A, b, c))
        errs.append(np.abs(X - ref).max())
    rates = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    assert min(rates) > p - 0.3, (name, rates)


# ---------------------------------------------------------------- traces across several steps (Sec. 2.3.3)


def test_span_single_interval_is_the_step(oracle_mod):
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    xt = torch.from_numpy(x.T.copy())
    U0 = W.swirl_velocity(xt, 0.3).numpy().T.copy()
    U1 = W.swirl_velocity(xt, 0.3 + wl.dt).numpy().T.copy()
    c0 = W.two_blobs(xt).numpy()
    ch, X, _ = m.trace(U0, U1, c0, wl.dt, 3)
    ch2, X2, _ = m.trace_span([U0, U1], c0, wl.dt, 3)
    assert np.array_equal(X, X2) and np.array_equal(ch, ch2)


def test_span_piecewise_linear_translation(oracle_mod):
    """Spatially constant levels a_l: RK4 integrates a velocity linear in time
    exactly on each sub-step, and every sub-step lies in one interval, so
    X = x - sum_l tau (a_l + a_{l+1}) / 2."""
    rng = np.random.default_rng(41)
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    a = rng.normal(size=(5, 3)) * 0.2
    levels = [np.tile(al[:, None], (1, m.N)) for al in a]
    tau = 0.07
    for S in (1, 2):
        _, X, _ = m.trace_span(levels, np.zeros(m.N), tau, S)
        disp = sum(tau * 0.5 * (a[l] + a[l + 1]) for l in range(4))
        assert np.abs(X - (x - disp[:, None])).max() < 1e-14


def test_span_swirl_period_is_identity(oracle_mod):
    """Levels of the swirl at t_k = k T / K, k = 0..K: the piecewise-linear
    interpolation of g(t) = cos(pi t / T) at nodes symmetric about T/2 has
    zero integral over [0, T], and the field is g(t) v(x), so the exact flow
    map over the period is the identity.  RK4 approaches it as the sub-step
    shrinks; the P2 velocity is only continuous across element faces, so
    the observed rate is below four (the same bound as the single-step
    period test: a factor above 30 per fourfold refinement)."""
    wl, m, x = setup(oracle_mod, W.swirl3d, 2)
    xt = torch.from_numpy(x.T.copy())
    K = 6
    tau = W.SWIRL_T / K
    levels = [W.swirl_velocity(xt, k * tau).numpy().T.copy() for k in range(K + 1)]
    e = []
    for S in (4, 16):
        _, X, _ = m.trace_span(levels, np.zeros(m.N), tau, S)
        e.append(np.abs(X - x).max())
    assert e[0] / e[1] > 30 and e[1] < 1e-5
