"""An end-to-end pin of the oracle's trace on the blended spherical shell.

The blending map of the shell (per macro column, the radial projection
between the flat computational shell and the round one) is nonlinear, so a
general velocity has no closed-form trace there.  One family does.  Let
xi = Phi^-1(y) be the computational coordinates of a physical point y:
xi = y c |y| / (n . y), with the column's plane n . x = c through the tips
of its three unit directions.  For a velocity that is affine in them,
u(y) = A xi(y) + b, the P2 interpolant on any element of the column that
contains y equals u exactly (the nodal values are A xi_i + b, and xi is
affine in the element's reference coordinates; extrapolation past the
element is exact too).  So the tracer's velocity is the closed form at every
stage point it places in the right column, and its RK4 departure point
equals a mesh-free RK4 of dy/dt = -u(y) to rounding (Sec. 2.3: backward RK4
with S sub-steps, Alg. 1).  A wrong column shows: its plane gives a
different xi.  The scalar c = xi_0 is reproduced the same way, so
chat = Phi^-1(X)_0.

A is antisymmetric and b = 0: xi is parallel to y, so u = A xi is tangent to
the spheres and the particles keep their radius up to RK4's drift (a few
1e-9 here).  That drift pushes some DoFs of the inner and outer spheres out
of the shell, where a point keeps its last macro, whose column need not
contain it: the method then extrapolates from a neighbouring column and the
closed form no longer applies.  The DoFs on those two spheres are left out;
every other DoF is compared.

The reference here uses the mesh's vertex and macro lists only: it rebuilds
each column's directions and plane, and finds the column of a point as the
cone of three directions that contains it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2103_02388_amd import workloads as W


class Columns:
    """The macro columns of a blended shell (3D: cones of three unit
    directions) or annulus (2D: sectors of two) from the vertex and macro
    lists."""

    def __init__(self, v, m):
        d = v.shape[1]
        unit = v / np.linalg.norm(v, axis=1, keepdims=True)
        key = {}
        cols = []
        for mac in m:
            ds = []
            for a in mac:
                q = unit[a]
                if not any(np.abs(q - e).sum() < 1e-9 for e in ds):
                    ds.append(q)
            assert len(ds) == d
            k = tuple(sorted(tuple(np.round(e * 1e9).astype(np.int64)) for e in ds))
            if k not in key:
                key[k] = len(cols)
                cols.append(np.array(ds))
        D = np.stack(cols)                       # [C, d directions, d]
        self.Dinv = np.linalg.inv(np.transpose(D, (0, 2, 1)))   # y = D^T alpha
        if d == 3:
            n = np.cross(D[:, 1] - D[:, 0], D[:, 2] - D[:, 0])
        else:                                    # normal of the chord between the two directions
            e = D[:, 1] - D[:, 0]
            n = np.stack([-e[:, 1], e[:, 0]], axis=1)
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        c = np.einsum("ci,ci->c", n, D[:, 0])
        s = np.where(c < 0, -1.0, 1.0)
        self.n, self.c = n * s[:, None], c * s

    def column(self, y):
        """index of the cone containing each point (largest smallest cone
        coordinate: a point on a shared face may take either column)"""
        out = np.empty(len(y), dtype=np.int64)
        for lo in range(0, len(y), 4096):
            a = np.einsum("cij,pj->pci", self.Dinv, y[lo:lo + 4096])
            out[lo:lo + 4096] = np.argmax(a.min(axis=2), axis=1)
        return out

    def phi_inv(self, y):
        k = self.column(y)
        n, c = self.n[k], self.c[k]
        f = c * np.linalg.norm(y, axis=1) / np.einsum("pi,pi->p", n, y)
        return y * f[:, None]


A0 = np.array([[0.0, -1.0, 0.3], [1.0, 0.0, -0.2], [-0.3, 0.2, 0.0]])
B0 = np.zeros(3)


def rk4_reference(cols, A, b, x, dt, S):
    """backward RK4 with S sub-steps of dy/dt = -(A Phi^-1(y) + b)"""
    def u(y):
        return cols.phi_inv(y) @ A.T + b
    h = dt / S
    Y = x.copy()
    for _ in range(S):
        k1 = u(Y)
        k2 = u(Y - 0.5 * h * k1)
        k3 = u(Y - 0.5 * h * k2)
        k4 = u(Y - h * k3)
        Y = Y - h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return Y


@pytest.mark.parametrize("level", [1, 2])
def test_shell_trace_with_velocity_affine_in_the_computational_coordinates(level):
    wl = W.shell3d(level=level)
    v, m = W.shell(4, 4)
    cols = Columns(v, m)
    assert len(cols.c) == 320 and np.all(cols.c > 0)
    om = O.Mesh.from_workload(wl)
    x = om.dof_coords().T.copy()                 # [N, 3] physical DoF positions
    xi = cols.phi_inv(x)
    r = np.linalg.norm(x, axis=1)
    u_nodes = xi @ A0.T + B0
    scale = 1.0 / np.abs(u_nodes).max()
    A, b = A0 * scale, B0 * scale
    u_nodes = u_nodes * scale
    interior = np.nonzero((r > 0.55 + 1e-9) & (r < 1.0 - 1e-9))[0]
    rng = np.random.default_rng(level)
    ids = np.sort(rng.choice(interior, min(len(interior), 8000), replace=False))
    S = 4
    ch, X, st = om.trace(u_nodes.T, None, xi[:, 0], wl.dt, S, ids=ids, threads=8)
    Xr = rk4_reference(cols, A, b, x[ids], wl.dt, S)
    ex = np.abs(X.T - Xr).max()
    chr_ = cols.phi_inv(X.T)[:, 0]
    ec = np.abs(ch - chr_).max()
    moved = np.linalg.norm(X.T - x[ids], axis=1)
    print("level %d: %d particles, walks %d, |X - X_ref| %.2e, |chat - xi0(X)| %.2e, "
          "mean displacement %.3f (h_min %.4f)"
          % (level, len(ids), st[1], ex, ec, moved.mean(), wl.extra["h_min"]))
    assert st[1] > 0 and st[0] == 0              # stage points walk across macros, none leaves
    assert np.all(np.abs(np.linalg.norm(X, axis=0) - r[ids]) < 1e-6)   # tangential
    assert ex <= 1e-12
    assert ec <= 1e-12


def test_annulus_trace_with_velocity_affine_in_the_computational_coordinates():
    """The same pin in 2D on the blended annulus of the diffusion benchmark
    (6 sectors, levels 4 and 5): u = J xi with J the quarter turn, tangent to
    the circles.  The DoFs on the inner and outer circles are left out."""
    v, m = W.annulus()
    cols = Columns(v, m)
    assert len(cols.c) == 6 and np.all(cols.c > 0)
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    for level in (4, 5):
        wl = W.annulus2d(level=level)
        om = O.Mesh.from_workload(wl)
        x = om.dof_coords().T.copy()
        xi = cols.phi_inv(x)
        r = np.linalg.norm(x, axis=1)
        interior = np.nonzero((r > 0.5 + 1e-9) & (r < 1.5 - 1e-9))[0]
        u_nodes = xi @ J.T
        ids = np.sort(np.random.default_rng(level).choice(interior, 6000, replace=False))
        dt = 0.3                                 # several macros' worth of walk per step
        ch, X, st = om.trace(u_nodes.T, None, xi[:, 0], dt, 4, ids=ids, threads=8)
        Xr = rk4_reference(cols, J, np.zeros(2), x[ids], dt, 4)
        ex = np.abs(X.T - Xr).max()
        ec = np.abs(ch - cols.phi_inv(X.T)[:, 0]).max()
        print("annulus level %d: %d particles, walks %d, |X - X_ref| %.2e, |chat - xi0(X)| %.2e"
              % (level, len(ids), st[1], ex, ec))
        assert st[1] > 0 and st[0] == 0
        assert ex <= 1e-12 and ec <= 1e-12


def test_shell_trace_between_two_velocity_levels():
    """Two velocity levels u^n = A1 xi, u^{n+1} = A2 xi (both antisymmetric),
    linear in time: at sub-step j and RK4 node a the tracer takes the later
    level with weight theta = 1 - (j + a) / S (the trace runs back from
    t_{n+1}), so the mesh-free reference integrates
    u(y, theta) = ((1 - theta) A1 + theta A2) Phi^-1(y) with those weights."""
    wl = W.shell3d(level=1)
    v, m = W.shell(4, 4)
    cols = Columns(v, m)
    om = O.Mesh.from_workload(wl)
    x = om.dof_coords().T.copy()
    xi = cols.phi_inv(x)
    r = np.linalg.norm(x, axis=1)
    A1 = A0 / np.abs(xi @ A0.T).max()
    K = np.array([[0.0, 0.4, -1.0], [-0.4, 0.0, 0.6], [1.0, -0.6, 0.0]])
    A2 = K / np.abs(xi @ K.T).max()
    interior = np.nonzero((r > 0.55 + 1e-9) & (r < 1.0 - 1e-9))[0]
    ids = np.sort(np.random.default_rng(5).choice(interior, 8000, replace=False))
    S, dt = 4, wl.dt
    ch, X, st = om.trace((xi @ A1.T).T, (xi @ A2.T).T, xi[:, 0], dt, S, ids=ids, threads=8)
    h = dt / S

    def u(y, theta):
        return cols.phi_inv(y) @ ((1.0 - theta) * A1 + theta * A2).T
    Y = x[ids].copy()
    for j in range(S):
        k1 = u(Y, 1.0 - j / S)
        k2 = u(Y - 0.5 * h * k1, 1.0 - (j + 0.5) / S)
        k3 = u(Y - 0.5 * h * k2, 1.0 - (j + 0.5) / S)
        k4 = u(Y - h * k3, 1.0 - (j + 1.0) / S)
        Y = Y - h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    ex = np.abs(X.T - Y).max()
    ec = np.abs(ch - cols.phi_inv(X.T)[:, 0]).max()
    # the other direction of the time weights is far off
    Yw = x[ids].copy()
    for j in range(S):
        k1 = u(Yw, j / S)
        k2 = u(Yw - 0.5 * h * k1, (j + 0.5) / S)
        k3 = u(Yw - 0.5 * h * k2, (j + 0.5) / S)
        k4 = u(Yw - h * k3, (j + 1.0) / S)
        Yw = Yw - h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    print("two levels: walks %d, |X - X_ref| %.2e, |chat - xi0(X)| %.2e, reversed weights %.2e"
          % (st[1], ex, ec, np.abs(X.T - Yw).max()))
    assert st[0] == 0 and ex <= 1e-12 and ec <= 1e-12
    assert np.abs(X.T - Yw).max() > 1e-3


def test_reference_column_map_is_continuous_and_exact_on_the_directions():
    """The reference Phi^-1 itself: the identity on the column directions'
    rays through the macro vertices, continuous across column faces (points
    on a shared face map alike from both sides), and sending the round
    sphere of radius r to the flat shell n . xi = c r."""
    v, m = W.shell(4, 4)
    cols = Columns(v, m)
    assert np.abs(cols.phi_inv(v) - v).max() < 1e-14
    rng = np.random.default_rng(3)
    y = rng.normal(size=(20000, 3))
    y *= (0.55 + 0.45 * rng.random(20000))[:, None] / np.linalg.norm(y, axis=1, keepdims=True)
    k = cols.column(y)
    xi = cols.phi_inv(y)
    assert np.abs(np.einsum("pi,pi->p", cols.n[k], xi) - cols.c[k] * np.linalg.norm(y, axis=1)).max() < 1e-14
    # the same point through every column whose cone holds it (faces and edges)
    a = np.einsum("cij,pj->pci", cols.Dinv, y[:2000])
    for p in range(2000):
        inside = np.nonzero(a[p].min(axis=1) > -1e-12)[0]
        vals = [y[p] * cols.c[j] * np.linalg.norm(y[p]) / (cols.n[j] @ y[p]) for j in inside]
        assert max(np.abs(w - vals[0]).max() for w in vals) < 1e-14
