"""Oracle pins: P2 evaluation, micro location, macro walk.

* any quadratic is reproduced exactly by its P2 interpolant, inside the
  domain and (by extrapolation of the selected element) outside it;
* the O(1) micro location agrees with a brute-force search over all micro
  simplices (barycentrics computed here from vertex coordinates);
* the walk agrees with brute force, and on the Kuhn cube with the global
  Freudenthal rule (the macro is given by the order of the coordinates).
"""
import itertools

import numpy as np
import pytest

from paper_2103_02388_amd import workloads as W


def rand_quadratic(rng, d):
    A = rng.normal(size=(d, d))
    b = rng.normal(size=d)
    c0 = rng.normal()
    return lambda p: np.einsum("ij,ni,nj->n", A, p, p) + p @ b + c0


@pytest.mark.parametrize("wlf,level", [(W.rotation2d, 1), (W.rotation2d, 3), (W.swirl3d, 1), (W.swirl3d, 3)])
def test_p2_reproduces_quadratics_inside_and_outside(oracle_mod, wlf, level):
    rng = np.random.default_rng(level)
    wl = wlf()
    m = oracle_mod.Mesh.from_workload(wl, level=level)
    q = rand_quadratic(rng, m.dim)
    f = q(m.dof_coords().T)
    pts = np.concatenate([rng.uniform(0, 1, size=(3000, m.dim)), rng.uniform(-0.3, 1.3, size=(1000, m.dim))])
    for start in (None, 0):
        out, _, _ = m.eval(f, pts, start=start)
        assert np.abs(out[:, 0] - q(pts)).max() < 1e-13 * max(1.0, np.abs(q(pts)).max())


def test_p2_kronecker_and_partition_of_unity(oracle_mod):
    for wl in (W.rotation2d(), W.swirl3d()):
        m = oracle_mod.Mesh.from_workload(wl, level=1)
        x = m.dof_coords()
        E = np.eye(m.N)
        out, _, _ = m.eval(E, x.T, start=0)
        assert np.abs(out - np.eye(m.N)).max() < 1e-13
        rng = np.random.default_rng(1)
        pts = rng.uniform(0, 1, size=(500, m.dim))
        out, _, _ = m.eval(np.ones(m.N), pts)
        assert np.abs(out - 1).max() < 1e-13


def _contains(verts, p, tol=1e-12):
    """barycentrics of p w.r.t. simplex verts [(d+1), d] computed from scratch"""
    d = len(p)
    T = np.stack([verts[a] - verts[0] for a in range(1, d + 1)], axis=1)
    s = np.linalg.solve(T, p - verts[0])
    lam = np.concatenate([[1 - s.sum()], s])
    return lam.min() >= -tol, lam


@pytest.mark.parametrize("wlf,level", [(W.rotation2d, 2), (W.swirl3d, 1), (W.swirl3d, 2)])
def test_micro_locate_matches_brute_force(oracle_mod, wlf, level):
    rng = np.random.default_rng(7 + level)
    wl = wlf()
    m = oracle_mod.Mesh.from_workload(wl, level=level)
    d, n = m.dim, m.n
    allsimp = m.micro_simplices()
    for M in range(m.nm):
        v0, B, _, _ = m.geometry(M)
        # random interior points, lattice points (ties), points on lattice planes
        s = rng.dirichlet(np.ones(d + 1), size=300)[:, 1:]
        lat = []
        for I in range(n + 1):
            for J in range(I + 1):
                for K in range(J + 1 if d == 3 else 1):
                    w = np.array([I, J, K][:d], dtype=float) / n
                    lat.append(np.append(w[:-1] - w[1:], w[-1]))
        half = rng.integers(0, 2 * n + 1, size=(100, d)) / (2 * n)
        half = np.sort(half, axis=1)[:, ::-1]  # Kuhn-ordered w
        half = np.stack([np.append(w[:-1] - w[1:], w[-1]) for w in half])
        for sv in np.concatenate([s, np.array(lat), half]):
            p = v0 + B @ sv
            V, mu = m.micro_simplex(M, p)
            # vertices in physical space
            Vp = np.array([v0 + B @ np.append(w[:-1] - w[1:], w[-1]) for w in V / n])
            ok, lam = _contains(Vp, p)
            assert ok, (M, sv, V, lam)
            assert np.abs(lam - mu).max() < 1e-12
            assert any(frozenset(map(tuple, V.tolist())) == frozenset(map(tuple, S.tolist())) for S in allsimp)


@pytest.mark.parametrize("wlf", [W.rotation2d, W.swirl3d])
def test_walk_matches_brute_force(oracle_mod, wlf):
    rng = np.random.default_rng(3)
    wl = wlf()
    m = oracle_mod.Mesh.from_workload(wl, level=0)
    for _ in range(2000):
        p = rng.uniform(0, 1, size=m.dim)
        start = int(rng.integers(0, m.nm))
        M, fl = m.walk(start, p)
        Mb = m.brute(p)
        assert M == Mb or m.bary(M, p).min() >= -1e-12
        assert m.bary(M, p).min() >= -1e-12
        assert fl & 1 == 0
    for _ in range(500):
        p = rng.uniform(-0.5, 1.5, size=m.dim)
        M, fl = m.walk(int(rng.integers(0, m.nm)), p)
        inside = np.all((p >= 0) & (p <= 1))
        if not inside:
            assert fl & 1  # flagged outside


def test_cube_walk_is_global_freudenthal(oracle_mod):
    """In the six-tet cube the macro containing p is the Kuhn tet of the
    permutation that sorts p's coordinates in descending order."""
    rng = np.random.default_rng(11)
    wl = W.swirl3d()
    m = oracle_mod.Mesh.from_workload(wl, level=0)
    perms = list(itertools.permutations(range(3)))
    for _ in range(2000):
        p = rng.uniform(0, 1, size=3)
        order = tuple(int(i) for i in np.argsort(-p))
        M, _ = m.walk(int(rng.integers(0, 6)), p)
        assert perms[M][:2] == order[:2]


def test_walk_hop_limit_falls_back_to_brute_force(oracle_mod):
    wl = W.swirl3d()
    m = oracle_mod.Mesh.from_workload(wl, level=0)
    rng = np.random.default_rng(5)
    for _ in range(200):
        p = rng.uniform(0, 1, size=3)
        M0, _ = m.walk(0, p, max_hops=64)
        M1, fl = m.walk(0, p, max_hops=0)
        if m.bary(0, p).min() < -1e-12:
            assert fl & 4
        assert m.bary(M1, p).min() >= -1e-12 and (M1 == M0 or m.bary(M0, p).min() >= -1e-12)


def test_shell_blending_roundtrip_and_layers(oracle_mod):
    wl = W.shell3d(level=1)
    m = oracle_mod.Mesh.from_workload(wl, level=1)
    x = m.dof_coords()
    r = np.linalg.norm(x, axis=0)
    radii = np.linspace(0.55, 1.0, 4 * 4 + 1)
    # every DoF lies on one of the refined layer spheres
    assert np.abs(r[:, None] - radii[None, :]).min(axis=1).max() < 1e-14
    assert r.min() > 0.55 - 1e-14 and r.max() < 1.0 + 1e-14
    # Phi(Phi^-1(z)) = z per column, checked with plane data from the oracle
    rng = np.random.default_rng(2)
    for M in rng.integers(0, m.nm, size=50):
        nrm, c = m.plane(M)
        z = rng.normal(size=3)
        z = z / np.linalg.norm(z) * rng.uniform(0.55, 1.0)
        if nrm @ z <= 0:
            continue
        xc = z * c * np.linalg.norm(z) / (nrm @ z)
        back = xc * (nrm @ xc) / (c * np.linalg.norm(xc))
        assert np.abs(back - z).max() < 1e-14
        assert abs(nrm @ xc - c * np.linalg.norm(z)) < 1e-14


def test_shell_quadratic_in_computational_space(oracle_mod):
    """With blending, a field that is quadratic in computational coordinates
    (q(Phi^-1(z))) is reproduced exactly at any physical point."""
    wl = W.shell3d(level=1)
    m = oracle_mod.Mesh.from_workload(wl, level=1)
    rng = np.random.default_rng(4)
    A = rng.normal(size=(3, 3))
    q = lambda p: np.einsum("ij,ni,nj->n", A, p, p)
    own, _ = m.dof_owner()
    x = m.dof_coords().T

    def comp(M, z):
        nrm, c = m.plane(M)
        return z * c * np.linalg.norm(z) / (nrm @ z)

    f = np.array([q(comp(own[u], x[u])[None])[0] for u in range(m.N)])
    pts = rng.normal(size=(300, 3))
    pts = pts / np.linalg.norm(pts, axis=1, keepdims=True) * rng.uniform(0.56, 0.99, size=(300, 1))
    out, mac, _ = m.eval(f, pts)
    ref = np.array([q(comp(mac[i], pts[i])[None])[0] for i in range(300)])
    assert np.abs(out[:, 0] - ref).max() < 1e-12
