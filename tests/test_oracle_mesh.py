"""Oracle pins: refinement lattice, unique DoF enumeration, neighbours.

The P2 DoFs of the refined Kuhn cube / square are exactly the global grid
(i/m)^d, so their count and positions pin the enumeration; the paper's DoF
count for the 2D rotation mesh is 16641 (Table 1 caption, Sec. 3.2).  The
refinement is pinned to Bey's rule by refining recursively with the
eight-children formula and comparing the micro simplices.
"""
import itertools

import numpy as np
import pytest

from paper_2103_02388_amd import workloads as W


def mesh(O, wl, level):
    return O.Mesh.from_workload(wl, level=level)


def test_dof_count_matches_paper(oracle_mod):
    m = mesh(oracle_mod, W.rotation2d(), 6)
    assert m.N == 16641  # Table 1 caption: 16641 DoFs for P2 with h = 1/64


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_cube_dofs_are_the_global_grid(oracle_mod, level):
    m = mesh(oracle_mod, W.swirl3d(), level)
    mm = 2 ** (level + 1)
    assert m.N == (mm + 1) ** 3
    x = m.dof_coords()
    ijk = np.rint(x * mm).astype(np.int64)
    assert np.abs(x * mm - ijk).max() < 1e-12
    keys = ijk[0] * (mm + 1) ** 2 + ijk[1] * (mm + 1) + ijk[2]
    assert len(np.unique(keys)) == m.N and keys.min() == 0 and keys.max() == (mm + 1) ** 3 - 1


@pytest.mark.parametrize("level", [0, 2, 4])
def test_square_dofs_are_the_global_grid(oracle_mod, level):
    m = mesh(oracle_mod, W.rotation2d(), level)
    mm = 2 ** (level + 1)
    x = m.dof_coords()
    ij = np.rint(x * mm).astype(np.int64)
    assert np.abs(x * mm - ij).max() < 1e-12
    assert len(np.unique(ij[0] * (mm + 1) + ij[1])) == m.N == (mm + 1) ** 2


def test_lattice_index_is_enumeration_order(oracle_mod):
    for dim in (2, 3):
        cnt = 0
        m = 6
        for I in range(m + 1):
            for J in range(I + 1):
                for K in range(J + 1 if dim == 3 else 1):
                    assert oracle_mod.lat_idx(dim, I, J, K) == cnt
                    cnt += 1


@pytest.mark.parametrize("wlf,level", [(W.swirl3d, 2), (W.rotation2d, 3)])
def test_owner_is_lowest_containing_macro(oracle_mod, wlf, level):
    wl = wlf()
    m = mesh(oracle_mod, wl, level)
    x = m.dof_coords()
    own, lat = m.dof_owner()
    # macro-major order
    assert np.all(np.diff(own) >= 0)
    for u in range(0, m.N, 7):
        containing = [M for M in range(m.nm) if m.bary(M, x[:, u]).min() >= -1e-13]
        assert own[u] == min(containing)
    # within a macro, lattice order increases
    idx = np.array([oracle_mod.lat_idx(m.dim, *lat[u][: 3]) for u in range(m.N)])
    for M in range(m.nm):
        assert np.all(np.diff(idx[own == M]) > 0)


def test_neighbours_symmetric_and_share_faces(oracle_mod):
    for wl in (W.swirl3d(), W.rotation2d()):
        m = mesh(oracle_mod, wl, 0)
        d = m.dim
        for M in range(m.nm):
            _, _, _, nb = m.geometry(M)
            for k in range(d + 1):
                if nb[k] < 0:
                    continue
                face = set(wl.macros[M]) - {wl.macros[M][k]}
                assert face <= set(wl.macros[nb[k]])
                _, _, _, nb2 = m.geometry(nb[k])
                assert M in nb2


def test_shell_mesh_counts(oracle_mod):
    wl = W.shell3d(level=0)
    assert wl.macros.shape[0] == 3840
    m = mesh(oracle_mod, wl, 0)
    # P2 at level 0: vertices + edges of the macro mesh
    assert m.N > 0
    # every shared face appears in exactly two macros; boundary faces lie on the two spheres
    nbr = np.array([m.geometry(M)[3] for M in range(m.nm)])
    for M in range(0, m.nm, 37):
        for k in range(4):
            if nbr[M, k] < 0:
                face = [v for i, v in enumerate(wl.macros[M]) if i != k]
                r = np.linalg.norm(wl.vertices[face], axis=1)
                assert np.ptp(r) < 1e-12 and (abs(r[0] - 0.55) < 1e-12 or abs(r[0] - 1.0) < 1e-12)


def test_shell_dof_count_formula(oracle_mod):
    # one icosahedral face at subdivision s and level L carries s*2^(L+1) P2 intervals per edge
    for level in (0, 1):
        wl = W.shell3d(level=level)
        m = mesh(oracle_mod, wl, level)
        e = 4 * 2 ** (level + 1)
        radial = 4 * 2 ** (level + 1) + 1
        assert m.N == (10 * e * e + 2) * radial


def _bey_children(T):
    x0, x1, x2, x3 = T
    mid = lambda a, b: tuple((np.array(a) + np.array(b)) / 2)
    x01, x02, x03, x12, x13, x23 = mid(x0, x1), mid(x0, x2), mid(x0, x3), mid(x1, x2), mid(x1, x3), mid(x2, x3)
    return [(x0, x01, x02, x03), (x01, x1, x12, x13), (x02, x12, x2, x23), (x03, x13, x23, x3),
            (x01, x02, x03, x13), (x01, x02, x12, x13), (x02, x03, x13, x23), (x02, x12, x13, x23)]


@pytest.mark.parametrize("level", [1, 2, 3])
def test_micro_simplices_follow_bey_refinement(oracle_mod, level):
    """The oracle's micro simplices (Kuhn/Freudenthal lattice) are the
    tetrahedra of Bey's recursive eight-child refinement of the Kuhn simplex."""
    wl = W.swirl3d()
    m = mesh(oracle_mod, wl, level)
    V = m.micro_simplices()  # n-lattice Kuhn coordinates
    n = 2 ** level
    assert V.shape[0] == n ** 3
    ours = {frozenset(tuple(int(c) for c in v) for v in simp) for simp in V}
    T = [((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (1.0, 1.0, 0.0), (1.0, 1.0, 1.0))]
    for _ in range(level):
        T = [c for t in T for c in _bey_children(t)]
    bey = {frozenset(tuple(int(round(c * n)) for c in v) for v in t) for t in T}
    assert ours == bey


@pytest.mark.parametrize("level", [1, 2, 3])
def test_micro_simplices_2d_red_refinement(oracle_mod, level):
    m = mesh(oracle_mod, W.rotation2d(), level)
    V = m.micro_simplices()
    n = 2 ** level
    assert V.shape[0] == n ** 2
    T = [((0.0, 0.0), (1.0, 0.0), (1.0, 1.0))]
    for _ in range(level):
        nxt = []
        for (a, b, c) in T:
            mid = lambda p, q: tuple((np.array(p) + np.array(q)) / 2)
            ab, ac, bc = mid(a, b), mid(a, c), mid(b, c)
            nxt += [(a, ab, ac), (ab, b, bc), (ac, bc, c), (ab, ac, bc)]
        T = nxt
    ref = {frozenset(tuple(int(round(x * n)) for x in v) for v in t) for t in T}
    ours = {frozenset(tuple(int(c) for c in v) for v in s) for s in V}
    assert ours == ref


def _micro_faces_on_macro_face(O, m, wl, M, k):
    """Physical micro faces (as frozensets of rounded points) of macro M lying on its face k."""
    v0, B, _, _ = m.geometry(M)
    n = m.n
    out = set()
    for simp in m.micro_simplices():
        for drop in range(m.dim + 1):
            face = [simp[a] for a in range(m.dim + 1) if a != drop]
            pts = []
            on = True
            for w in face:
                # Kuhn coordinates -> reference s -> barycentric of local vertex k
                w = np.asarray(w, dtype=np.float64) / n
                s = np.append(w[:-1] - w[1:], w[-1])
                lam = np.concatenate([[1.0 - s.sum()], s])
                if abs(lam[k]) > 1e-14:
                    on = False
                    break
                pts.append(tuple(np.round(v0 + B @ s, 12)))
            if on:
                out.add(frozenset(pts))
    return out


@pytest.mark.parametrize("wlf,level", [(W.swirl3d, 2), (W.rotation2d, 2)])
def test_micro_meshes_conform_across_macro_faces(oracle_mod, wlf, level):
    wl = wlf()
    m = mesh(oracle_mod, wl, level)
    for M in range(m.nm):
        nb = m.geometry(M)[3]
        for k in range(m.dim + 1):
            N2 = nb[k]
            if N2 < 0 or N2 < M:
                continue
            kk = [i for i in range(m.dim + 1) if m.geometry(N2)[3][i] == M][0]
            a = _micro_faces_on_macro_face(oracle_mod, m, wl, M, k)
            b = _micro_faces_on_macro_face(oracle_mod, m, wl, N2, kk)
            assert len(a) == m.n ** (m.dim - 1) and a == b
