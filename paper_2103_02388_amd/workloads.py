"""Seeded synthetic workloads: coarse macro meshes and analytic fields.

This module only produces *inputs*: the coarse mesh (vertex coordinates and
macro-element vertex lists, the way a mesh file would hand them over) and
closed-form velocity / scalar functions that a caller samples at whatever
points it likes.  It holds none of the method's arithmetic: no refinement
lattice, no degree-of-freedom enumeration, no interpolation, no point
location and no time integration.  Both the test oracle and the GPU library
consume what it returns, each through its own code.

The shapes follow the paper's benchmarks (Sec. 3 and 4):

* ``square2``  -- unit square split into two triangles along (0,0)-(1,1)
  (Sec. 3.2: squares divided into two triangles), used with the rotation
  field u = (0.5 - y, x - 0.5).
* ``cube6``    -- unit cube split into the six Kuhn tetrahedra, used with the
  LeVeque swirl field of Sec. 3.3 and with the rising-plume field.
* ``annulus``  -- annulus r in [0.5, 1.5] of 6 x 2 quadrilateral cells cut
  into triangles (Sec. 4, advection-diffusion), with radial blending.
* ``shell``    -- thick spherical shell: a subdivided icosahedron extruded into
  radial layers, each prism split into three tetrahedra (Sec. 5.3 uses a
  shell of tetrahedral macro cells projected onto the sphere).

Every random draw is seeded with ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch

# ---------------------------------------------------------------------------
# coarse meshes
# ---------------------------------------------------------------------------


def square2():
    """Unit square as two triangles sharing the diagonal (0,0)-(1,1).

    Local vertex orders are chosen so that the shared edge has the same
    relative order in both triangles: T_A = [(0,0),(1,0),(1,1)],
    T_B = [(0,0),(0,1),(1,1)].
    """
    v = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    m = np.array([[0, 1, 2], [0, 3, 2]], dtype=np.int32)
    return v, m


def cube6():
    """Unit cube as the six Kuhn tetrahedra [0, e_a, e_a + e_b, (1,1,1)].

    Vertex id of corner (x, y, z) is x + 2y + 4z.  Macros are listed in
    lexicographic order of the axis permutation (a, b, c).
    """
    v = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=np.float64)
    macros = []
    for a, b, _c in itertools.permutations(range(3)):
        ea = 1 << a
        eb = 1 << b
        macros.append([0, ea, ea | eb, 7])
    return v, np.array(macros, dtype=np.int32)


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
         (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = np.array(v, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def shell(subdiv: int = 4, layers: int = 4, r_min: float = 0.55, r_max: float = 1.0):
    """Thick spherical shell r in [r_min, r_max] as tetrahedral macro cells.

    Each icosahedron face is split into ``subdiv**2`` triangles whose corners
    are pushed onto the unit sphere; the resulting ``20*subdiv**2`` flat
    triangles are extruded over ``layers`` uniform radial layers, and each
    prism is cut into three tetrahedra.  Vertex id = layer * n_dir + dir.
    Every quad side face of a prism is cut along the diagonal through its
    smallest vertex id, which makes neighbouring prisms agree; each
    tetrahedron lists its vertices in ascending id, so that every shared face
    carries the same relative vertex order on both sides.  Vertices lie on the
    spheres r_k: the flat (computational) shell is mapped onto the curved one
    by the caller's blending map.
    """
    iv, faces = _icosahedron()
    dirs: list = []
    key: dict = {}

    def vid(p):
        q = p / np.linalg.norm(p)
        k = tuple(np.round(q * 1e9).astype(np.int64))
        if k not in key:
            key[k] = len(dirs)
            dirs.append(q)
        return key[k]

    tris = []
    for (a, b, c) in faces:
        A, B, C = iv[a], iv[b], iv[c]
        grid = {}
        for i in range(subdiv + 1):
            for j in range(subdiv + 1 - i):
                grid[(i, j)] = vid(A + (B - A) * (i / subdiv) + (C - A) * (j / subdiv))
        for i in range(subdiv):
            for j in range(subdiv - i):
                tris.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if j + i + 1 < subdiv:
                    tris.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    nd = len(dirs)
    dirs = np.array(dirs)
    radii = np.linspace(r_min, r_max, layers + 1)
    verts = np.concatenate([dirs * r for r in radii], axis=0)
    macros = []
    for k in range(layers):
        for t in tris:
            # order the three directions by descending id: the staircase
            # (c,b,a,c'), (b,a,c',b'), (a,c',b',a') then cuts every quad
            # along the diagonal through its smallest id (a bottom vertex)
            c, b, a = sorted(t, reverse=True)
            bot = lambda d: k * nd + d
            top = lambda d: (k + 1) * nd + d
            for tet in ((bot(c), bot(b), bot(a), top(c)),
                        (bot(b), bot(a), top(c), top(b)),
                        (bot(a), top(c), top(b), top(a))):
                macros.append(sorted(tet))
    return verts, np.array(macros, dtype=np.int32)


def annulus(n_ang: int = 6, n_rad: int = 2, r_min: float = 0.5, r_max: float = 1.5):
    """Annulus r in [r_min, r_max] as triangles (Sec. 4: a coarse triangular
    mesh refined uniformly and projected onto the annulus).

    ``n_ang`` sectors times ``n_rad`` radial layers of quadrilateral cells,
    each cut along the diagonal through its smallest vertex id; vertex id =
    layer * n_ang + sector, vertex (r_j cos phi_k, r_j sin phi_k) with
    phi_k = 2 pi k / n_ang.  Each triangle lists its vertices in ascending
    id.  The flat mesh is mapped onto the round annulus by the caller's
    blending map.
    """
    radii = np.linspace(r_min, r_max, n_rad + 1)
    ang = 2.0 * np.pi * np.arange(n_ang) / n_ang
    verts = np.array([[r * math.cos(a), r * math.sin(a)] for r in radii for a in ang])
    tris = []
    for j in range(n_rad):
        for k in range(n_ang):
            a, b = j * n_ang + k, j * n_ang + (k + 1) % n_ang
            c, d = a + n_ang, b + n_ang
            lo = min(a, b, c, d)
            opp = {a: d, b: c, c: b, d: a}[lo]  # the diagonal through the smallest id
            rest = [v for v in (a, b, c, d) if v not in (lo, opp)]
            for v in rest:
                tris.append(sorted((lo, opp, v)))
    return verts, np.array(tris, dtype=np.int32)


# ---------------------------------------------------------------------------
# analytic fields (torch, float64, any device)
# ---------------------------------------------------------------------------


def rotation_velocity(x: torch.Tensor, t: float = 0.0) -> torch.Tensor:
    """Solid-body rotation about (0.5, 0.5): u = (0.5 - y, x - 0.5) (Sec. 3.2)."""
    return torch.stack([0.5 - x[:, 1], x[:, 0] - 0.5], dim=1)


def _r(x, centre, r0):
    c = torch.tensor(centre, dtype=x.dtype, device=x.device)
    return torch.linalg.norm(x - c, dim=1) / r0


def hill(x: torch.Tensor) -> torch.Tensor:
    """Smooth hill of Sec. 3.2: (1 + cos(pi r)) / 4 inside r <= 1, centre (0.25, 0.5)."""
    r = _r(x, (0.25, 0.5), 0.15)
    return torch.where(r <= 1.0, 0.25 * (1.0 + torch.cos(math.pi * r)), torch.zeros_like(r))


def cone(x: torch.Tensor) -> torch.Tensor:
    """Cone of Sec. 3.2: 1 - r inside r <= 1, centre (0.5, 0.25)."""
    r = _r(x, (0.5, 0.25), 0.15)
    return torch.where(r <= 1.0, 1.0 - r, torch.zeros_like(r))


def slotted_cylinder(x: torch.Tensor) -> torch.Tensor:
    """Slotted cylinder of Sec. 3.2, centre (0.5, 0.75), radius 0.15.

    The printed condition lists three clauses separated by commas; read as a
    conjunction it leaves only a cap, so the slot is taken as
    ``|x1 - 0.5| >= 0.025 or x2 >= 0.85`` inside the disc (the classical shape).
    """
    r = _r(x, (0.5, 0.75), 0.15)
    keep = (torch.abs(x[:, 0] - 0.5) >= 0.025) | (x[:, 1] >= 0.85)
    return torch.where((r <= 1.0) & keep, torch.ones_like(r), torch.zeros_like(r))


def gaussian(x: torch.Tensor, centre, sigma: float) -> torch.Tensor:
    c = torch.tensor(centre, dtype=x.dtype, device=x.device)
    return torch.exp(-((x - c) ** 2).sum(dim=1) / (2.0 * sigma * sigma))


def cone_gaussian_and_slotted(x: torch.Tensor) -> torch.Tensor:
    """Scalar of the 2D rotation workload: Gaussian (sigma 0.05) at the cone
    centre (0.5, 0.25) plus the slotted cylinder."""
    return gaussian(x, (0.5, 0.25), 0.05) + slotted_cylinder(x)


SWIRL_T = 1.5


def swirl_velocity(x: torch.Tensor, t: float) -> torch.Tensor:
    """LeVeque's 3D deformation field of Sec. 3.3 with g(t) = cos(pi t / T), T = 1.5.

    The first component carries the factor 2 that makes the field
    divergence-free; all normal components vanish on the cube faces.
    """
    g = math.cos(math.pi * t / SWIRL_T)
    px, py, pz = (math.pi * x[:, i] for i in range(3))
    s2x, s2y, s2z = torch.sin(px) ** 2, torch.sin(py) ** 2, torch.sin(pz) ** 2
    sx, sy, sz = torch.sin(2 * px), torch.sin(2 * py), torch.sin(2 * pz)
    return torch.stack([2.0 * s2x * sy * sz * g, -sx * s2y * sz * g, -sx * sy * s2z * g], dim=1)


def circular_velocity(x: torch.Tensor, t: float = 0.0) -> torch.Tensor:
    """Rotation about the origin, u = (-x2, x1) (Sec. 4, annulus)."""
    return torch.stack([-x[:, 1], x[:, 0]], dim=1)


class MovingGaussian:
    """Smeared Gaussian hill of the advection-diffusion benchmark (Sec. 4):
    c(x, t) = exp(-|x - xhat(t)|^2 / (4 t kappa)) / (4 pi t kappa), the
    centre xhat(t) = (xb1 cos t - xb2 sin t, -xb1 sin t + xb2 cos t) with
    xb = (0, 1), which the field u = (-x2, x1) carries.  The run starts at
    t0 = 2 pi 1e-3 / kappa, so that the initial shape does not depend on
    kappa, and ends after one revolution at t0 + 2 pi."""

    def __init__(self, kappa: float, xbar=(0.0, 1.0)):
        self.kappa = float(kappa)
        self.xbar = (float(xbar[0]), float(xbar[1]))
        self.t0 = 2.0 * math.pi * 1e-3 / self.kappa

    def centre(self, t: float):
        x1, x2 = self.xbar
        return (x1 * math.cos(t) - x2 * math.sin(t), -x1 * math.sin(t) + x2 * math.cos(t))

    def __call__(self, x: torch.Tensor, t: float) -> torch.Tensor:
        c1, c2 = self.centre(t)
        r2 = (x[:, 0] - c1) ** 2 + (x[:, 1] - c2) ** 2
        s = 4.0 * t * self.kappa
        return torch.exp(-r2 / s) / (math.pi * s)


def two_blobs(x: torch.Tensor) -> torch.Tensor:
    """Two Gaussian blobs (sigma 0.1) at (0.35,0.5,0.5) and (0.65,0.5,0.5)."""
    return gaussian(x, (0.35, 0.5, 0.5), 0.1) + gaussian(x, (0.65, 0.5, 0.5), 0.1)


class PlumeField:
    """Sum of eight rising-plume modes in the unit cube (seed 6).

    Mode k has vector potential A_k = B * G_k * (-(y - y_k), x - x_k, 0) with
    B = 64 x(1-x) y(1-y) z(1-z) (vanishes on the boundary, so u.n = 0) and
    G_k a Gaussian of width 0.12 centred at (x_k, y_k, z_k).  The velocity is
    u = sum_k w_k(t) a_k curl(A_k), with w_k(t) = exp(-((t - t_k)/D)^2),
    t_k = (k - 1/2) T/8, D = T/8, T = 200 steps.  Time enters only through
    t / T, so the field can be sampled at step indices before dt is known.
    """

    def __init__(self, seed: int = 6, n_modes: int = 8, width: float = 0.12):
        rng = np.random.default_rng(seed)
        self.xy = rng.uniform(0.25, 0.75, size=(n_modes, 2))
        self.z = rng.uniform(0.15, 0.45, size=n_modes)
        self.a = rng.uniform(0.5, 2.0, size=n_modes)
        self.s = width
        self.n = n_modes

    def weight(self, k: int, phase: float) -> float:
        tk = (k + 0.5) / self.n
        return math.exp(-(((phase - tk) * self.n) ** 2))

    def velocity_phase(self, x: torch.Tensor, phase: float) -> torch.Tensor:
        X0, Y0, Z0 = x[:, 0], x[:, 1], x[:, 2]
        B = 64.0 * X0 * (1 - X0) * Y0 * (1 - Y0) * Z0 * (1 - Z0)
        Bx = 64.0 * (1 - 2 * X0) * Y0 * (1 - Y0) * Z0 * (1 - Z0)
        By = 64.0 * X0 * (1 - X0) * (1 - 2 * Y0) * Z0 * (1 - Z0)
        Bz = 64.0 * X0 * (1 - X0) * Y0 * (1 - Y0) * (1 - 2 * Z0)
        u = torch.zeros_like(x)
        inv_s2 = 1.0 / (self.s * self.s)
        for k in range(self.n):
            w = self.weight(k, phase) * self.a[k]
            if w < 1e-300:
                continue
            X = X0 - self.xy[k, 0]
            Y = Y0 - self.xy[k, 1]
            Z = Z0 - self.z[k]
            G = torch.exp(-(X * X + Y * Y + Z * Z) * (0.5 * inv_s2))
            phi = B * G
            phix = Bx * G - phi * X * inv_s2
            phiy = By * G - phi * Y * inv_s2
            phiz = Bz * G - phi * Z * inv_s2
            # curl of phi * (-Y, X, 0)
            u[:, 0] += w * (-X * phiz)
            u[:, 1] += w * (-Y * phiz)
            u[:, 2] += w * (2.0 * phi + X * phix + Y * phiy)
        return u


def exp_profile_z(x: torch.Tensor) -> torch.Tensor:
    """exp(-10 z): the exponential profile of the mantle run's initial temperature (Sec. 5.3)."""
    return torch.exp(-10.0 * x[:, 2])


# --- spherical-shell modes --------------------------------------------------


def _real_sph_harm(l: int, m: int, x: torch.Tensor) -> torch.Tensor:
    """Real orthonormal spherical harmonic Y_lm at the direction of x (rows).

    Written in Cartesian form so that it is smooth everywhere off the origin
    (no angles): with u = x/|x|, P_l^|m|(u_z) = (1 - u_z^2)^(|m|/2) Q(u_z) for a
    polynomial Q, and (1 - u_z^2)^(|m|/2) (cos |m| phi, sin |m| phi) are the real
    and imaginary parts of (u_x + i u_y)^|m|.  No Condon-Shortley phase.
    """
    am = abs(m)
    r = torch.linalg.norm(x, dim=1)
    ux, uy, uz = x[:, 0] / r, x[:, 1] / r, x[:, 2] / r
    # Q_am^am = (2am - 1)!!, Q_{am+1}^am = (2am + 1) u_z Q_am^am, then upward in l
    dfact = 1.0
    for k in range(1, 2 * am, 2):
        dfact *= k
    q0 = torch.full_like(uz, dfact)
    if l == am:
        q = q0
    else:
        q1 = uz * (2 * am + 1) * q0
        for ll in range(am + 2, l + 1):
            q0, q1 = q1, ((2 * ll - 1) * uz * q1 - (ll + am - 1) * q0) / (ll - am)
        q = q1
    re, im = torch.ones_like(ux), torch.zeros_like(ux)
    for _ in range(am):
        re, im = re * ux - im * uy, re * uy + im * ux
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    if m > 0:
        return math.sqrt(2.0) * norm * q * re
    if m < 0:
        return math.sqrt(2.0) * norm * q * im
    return norm * q


class ShellModes:
    """Seeded sum of toroidal and poloidal modes in r in [r_min, r_max] (seed 3).

    Toroidal: u = grad(psi) x x.  Poloidal: u = curl(grad(chi) x x).  With
    psi, chi = sin(pi rho) Y_lm, rho = (r - r_min)/(r_max - r_min), the radial
    component vanishes at both radii.  Derivatives are taken by float64
    autograd.  The field is rescaled by ``scale`` (set by the caller so that
    the largest nodal speed is 1).
    """

    def __init__(self, seed: int = 3, n_tor: int = 8, n_pol: int = 8, lmax: int = 8,
                 r_min: float = 0.55, r_max: float = 1.0):
        rng = np.random.default_rng(seed)
        self.modes = []
        for kind, cnt in (("tor", n_tor), ("pol", n_pol)):
            for _ in range(cnt):
                l = int(rng.integers(1, lmax + 1))
                m = int(rng.integers(-l, l + 1))
                a = float(rng.uniform(-1.0, 1.0))
                self.modes.append((kind, l, m, a))
        self.r_min, self.r_max = r_min, r_max
        self.scale = 1.0

    def _pot(self, x, kind):
        r = torch.linalg.norm(x, dim=1)
        rho = (r - self.r_min) / (self.r_max - self.r_min)
        radial = torch.sin(math.pi * rho)
        out = torch.zeros_like(r)
        for (k, l, m, a) in self.modes:
            if k == kind:
                out = out + a * radial * _real_sph_harm(l, m, x)
        return out

    def normalise(self, n_points: int = 1 << 18, seed: int = 30):
        """Scales the field so that its largest speed over a seeded uniform
        sample of the shell is 1."""
        rng = np.random.default_rng(seed)
        d = rng.normal(size=(n_points, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = (self.r_min ** 3 + rng.uniform(size=(n_points, 1)) * (self.r_max ** 3 - self.r_min ** 3)) ** (1 / 3)
        self.scale = 1.0
        u = self.velocity(torch.from_numpy(d * r))
        self.scale = 1.0 / float(torch.linalg.norm(u, dim=1).max())
        return self

    def velocity(self, x: torch.Tensor, t: float = 0.0, batch: int = 1 << 21) -> torch.Tensor:
        outs = []
        for s in range(0, x.shape[0], batch):
            xb = x[s:s + batch].detach().clone().requires_grad_(True)
            with torch.enable_grad():
                psi = self._pot(xb, "tor")
                (gpsi,) = torch.autograd.grad(psi.sum(), xb)
                u_tor = torch.linalg.cross(gpsi, xb.detach())
                chi = self._pot(xb, "pol")
                (gchi,) = torch.autograd.grad(chi.sum(), xb, create_graph=True)
                v = torch.linalg.cross(gchi, xb)
                # curl v
                rows = []
                for i in range(3):
                    (gi,) = torch.autograd.grad(v[:, i].sum(), xb, retain_graph=True)
                    rows.append(gi)
                J = torch.stack(rows, dim=1)  # J[:, i, j] = d v_i / d x_j
                curl = torch.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0],
                                    J[:, 1, 0] - J[:, 0, 1]], dim=1)
            outs.append(((u_tor + curl) * self.scale).detach())
        return torch.cat(outs, dim=0)


def shell_step_scalar(x: torch.Tensor, seed: int = 4, r_step: float = 0.8) -> torch.Tensor:
    """Step at r = 0.8 plus 1% uniform noise drawn per node in the given order."""
    r = torch.linalg.norm(x, dim=1)
    rng = np.random.default_rng(seed)
    xi = torch.from_numpy(rng.uniform(-1.0, 1.0, size=x.shape[0])).to(x.device, x.dtype)
    return (r < r_step).to(x.dtype) + 0.01 * xi


# ---------------------------------------------------------------------------
# workload records
# ---------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    dim: int
    level: int
    vertices: np.ndarray
    macros: np.ndarray
    blend: int                # 0: identity, 1: radial blending (shell, annulus)
    dt: float
    substeps: int
    steps: int
    stationary: bool
    velocity: Callable        # (x [N,d] float64 tensor, t) -> [N,d]
    scalar0: Callable         # (x [N,d]) -> [N]
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_macros(self) -> int:
        return int(self.macros.shape[0])


def rotation2d(level: int = 6) -> Workload:
    v, m = square2()
    return Workload("rotation2d", 2, level, v, m, 0, 1.0 / 200.0, 4, 1, True,
                    rotation_velocity, cone_gaussian_and_slotted,
                    "unit square, 2 macro triangles, solid-body rotation; "
                    "Gaussian (sigma 0.05) + slotted cylinder")


def swirl3d(level: int = 5, steps: int = 50) -> Workload:
    v, m = cube6()
    return Workload("swirl3d", 3, level, v, m, 0, SWIRL_T / 20.0, 4, steps, False,
                    swirl_velocity, two_blobs,
                    "unit cube, 6 Kuhn macro tets, LeVeque swirl, cos(pi t/T), T=1.5; two Gaussian blobs")


def plume3d(level: int = 7, steps: int = 200, umax_level: int = 5) -> Workload:
    """Rising-plume cube workload; dt = 5 * (1/128) / U_max, with U_max the
    largest speed over a uniform (2^umax_level + 1)^3 grid and 201 time levels."""
    v, m = cube6()
    pf = PlumeField()
    g = torch.linspace(0.0, 1.0, 2 ** umax_level + 1, dtype=torch.float64)
    X = torch.stack(torch.meshgrid(g, g, g, indexing="ij"), dim=-1).reshape(-1, 3)
    umax = 0.0
    for n in range(steps + 1):
        umax = max(umax, float(torch.linalg.norm(pf.velocity_phase(X, n / steps), dim=1).max()))
    dt = 5.0 * (1.0 / 128.0) / umax
    T = steps * dt
    vel = lambda x, t: pf.velocity_phase(x, t / T)
    return Workload("plume3d", 3, level, v, m, 0, dt, 4, steps, False, vel, exp_profile_z,
                    "unit cube, 6 Kuhn macro tets, 8 rising-plume modes (seed 6); exp(-10 z)",
                    extra={"umax": umax, "T": T})


def shell3d(level: int = 5, subdiv: int = 4, layers: int = 4) -> Workload:
    """Spherical shell r in [0.55, 1]; stationary seeded toroidal/poloidal flow.

    dt = 5 h_min / max|u| with h_min the radial micro-edge length; the caller
    normalises the field so that the largest nodal speed is 1 (``scale``).
    """
    v, m = shell(subdiv, layers)
    sm = ShellModes().normalise()
    h_min = (1.0 - 0.55) / layers / (2 ** level)
    return Workload("shell3d", 3, level, v, m, 1, 5.0 * h_min, 4, 1, True,
                    sm.velocity, shell_step_scalar,
                    "thick spherical shell r in [0.55,1], icosahedral macro mesh; "
                    "16 seeded toroidal/poloidal modes; step at r=0.8 + 1% noise",
                    extra={"modes": sm, "h_min": h_min})


ANNULUS_STEPS = 63  # tau = 2 pi / 63, about 0.1 (Sec. 4, Table 4)


def annulus2d(level: int = 4, kappa: float = 1e-3) -> Workload:
    """Advection-diffusion on the blended annulus r in [0.5, 1.5] (Sec. 4,
    Table 4): 6 sectors x 2 layers of macro triangles (levels 4, 5, 6 give
    the printed 12,480 / 49,536 / 197,376 P2 DoFs), u = (-x2, x1), the
    moving Gaussian hill, one revolution in 63 steps of tau = 2 pi / 63, one
    RK4 step per tau (b = 1: the field is interpolated every step)."""
    v, m = annulus()
    hill = MovingGaussian(kappa)
    return Workload("annulus2d", 2, level, v, m, 1, 2.0 * math.pi / ANNULUS_STEPS, 1, ANNULUS_STEPS, True,
                    circular_velocity, lambda x: hill(x, hill.t0),
                    "annulus r in [0.5, 1.5], 6x2 macro triangles, radial blending; rotation (-x2, x1); "
                    "Gaussian hill, kappa %g" % kappa,
                    extra={"kappa": kappa, "hill": hill})


CONFIGS = {
    "rotation2d": rotation2d,
    "swirl3d": swirl3d,
    "shell3d": shell3d,
    "plume3d": plume3d,
    "annulus2d": annulus2d,
}
