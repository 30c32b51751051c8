"""ctypes wrapper of the CPU oracle (``mmoc_oracle.c``).

TEST INFRASTRUCTURE: only the test-suite, the smoke check and the benchmark's
CPU-baseline leg import this module.  The GPU library never does.

Arrays follow the oracle's C conventions: fields are structure-of-arrays
``[ncomp][N]`` float64 in the oracle's unique DoF order (macro-major, first
occurrence, nodes of a macro in lexicographic lattice order).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "mmoc_oracle.c"), os.path.join(HERE, "mlp_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction)."""
    srcs = [s for s in SRC if os.path.exists(s)]
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall",
               "-Wno-unused-function", "-shared", "-fPIC", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB)
                                              for s in SRC if os.path.exists(s)):
                build(force=True)
            L = C.CDLL(LIB)
            P = C.c_void_p
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int32)
            lp = C.POINTER(C.c_int64)
            L.orc_mesh_new.restype = P
            L.orc_mesh_new.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_int, ip, C.c_int]
            L.orc_mesh_new_order.restype = P
            L.orc_mesh_new_order.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_int, ip, C.c_int]
            L.orc_mesh_free.argtypes = [P]
            L.orc_num_dofs.restype = C.c_int64
            L.orc_num_dofs.argtypes = [P]
            L.orc_nodes_per_macro.restype = C.c_int64
            L.orc_nodes_per_macro.argtypes = [P]
            L.orc_lat_idx.restype = C.c_int64
            L.orc_lat_idx.argtypes = [C.c_int] * 4
            L.orc_macro_geometry.argtypes = [P, C.c_int, dp, dp, dp, ip]
            L.orc_plane.argtypes = [P, C.c_int, dp, dp]
            L.orc_dof_coords.argtypes = [P, dp]
            L.orc_dof_owner.argtypes = [P, ip, ip]
            L.orc_slot_uids.argtypes = [P, ip]
            L.orc_bary.argtypes = [P, C.c_int, dp, dp]
            L.orc_brute.restype = C.c_int
            L.orc_brute.argtypes = [P, dp]
            L.orc_walk.restype = C.c_int
            L.orc_walk.argtypes = [P, C.c_int, dp, C.c_int, C.POINTER(C.c_int)]
            L.orc_micro_simplex.argtypes = [P, C.c_int, dp, ip, dp]
            L.orc_eval.argtypes = [P, C.c_int, dp, C.c_int64, dp, ip, C.c_int, dp, ip, ip]
            L.orc_trace.restype = C.c_int
            L.orc_trace.argtypes = [P, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_int64, lp,
                                    dp, dp, lp]
            L.orc_trace_rk.restype = C.c_int
            L.orc_trace_rk.argtypes = [P, dp, dp, dp, C.c_double, C.c_int, C.c_int, dp, dp, dp, C.c_int,
                                       C.c_int64, lp, dp, dp, lp]
            L.orc_trace_span.restype = C.c_int
            L.orc_trace_span.argtypes = [P, C.POINTER(dp), C.c_int, dp, C.c_double, C.c_int, C.c_int, C.c_int64,
                                         lp, dp, dp, lp]
            L.orc_p2_mass_ref.argtypes = [C.c_int, dp]
            L.orc_micro_simplices.restype = C.c_int64
            L.orc_micro_simplices.argtypes = [P, ip, C.c_int64]
            L.orc_mass_quadform.restype = C.c_double
            L.orc_mass_quadform.argtypes = [P, dp, dp]
            L.orc_assemble.restype = C.c_int64
            L.orc_assemble.argtypes = [P, C.c_int, dp, dp, C.c_int64, lp, lp, dp, dp]
            L.orc_boundary_mask.argtypes = [P, C.POINTER(C.c_uint8)]
            if hasattr(L, "orc_mlp_forward"):
                _bind_mlp(L)
            _lib = L
        return _lib


def _bind_mlp(L):
    dp = C.POINTER(C.c_double)
    fp = C.POINTER(C.c_float)
    L.orc_mlp_nparams.restype = C.c_int64
    L.orc_mlp_nparams.argtypes = []
    L.orc_mlp_forward.argtypes = [dp, C.c_int64, dp, dp, C.c_int]
    L.orc_mlp_loss_grad.restype = C.c_double
    L.orc_mlp_loss_grad.argtypes = [dp, C.c_int64, dp, dp, dp, C.c_int]
    L.orc_bf16_round.restype = C.c_double
    L.orc_bf16_round.argtypes = [C.c_double]
    L.orc_gelu.restype = C.c_double
    L.orc_gelu.argtypes = [C.c_double]
    L.orc_adam_step.argtypes = [dp, dp, dp, dp, C.c_int64, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_int64]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


class Mesh:
    """Oracle view of a macro mesh refined to ``level``, with P2 (order 2)
    or P1 (order 1) elements."""

    def __init__(self, dim, level, vertices, macros, blend=0, order=2):
        L = lib()
        self.dim, self.level, self.blend, self.order = int(dim), int(level), int(blend), int(order)
        self.n = 1 << self.level
        self.m = self.order * self.n
        self.vertices = np.ascontiguousarray(vertices, dtype=np.float64)
        self.macros = np.ascontiguousarray(macros, dtype=np.int32)
        self._h = L.orc_mesh_new_order(self.dim, self.level, self.order, self.vertices.shape[0],
                                       _dp(self.vertices), self.macros.shape[0], _ip(self.macros), self.blend)
        if not self._h:
            raise ValueError("oracle rejected the mesh")
        self.N = int(L.orc_num_dofs(self._h))
        self.npm = int(L.orc_nodes_per_macro(self._h))
        self.nm = int(self.macros.shape[0])

    @classmethod
    def from_workload(cls, wl, level=None, order=2):
        return cls(wl.dim, wl.level if level is None else level, wl.vertices, wl.macros, wl.blend, order)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc_mesh_free(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def dof_coords(self):
        out = np.empty((self.dim, self.N))
        lib().orc_dof_coords(self._h, _dp(out))
        return out

    def dof_owner(self):
        own = np.empty(self.N, dtype=np.int32)
        lat = np.empty((self.N, 3), dtype=np.int32)
        lib().orc_dof_owner(self._h, _ip(own), _ip(lat))
        return own, lat

    def slot_uids(self):
        out = np.empty((self.nm, self.npm), dtype=np.int32)
        lib().orc_slot_uids(self._h, _ip(out))
        return out

    def geometry(self, M):
        d = self.dim
        v0, B, Bi = np.empty(d), np.empty((d, d)), np.empty((d, d))
        nb = np.empty(d + 1, dtype=np.int32)
        lib().orc_macro_geometry(self._h, int(M), _dp(v0), _dp(B), _dp(Bi), _ip(nb))
        return v0, B, Bi, nb

    def plane(self, M):
        n = np.empty(3)
        c = np.empty(1)
        lib().orc_plane(self._h, int(M), _dp(n), _dp(c))
        return n, float(c[0])

    def bary(self, M, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        lam = np.empty(self.dim + 1)
        lib().orc_bary(self._h, int(M), _dp(y), _dp(lam))
        return lam

    def brute(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        return int(lib().orc_brute(self._h, _dp(y)))

    def walk(self, M, y, max_hops=64):
        y = np.ascontiguousarray(y, dtype=np.float64)
        fl = C.c_int(0)
        r = lib().orc_walk(self._h, int(M), _dp(y), int(max_hops), C.byref(fl))
        return int(r), int(fl.value)

    def micro_simplex(self, M, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        V = np.zeros((4, 3), dtype=np.int32)
        mu = np.zeros(4)
        lib().orc_micro_simplex(self._h, int(M), _dp(y), _ip(V), _dp(mu))
        return V[: self.dim + 1, : self.dim], mu[: self.dim + 1]

    def micro_simplices(self):
        cnt = int(lib().orc_micro_simplices(self._h, None, 0))
        V = np.zeros((cnt, 4, 3), dtype=np.int32)
        lib().orc_micro_simplices(self._h, _ip(V), cnt)
        return V[:, : self.dim + 1, : self.dim]

    def eval(self, field, pts, start=None, max_hops=64):
        """Evaluate P2 field(s) ``[ncomp][N]`` (or ``[N]``) at points ``[npts][dim]``."""
        f = np.ascontiguousarray(np.atleast_2d(field), dtype=np.float64)
        ncomp = f.shape[0]
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, self.dim)
        npts = pts.shape[0]
        out = np.empty((npts, ncomp))
        mac = np.empty(npts, dtype=np.int32)
        fl = np.empty(npts, dtype=np.int32)
        st = None
        if start is not None:
            st = np.ascontiguousarray(np.broadcast_to(np.asarray(start, dtype=np.int32), (npts,)))
        lib().orc_eval(self._h, ncomp, _dp(f), npts, _dp(pts), _ip(st) if st is not None else None,
                       int(max_hops), _dp(out), _ip(mac), _ip(fl))
        return out, mac, fl

    def trace(self, u0, u1, c, dt, substeps, ids=None, max_hops=64, threads=1, tableau=None):
        """One advection step; returns (chat [n], X [dim][n], stats [4]).
        tableau = (A [s][s], b [s], c [s]) selects a general explicit RK
        method (orc_trace_rk); None is the classical RK4 (orc_trace)."""
        u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(self.dim, self.N)
        u1 = None if u1 is None else np.ascontiguousarray(u1, dtype=np.float64).reshape(self.dim, self.N)
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.N)
        if ids is None:
            ids_arr = np.arange(self.N, dtype=np.int64)
        else:
            ids_arr = np.ascontiguousarray(ids, dtype=np.int64)
        n = ids_arr.shape[0]
        chat = np.empty(n)
        X = np.empty((self.dim, n))
        stats = np.zeros(4, dtype=np.int64)
        L = lib()
        if tableau is not None:
            tA = np.ascontiguousarray(tableau[0], dtype=np.float64)
            tb = np.ascontiguousarray(tableau[1], dtype=np.float64)
            tc = np.ascontiguousarray(tableau[2], dtype=np.float64)
            ns = tb.shape[0]
            assert tA.shape == (ns, ns) and tc.shape == (ns,)

        def run(lo, hi, st):
            sub_ids = np.ascontiguousarray(ids_arr[lo:hi])
            ch = np.empty(hi - lo)
            Xs = np.empty((self.dim, hi - lo))
            if tableau is None:
                r = L.orc_trace(self._h, _dp(u0), _dp(u1) if u1 is not None else None, _dp(c),
                                float(dt), int(substeps), int(max_hops), hi - lo, _lp(sub_ids),
                                _dp(ch), _dp(Xs), _lp(st))
            else:
                r = L.orc_trace_rk(self._h, _dp(u0), _dp(u1) if u1 is not None else None, _dp(c),
                                   float(dt), int(substeps), ns, _dp(tA), _dp(tb), _dp(tc), int(max_hops),
                                   hi - lo, _lp(sub_ids), _dp(ch), _dp(Xs), _lp(st))
            if r != 0:
                raise ValueError("oracle trace rejected its arguments")
            chat[lo:hi] = ch
            X[:, lo:hi] = Xs

        if threads <= 1 or n < 2 * threads:
            run(0, n, stats)
        else:
            bounds = np.linspace(0, n, threads + 1).astype(np.int64)
            sts = [np.zeros(4, dtype=np.int64) for _ in range(threads)]
            ths = [threading.Thread(target=run, args=(int(bounds[k]), int(bounds[k + 1]), sts[k]))
                   for k in range(threads)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            stats = sum(sts)
        return chat, X, stats

    def trace_span(self, levels, c, tau, substeps, ids=None, max_hops=64, threads=1):
        """Trace across len(levels) - 1 time steps of length tau: levels[l] is
        the velocity ([dim][N]) at t_0 + l tau, linear in time on each step;
        RK4 with `substeps` sub-steps per step; c is known at t_0.  Returns
        (chat [n], X [dim][n], stats [4])."""
        Us = [np.ascontiguousarray(u, dtype=np.float64).reshape(self.dim, self.N) for u in levels]
        n_int = len(Us) - 1
        arr = (C.POINTER(C.c_double) * len(Us))(*[_dp(u) for u in Us])
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.N)
        ids_arr = np.arange(self.N, dtype=np.int64) if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
        n = ids_arr.shape[0]
        chat = np.empty(n)
        X = np.empty((self.dim, n))
        stats = np.zeros(4, dtype=np.int64)
        L = lib()

        def run(lo, hi, st):
            sub = np.ascontiguousarray(ids_arr[lo:hi])
            ch = np.empty(hi - lo)
            Xs = np.empty((self.dim, hi - lo))
            if L.orc_trace_span(self._h, arr, n_int, _dp(c), float(tau), int(substeps), int(max_hops), hi - lo,
                                _lp(sub), _dp(ch), _dp(Xs), _lp(st)) != 0:
                raise ValueError("oracle trace_span rejected its arguments")
            chat[lo:hi] = ch
            X[:, lo:hi] = Xs

        if threads <= 1 or n < 2 * threads:
            run(0, n, stats)
        else:
            bounds = np.linspace(0, n, threads + 1).astype(np.int64)
            sts = [np.zeros(4, dtype=np.int64) for _ in range(threads)]
            ths = [threading.Thread(target=run, args=(int(bounds[k]), int(bounds[k + 1]), sts[k]))
                   for k in range(threads)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            stats = sum(sts)
        return chat, X, stats

    def mass_quadform(self, a, b):
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        return float(lib().orc_mass_quadform(self._h, _dp(a), _dp(b)))


    # ------------------------------------------------ diffusion (Sec. 2.2)

    def assemble(self, rule=None):
        """Mass and stiffness matrices (scipy CSR, N x N) of the mesh's
        elements, integrated with ``rule`` = (points [nq][d], weights [nq])
        on the reference simplex; default: the collapsed Gauss rule with 4
        points per direction (exact to degree 6 in 2D, 5 in 3D)."""
        import scipy.sparse as sp
        qp, qw = simplex_rule(self.dim, 4) if rule is None else rule
        qp = np.ascontiguousarray(qp, dtype=np.float64)
        qw = np.ascontiguousarray(qw, dtype=np.float64)
        L = lib()
        cnt = int(L.orc_assemble(self._h, qw.shape[0], _dp(qp), _dp(qw), 0, None, None, None, None))
        rows = np.empty(cnt, dtype=np.int64)
        cols = np.empty(cnt, dtype=np.int64)
        mv = np.empty(cnt)
        av = np.empty(cnt)
        L.orc_assemble(self._h, qw.shape[0], _dp(qp), _dp(qw), cnt, _lp(rows), _lp(cols), _dp(mv), _dp(av))
        Mm = sp.coo_matrix((mv, (rows, cols)), shape=(self.N, self.N)).tocsr()
        Am = sp.coo_matrix((av, (rows, cols)), shape=(self.N, self.N)).tocsr()
        return Mm, Am

    def boundary_mask(self):
        out = np.empty(self.N, dtype=np.uint8)
        lib().orc_boundary_mask(self._h, out.ctypes.data_as(C.POINTER(C.c_uint8)))
        return out.astype(bool)


def simplex_rule(dim, n):
    """Collapsed (conical product) Gauss rule on the reference simplex
    {xi >= 0, sum xi <= 1}: Gauss-Legendre nodes u, v (, w) on [0, 1] mapped
    by xi = (u, v (1 - u)) in 2D and (u, v (1 - u), w (1 - u)(1 - v)) in 3D,
    the weights multiplied by the map's Jacobian (1 - u), resp.
    (1 - u)^2 (1 - v).  The Jacobian raises the degree in u by dim - 1, so
    the rule is exact for polynomials of total degree 2n - dim."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = (g + 1.0) / 2.0
    w = w / 2.0
    pts, wts = [], []
    if dim == 2:
        for i in range(n):
            for j in range(n):
                u, v = g[i], g[j]
                pts.append((u, v * (1 - u)))
                wts.append(w[i] * w[j] * (1 - u))
    else:
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    u, v, t = g[i], g[j], g[k]
                    pts.append((u, v * (1 - u), t * (1 - u) * (1 - v)))
                    wts.append(w[i] * w[j] * w[k] * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def diffusion_solve(M, A, c_hat, tau, kappa, theta=1.0, q0=None, q1=None, mask=None, g=None):
    """One diffusion step of the Theta-method (Sec. 2.2, eq. linear-system):
    (M + tau Theta kappa A) c = (M - tau (1 - Theta) kappa A) c_hat
                                + tau (Theta q1 + (1 - Theta) q0),
    q0 / q1 the load vectors (q(t_n), v_i) and (q(t_{n+1}), v_i) (None:
    zero).  Dirichlet DoFs (mask True) take the values g; their rows are the
    identity and their known values move to the right-hand side of the other
    rows.  Solved exactly by a sparse direct factorisation."""
    import scipy.sparse.linalg as sla
    N = M.shape[0]
    E = (M + (tau * theta * kappa) * A).tocsr()
    rhs = (M - (tau * (1.0 - theta) * kappa) * A) @ c_hat
    if q0 is not None or q1 is not None:
        q0 = np.zeros(N) if q0 is None else q0
        q1 = np.zeros(N) if q1 is None else q1
        rhs = rhs + tau * (theta * q1 + (1.0 - theta) * q0)
    if mask is None or not mask.any():
        return sla.spsolve(E.tocsc(), rhs)
    free = ~mask
    x = np.zeros(N)
    x[mask] = g[mask]
    rf = rhs[free] - E[free][:, mask] @ g[mask]
    x[free] = sla.spsolve(E[free][:, free].tocsc(), rf)
    return x


def p2_mass_ref(dim):
    nb = (dim + 1) * (dim + 2) // 2
    out = np.empty((nb, nb))
    lib().orc_p2_mass_ref(int(dim), _dp(out))
    return out


def lat_idx(dim, I, J, K=0):
    return int(lib().orc_lat_idx(int(dim), int(I), int(J), int(K)))


# ------------------------------------------------------------- surrogate MLP

def mlp_nparams():
    return int(lib().orc_mlp_nparams())


def mlp_forward(params, x, bf16=False):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 4)
    y = np.empty((x.shape[0], 3))
    lib().orc_mlp_forward(_dp(p), x.shape[0], _dp(x), _dp(y), int(bool(bf16)))
    return y


def mlp_loss_grad(params, x, t, bf16=False):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 4)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, 3)
    g = np.empty(p.shape[0])
    loss = lib().orc_mlp_loss_grad(_dp(p), x.shape[0], _dp(x), _dp(t), _dp(g), int(bool(bf16)))
    return float(loss), g


def adam_step(p, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam_step(_dp(p), _dp(g), _dp(m), _dp(v), p.shape[0], float(lr), float(b1), float(b2), float(eps),
                        int(t))


def bf16_round(v):
    return float(lib().orc_bf16_round(float(v)))


def gelu(v):
    return float(lib().orc_gelu(float(v)))
