"""Python binding of the C-ABI in ``include/mmoc.h`` (``libmmoc.so``).

Argument marshalling only: torch tensors are passed as device pointers and
torch's current HIP stream as the stream handle; every step of the method
runs in the library's HIP kernels.  The functions keep the C names; each
raises :class:`MMOCError` with the library's reason when the call fails.
Importing this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from .build import LIB

MMOC_FP64 = 0
MMOC_FP32_MIXED = 1
MMOC_FP32_FIELDS = 2
MMOC_BLEND_NONE = 0
MMOC_BLEND_SHELL_RADIAL = 1
MMOC_MAT_MASS = 0
MMOC_MAT_STIFFNESS = 1

STATUS = {0: "MMOC_OK", -1: "MMOC_E_ARG", -2: "MMOC_E_MESH", -3: "MMOC_E_STATE", -4: "MMOC_E_HIP",
          -5: "MMOC_E_NOMEM", -6: "MMOC_E_UNSUPPORTED"}

EXPORTED = [
    "mmoc_default_options", "mmoc_create", "mmoc_set_stream", "mmoc_upload_mesh", "mmoc_num_dofs",
    "mmoc_dof_coords", "mmoc_set_velocity", "mmoc_set_stationary", "mmoc_swap_velocity_levels",
    "mmoc_set_scalar", "mmoc_trace_step", "mmoc_get_stats", "mmoc_reset_stats", "mmoc_mlp_nparams",
    "mmoc_mlp_configure", "mmoc_mlp_set_predictor", "mmoc_mlp_record", "mmoc_mlp_train", "mmoc_mlp_get_weights",
    "mmoc_mlp_set_weights", "mmoc_mlp_infer", "mmoc_trace_step_surrogate", "mmoc_last_error",
    "mmoc_destroy", "mmoc_mlp_forward", "mmoc_mlp_loss_grad", "mmoc_mass_inner", "mmoc_mass_inner_noalloc", "mmoc_field_range",
    "mmoc_lookback_run", "mmoc_set_rk_tableau", "mmoc_cfl_time_step", "mmoc_set_level_count", "mmoc_trace_span",
    "mmoc_fe_assemble", "mmoc_fe_export", "mmoc_fe_apply", "mmoc_boundary_mask", "mmoc_diffusion_step",
    "mmoc_set_fields", "mmoc_use_last_chat",
]


class MMOCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class mmoc_options(C.Structure):
    _fields_ = [("eps_in", C.c_double), ("eps32_macro", C.c_float), ("eps32_micro", C.c_float),
                ("max_hops", C.c_int), ("order", C.c_int), ("elem_cache", C.c_int), ("keep_chat", C.c_int),
                ("reserved", C.c_int)]


class mmoc_stats(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_outside", C.c_int64), ("n_multi_hop", C.c_int64),
                ("n_bruteforce", C.c_int64), ("n_tieband", C.c_int64), ("n_nan", C.c_int64),
                ("n_checked", C.c_int64), ("n_fallback", C.c_int64), ("max_check_residual", C.c_double),
                ("n_cache_lookups", C.c_int64), ("n_cache_hits", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mmoc_diffusion_args(C.Structure):
    _fields_ = [("theta", C.c_double), ("tau", C.c_double), ("kappa", C.c_double), ("q0", C.c_void_p),
                ("q1", C.c_void_p), ("dirichlet", C.c_void_p), ("rtol", C.c_double), ("max_iter", C.c_int),
                ("precond", C.c_int)]


class mmoc_diffusion_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("rel_residual", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Loads libmmoc.so (raises ImportError if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise ImportError("libmmoc.so is not built (%s); run __graft_entry__.build()" % LIB)
    L = C.CDLL(LIB)
    P, I, D, I64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
    st = C.c_int
    sig = {
        "mmoc_default_options": (None, [C.POINTER(mmoc_options)]),
        "mmoc_create": (st, [C.POINTER(P), I, I, I, C.POINTER(mmoc_options), P]),
        "mmoc_set_stream": (st, [P, P]),
        "mmoc_upload_mesh": (st, [P, I, P, I, P, I]),
        "mmoc_num_dofs": (st, [P, C.POINTER(I64), C.POINTER(I64)]),
        "mmoc_dof_coords": (st, [P, P]),
        "mmoc_set_velocity": (st, [P, I, P]),
        "mmoc_set_stationary": (st, [P, I]),
        "mmoc_swap_velocity_levels": (st, [P]),
        "mmoc_set_scalar": (st, [P, P]),
        "mmoc_use_last_chat": (st, [P]),
        "mmoc_set_fields": (st, [P, I, P, P]),
        "mmoc_trace_step": (st, [P, D, I, P, P]),
        "mmoc_get_stats": (st, [P, C.POINTER(mmoc_stats)]),
        "mmoc_reset_stats": (st, [P]),
        "mmoc_mlp_nparams": (I64, []),
        "mmoc_mlp_configure": (st, [P, P, P, D]),
        "mmoc_mlp_set_predictor": (st, [P, I, D, D]),
        "mmoc_mlp_record": (st, [P, D, D, P, I64]),
        "mmoc_mlp_train": (st, [P, I64, I, I, C.c_float, C.c_ulonglong, C.POINTER(D)]),
        "mmoc_mlp_get_weights": (st, [P, P, I64]),
        "mmoc_mlp_set_weights": (st, [P, P, I64]),
        "mmoc_mlp_infer": (st, [P, D, D, P]),
        "mmoc_mlp_forward": (st, [P, P, I64, P]),
        "mmoc_mlp_loss_grad": (st, [P, P, P, I64, P, C.POINTER(D)]),
        "mmoc_trace_step_surrogate": (st, [P, D, D, I, C.c_float, D, I64, P, P]),
        "mmoc_mass_inner": (st, [P, P, P, P, P, C.POINTER(D)]),
        "mmoc_mass_inner_noalloc": (st, [P, P, P, P, P, P]),
        "mmoc_field_range": (st, [P, P, C.POINTER(D), C.POINTER(D)]),
        "mmoc_lookback_run": (st, [P, D, I, I64, I64, P, I64, P]),
        "mmoc_set_rk_tableau": (st, [P, I, P, P, P]),
        "mmoc_cfl_time_step": (st, [P, D, I, C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
        "mmoc_set_level_count": (st, [P, I]),
        "mmoc_trace_span": (st, [P, I, I, D, I, P, P]),
        "mmoc_fe_assemble": (st, [P, C.POINTER(I64)]),
        "mmoc_fe_export": (st, [P, I, P, P, P]),
        "mmoc_fe_apply": (st, [P, I, P, P]),
        "mmoc_boundary_mask": (st, [P, P]),
        "mmoc_diffusion_step": (st, [P, C.POINTER(mmoc_diffusion_args), P, P, C.POINTER(mmoc_diffusion_info)]),
        "mmoc_last_error": (C.c_char_p, [P]),
        "mmoc_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check(ctx, status):
    if status != 0:
        msg = lib().mmoc_last_error(ctx).decode() if ctx else ""
        raise MMOCError(status, msg)


# ----------------------------------------------------------------- C names

def mmoc_default_options():
    o = mmoc_options()
    lib().mmoc_default_options(C.byref(o))
    return o


def mmoc_create(dim, level, prec=MMOC_FP64, opt: Optional[mmoc_options] = None, stream=None):
    h = C.c_void_p()
    s = lib().mmoc_create(C.byref(h), int(dim), int(level), int(prec),
                          C.byref(opt) if opt is not None else None, _stream(stream))
    if s != 0:
        raise MMOCError(s, "mmoc_create failed")
    return h


def mmoc_set_stream(ctx, stream=None):
    _check(ctx, lib().mmoc_set_stream(ctx, _stream(stream)))


def mmoc_upload_mesh(ctx, vertices: np.ndarray, macros: np.ndarray, blend=MMOC_BLEND_NONE):
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    m = np.ascontiguousarray(macros, dtype=np.int32)
    _check(ctx, lib().mmoc_upload_mesh(ctx, v.shape[0], v.ctypes.data_as(C.c_void_p), m.shape[0],
                                       m.ctypes.data_as(C.c_void_p), int(blend)))


def mmoc_num_dofs(ctx):
    n, b = C.c_int64(), C.c_int64()
    _check(ctx, lib().mmoc_num_dofs(ctx, C.byref(n), C.byref(b)))
    return n.value, b.value


def mmoc_dof_coords(ctx, out: torch.Tensor):
    _check(ctx, lib().mmoc_dof_coords(ctx, _ptr(out)))


def mmoc_set_velocity(ctx, level, u: torch.Tensor):
    _check(ctx, lib().mmoc_set_velocity(ctx, int(level), _ptr(u)))


def mmoc_set_stationary(ctx, on):
    _check(ctx, lib().mmoc_set_stationary(ctx, int(bool(on))))


def mmoc_swap_velocity_levels(ctx):
    _check(ctx, lib().mmoc_swap_velocity_levels(ctx))


def mmoc_set_scalar(ctx, c: torch.Tensor):
    _check(ctx, lib().mmoc_set_scalar(ctx, _ptr(c)))


def mmoc_use_last_chat(ctx):
    _check(ctx, lib().mmoc_use_last_chat(ctx))


def mmoc_set_fields(ctx, level, u: torch.Tensor, c: torch.Tensor):
    _check(ctx, lib().mmoc_set_fields(ctx, int(level), _ptr(u), _ptr(c)))


def mmoc_trace_step(ctx, dt, substeps, c_hat: torch.Tensor, X: Optional[torch.Tensor]):
    _check(ctx, lib().mmoc_trace_step(ctx, float(dt), int(substeps), _ptr(c_hat), _ptr(X)))


def mmoc_get_stats(ctx):
    s = mmoc_stats()
    _check(ctx, lib().mmoc_get_stats(ctx, C.byref(s)))
    return s.as_dict()


def mmoc_reset_stats(ctx):
    _check(ctx, lib().mmoc_reset_stats(ctx))


def mmoc_mlp_nparams():
    return int(lib().mmoc_mlp_nparams())


def mmoc_mlp_configure(ctx, lo, hi, U):
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    _check(ctx, lib().mmoc_mlp_configure(ctx, lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p),
                                         float(U)))


def mmoc_mlp_set_predictor(ctx, substeps, scale=1.0, period=0.0):
    _check(ctx, lib().mmoc_mlp_set_predictor(ctx, int(substeps), float(scale), float(period)))


def mmoc_mlp_record(ctx, t_np1, dt, X: torch.Tensor, capacity):
    _check(ctx, lib().mmoc_mlp_record(ctx, float(t_np1), float(dt), _ptr(X), int(capacity)))


def mmoc_mlp_train(ctx, n_samples, epochs, batch, lr, seed):
    loss = C.c_double()
    _check(ctx, lib().mmoc_mlp_train(ctx, int(n_samples), int(epochs), int(batch), float(lr), int(seed),
                                     C.byref(loss)))
    return loss.value


def mmoc_mlp_get_weights(ctx):
    n = mmoc_mlp_nparams()
    w = np.empty(n, dtype=np.float32)
    _check(ctx, lib().mmoc_mlp_get_weights(ctx, w.ctypes.data_as(C.c_void_p), n))
    return w


def mmoc_mlp_set_weights(ctx, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(ctx, lib().mmoc_mlp_set_weights(ctx, w.ctypes.data_as(C.c_void_p), w.shape[0]))


def mmoc_mlp_forward(ctx, inp: torch.Tensor, out: torch.Tensor):
    _check(ctx, lib().mmoc_mlp_forward(ctx, _ptr(inp), int(inp.shape[0]), _ptr(out)))


def mmoc_mlp_loss_grad(ctx, inp: torch.Tensor, target: torch.Tensor, grad: torch.Tensor):
    loss = C.c_double()
    _check(ctx, lib().mmoc_mlp_loss_grad(ctx, _ptr(inp), _ptr(target), int(inp.shape[0]), _ptr(grad),
                                         C.byref(loss)))
    return loss.value


def mmoc_mlp_infer(ctx, t_np1, dt, X: torch.Tensor):
    _check(ctx, lib().mmoc_mlp_infer(ctx, float(t_np1), float(dt), _ptr(X)))


def mmoc_trace_step_surrogate(ctx, t_np1, dt, substeps, check_fraction, tol, step, c_hat, X):
    _check(ctx, lib().mmoc_trace_step_surrogate(ctx, float(t_np1), float(dt), int(substeps),
                                                float(check_fraction), float(tol), int(step), _ptr(c_hat),
                                                _ptr(X)))


def mmoc_mass_inner(ctx, a, a_sub, b, b_sub):
    out = C.c_double()
    _check(ctx, lib().mmoc_mass_inner(ctx, _ptr(a), _ptr(a_sub), _ptr(b), _ptr(b_sub), C.byref(out)))
    return out.value


def mmoc_mass_inner_noalloc(ctx, a, a_sub, b, b_sub, out: torch.Tensor):
    """(a - a_sub)^T M (b - b_sub) into out (one float64 on the device),
    asynchronously, with no device allocation."""
    _check(ctx, lib().mmoc_mass_inner_noalloc(ctx, _ptr(a), _ptr(a_sub), _ptr(b), _ptr(b_sub), _ptr(out)))


def mmoc_field_range(ctx, c):
    lo, hi = C.c_double(), C.c_double()
    _check(ctx, lib().mmoc_field_range(ctx, _ptr(c), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def mmoc_lookback_run(ctx, tau, substeps, n_steps, b, ring: torch.Tensor, c_out: torch.Tensor):
    _check(ctx, lib().mmoc_lookback_run(ctx, float(tau), int(substeps), int(n_steps), int(b), _ptr(ring),
                                        int(ring.shape[0]), _ptr(c_out)))


def mmoc_set_rk_tableau(ctx, A=None, b=None, c=None):
    """A general explicit RK method (A [s][s], b [s], c [s]); None restores RK4."""
    if A is None:
        _check(ctx, lib().mmoc_set_rk_tableau(ctx, 0, None, None, None))
        return
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    dp = lambda x: x.ctypes.data_as(C.c_void_p)
    _check(ctx, lib().mmoc_set_rk_tableau(ctx, int(b.shape[0]), dp(A), dp(b), dp(c)))


def mmoc_cfl_time_step(ctx, cfl, level=0):
    """(tau, max |u|, h_min)."""
    t, u, h = C.c_double(), C.c_double(), C.c_double()
    _check(ctx, lib().mmoc_cfl_time_step(ctx, float(cfl), int(level), C.byref(t), C.byref(u), C.byref(h)))
    return t.value, u.value, h.value


def mmoc_set_level_count(ctx, levels):
    _check(ctx, lib().mmoc_set_level_count(ctx, int(levels)))


def mmoc_trace_span(ctx, first, n_int, dt, substeps, c_hat: torch.Tensor, X: Optional[torch.Tensor]):
    _check(ctx, lib().mmoc_trace_span(ctx, int(first), int(n_int), float(dt), int(substeps), _ptr(c_hat), _ptr(X)))


def mmoc_fe_assemble(ctx):
    nnz = C.c_int64()
    _check(ctx, lib().mmoc_fe_assemble(ctx, C.byref(nnz)))
    return nnz.value


def mmoc_fe_export(ctx, which, N):
    """(row_ptr [N+1] int64, cols [nnz] int32, vals [nnz] float64) as numpy arrays."""
    nnz = mmoc_fe_assemble(ctx)
    rp = np.empty(N + 1, dtype=np.int64)
    ci = np.empty(nnz, dtype=np.int32)
    va = np.empty(nnz, dtype=np.float64)
    vp = lambda x: x.ctypes.data_as(C.c_void_p)
    _check(ctx, lib().mmoc_fe_export(ctx, int(which), vp(rp), vp(ci), vp(va)))
    return rp, ci, va


def mmoc_fe_apply(ctx, which, x: torch.Tensor, y: torch.Tensor):
    _check(ctx, lib().mmoc_fe_apply(ctx, int(which), _ptr(x), _ptr(y)))


def mmoc_boundary_mask(ctx, N):
    out = np.empty(N, dtype=np.uint8)
    _check(ctx, lib().mmoc_boundary_mask(ctx, out.ctypes.data_as(C.c_void_p)))
    return out


def mmoc_diffusion_step(ctx, c_hat: torch.Tensor, c_out: torch.Tensor, theta, tau, kappa, q0=None, q1=None,
                        dirichlet=None, rtol=0.0, max_iter=0, precond=1):
    a = mmoc_diffusion_args(float(theta), float(tau), float(kappa), _ptr(q0), _ptr(q1), _ptr(dirichlet),
                            float(rtol), int(max_iter), int(precond))
    info = mmoc_diffusion_info()
    _check(ctx, lib().mmoc_diffusion_step(ctx, C.byref(a), _ptr(c_hat), _ptr(c_out), C.byref(info)))
    return info.as_dict()


def mmoc_last_error(ctx):
    return lib().mmoc_last_error(ctx).decode()


def mmoc_destroy(ctx):
    lib().mmoc_destroy(ctx)


# ------------------------------------------------------------ convenience

class Tracer:
    """Owns one library context on the current device (torch's current stream)."""

    def __init__(self, dim, level, vertices, macros, blend=0, precision=MMOC_FP64, options=None, stream=None):
        self.dim, self.level, self.precision = int(dim), int(level), int(precision)
        self.ctx = mmoc_create(dim, level, precision, options, stream)
        try:
            mmoc_upload_mesh(self.ctx, vertices, macros, blend)
        except Exception:
            mmoc_destroy(self.ctx)
            self.ctx = None
            raise
        self.N, self.n_block = mmoc_num_dofs(self.ctx)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_workload(cls, wl, precision=MMOC_FP64, level=None, options=None, order=None):
        """order: 2 (P2, default) or 1 (P1); sets options.order."""
        if order is not None:
            if options is None:
                options = mmoc_default_options()
            options.order = int(order)
        return cls(wl.dim, wl.level if level is None else level, wl.vertices, wl.macros, wl.blend, precision,
                   options)

    def close(self):
        if self.ctx is not None:
            mmoc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def scalar_dtype(self):
        return torch.float64 if self.precision == MMOC_FP64 else torch.float32

    def dof_coords(self):
        x = torch.empty((self.dim, self.N), dtype=torch.float64, device=self.device)
        mmoc_dof_coords(self.ctx, x)
        return x

    def set_velocity(self, level, u):
        mmoc_set_velocity(self.ctx, level, u)

    def set_stationary(self, on=True):
        mmoc_set_stationary(self.ctx, on)

    def set_scalar(self, c):
        mmoc_set_scalar(self.ctx, c)

    def use_last_chat(self):
        """the next step's scalar is the last step's chat (options.keep_chat)"""
        mmoc_use_last_chat(self.ctx)

    def set_fields(self, level, u, c):
        """velocity level and scalar in one ingestion pass"""
        mmoc_set_fields(self.ctx, level, u, c)

    def swap_levels(self):
        mmoc_swap_velocity_levels(self.ctx)

    def trace_step(self, dt, substeps, c_hat=None, X=None, want_X=True):
        if c_hat is None:
            c_hat = torch.empty(self.N, dtype=self.scalar_dtype, device=self.device)
        if X is None and want_X:
            X = torch.empty((self.dim, self.N), dtype=torch.float64, device=self.device)
        mmoc_trace_step(self.ctx, dt, substeps, c_hat, X)
        return c_hat, X

    def stats(self):
        return mmoc_get_stats(self.ctx)

    def reset_stats(self):
        mmoc_reset_stats(self.ctx)

    def set_level_count(self, levels):
        mmoc_set_level_count(self.ctx, levels)

    def trace_span(self, first, n_int, dt, substeps, c_hat=None, X=None, want_X=True):
        if c_hat is None:
            c_hat = torch.empty(self.N, dtype=self.scalar_dtype, device=self.device)
        if X is None and want_X:
            X = torch.empty((self.dim, self.N), dtype=torch.float64, device=self.device)
        mmoc_trace_span(self.ctx, first, n_int, dt, substeps, c_hat, X)
        return c_hat, X

    def mass_inner(self, a=None, a_sub=None, b=None, b_sub=None):
        """(a - a_sub)^T M (b - b_sub) with the P2 mass matrix (None: ones / zero)."""
        return mmoc_mass_inner(self.ctx, a, a_sub, b, b_sub)

    def field_range(self, c):
        return mmoc_field_range(self.ctx, c)

    # ---------------------------------------------------- diffusion (Sec. 2.2)

    def fe_assemble(self):
        return mmoc_fe_assemble(self.ctx)

    def fe_matrix(self, which):
        """(row_ptr, cols, vals) of the mass (0) or stiffness (1) matrix, on the host."""
        return mmoc_fe_export(self.ctx, which, self.N)

    def fe_apply(self, which, x, y=None):
        if y is None:
            y = torch.empty(self.N, dtype=torch.float64, device=self.device)
        mmoc_fe_apply(self.ctx, which, x, y)
        return y

    def boundary_mask(self):
        return mmoc_boundary_mask(self.ctx, self.N).astype(bool)

    def diffusion_step(self, c_hat, tau, kappa, theta=1.0, q0=None, q1=None, dirichlet=None, rtol=1e-12,
                       max_iter=0, precond=1, out=None):
        """One Theta-method step; returns (c, info)."""
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        info = mmoc_diffusion_step(self.ctx, c_hat, out, theta, tau, kappa, q0, q1, dirichlet, rtol, max_iter,
                                   precond)
        return out, info

    def lookback_run(self, c0, tau, n_steps, b, substeps=1):
        """c^{n_steps} from c^0 with look-back distance b (b <= 0: infinity);
        the velocity must be stationary.  Returns the new field."""
        span = n_steps if b <= 0 else min(b, n_steps)
        ring = torch.empty((1 if b <= 0 else span + 1, self.N), dtype=torch.float64, device=self.device)
        ring[0].copy_(c0)
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        mmoc_lookback_run(self.ctx, tau, substeps, n_steps, b, ring, out)
        return out


def _tracer_mlp_methods():
    def mlp_configure(self, lo, hi, U):
        mmoc_mlp_configure(self.ctx, lo, hi, U)

    def mlp_set_predictor(self, substeps, scale=1.0, period=0.0):
        mmoc_mlp_set_predictor(self.ctx, substeps, scale, period)

    def mlp_record(self, t_np1, dt, X, capacity):
        mmoc_mlp_record(self.ctx, t_np1, dt, X, capacity)

    def mlp_train(self, n_samples, epochs, batch=8192, lr=1e-3, seed=5):
        return mmoc_mlp_train(self.ctx, n_samples, epochs, batch, lr, seed)

    def mlp_infer(self, t_np1, dt, X=None):
        if X is None:
            X = torch.empty((self.dim, self.N), dtype=torch.float64, device=self.device)
        mmoc_mlp_infer(self.ctx, t_np1, dt, X)
        return X

    def trace_step_surrogate(self, t_np1, dt, substeps, check_fraction=0.01, tol=1e-4, step=0, c_hat=None, X=None):
        if c_hat is None:
            c_hat = torch.empty(self.N, dtype=self.scalar_dtype, device=self.device)
        if X is None:
            X = torch.empty((self.dim, self.N), dtype=torch.float64, device=self.device)
        mmoc_trace_step_surrogate(self.ctx, t_np1, dt, substeps, check_fraction, tol, step, c_hat, X)
        return c_hat, X

    for f in (mlp_configure, mlp_set_predictor, mlp_record, mlp_train, mlp_infer, trace_step_surrogate):
        setattr(Tracer, f.__name__, f)


_tracer_mlp_methods()
