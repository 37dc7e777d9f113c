"""Python binding of the pressure-projection library.

Argument marshalling only: every computation runs in the HIP kernels of
libpp.so.  PyTorch provides device memory (CUDA/HIP tensors) and the stream.
All arrays are float64 CUDA tensors of shape (nz, ny, nx), contiguous; face
arrays use the low-face convention of include/pp.h.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import torch

from . import _lib as L

PRECISIONS = {"fp64": L.PP_FP64, "fp32": L.PP_MIXED_FP32, "fp16": L.PP_MIXED_FP16}
OUTERS = {"pcg": L.PP_OUTER_PCG, "dc": L.PP_OUTER_DC}
CYCLES = {"v": L.PP_CYCLE_V, "w": L.PP_CYCLE_W, "f": L.PP_CYCLE_F}


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_field(t: torch.Tensor, shape, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64 (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def make_grid(shape: Sequence[int], h: float, bc: Sequence[int]) -> L.Grid:
    """shape is (nz, ny, nx); bc is (bc_x, bc_y, bc_z) with 0 periodic, 1 wall."""
    nz, ny, nx = (int(v) for v in shape)
    g = L.Grid()
    g.n[0], g.n[1], g.n[2] = nx, ny, nz
    g.h = float(h)
    for m in range(3):
        g.bc[m] = int(bc[m])
    return g


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def face_coeffs(rho: torch.Tensor, h: float, bc: Sequence[int],
                out: Optional[Tuple[torch.Tensor, ...]] = None):
    """beta_m = 2 / (rho_L + rho_R) on every face, 0 on wall faces."""
    lib = L.load()
    g = make_grid(rho.shape, h, bc)
    _check_field(rho, rho.shape, "rho")
    if out is None:
        out = tuple(torch.empty_like(rho) for _ in range(3))
    for m, t in enumerate(out):
        _check_field(t, rho.shape, f"beta[{m}]")
    L.check(lib.pp_face_coeffs(ctypes.byref(g), _ptr(rho), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                               _stream_handle(None)), "pp_face_coeffs")
    return out


class Solver:
    """A solver context for one set of face coefficients beta = 1/rho_f.

    With `sigma` (a cell field >= 0) or `general=True` the context holds the
    general operator A x - sigma x, where interior faces may also be closed
    (beta = 0) and cells with no open face and no sigma are excluded (see
    pp_setup_general in include/pp.h)."""

    def __init__(self, beta: Sequence[torch.Tensor], h: float, bc: Sequence[int],
                 precision: str = "fp32", outer: str = "pcg", nu_pre: int = 2, nu_post: int = 2,
                 max_outer: int = 500, warm_start: bool = False, fallback: bool = True,
                 coarse_graph: bool = False, nu_coarse: int = 4, omega: Optional[float] = None,
                 cycle: str = "v", coarsest: int = 64, stream: Optional[torch.cuda.Stream] = None,
                 sigma: Optional[torch.Tensor] = None, general: bool = False):
        lib = L.load()
        self._lib = lib
        self.shape = tuple(beta[0].shape)
        for m, t in enumerate(beta):
            _check_field(t, self.shape, f"beta[{m}]")
        self.h = float(h)
        self.bc = tuple(int(v) for v in bc)
        self.grid = make_grid(self.shape, h, bc)
        o = L.Opts()
        lib.pp_opts_default(ctypes.byref(o))
        o.precision = PRECISIONS[precision]
        o.outer = OUTERS[outer]
        o.nu_pre = nu_pre
        o.nu_post = nu_post
        o.max_outer = max_outer
        o.warm_start = int(bool(warm_start))
        o.fallback = int(bool(fallback))
        o.coarse_graph = int(bool(coarse_graph))
        o.nu_coarse = nu_coarse
        if omega is not None:       # None: the library's default
            o.omega = float(omega)
        o.cycle = CYCLES[cycle]
        o.coarsest = coarsest
        self.opts = o
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._ctx = ctypes.c_void_p()
        self.general = bool(general) or sigma is not None
        self.has_sigma = sigma is not None
        if self.general:
            if sigma is not None:
                _check_field(sigma, self.shape, "sigma")
            L.check(lib.pp_setup_general(ctypes.byref(self.grid), _ptr(beta[0]), _ptr(beta[1]),
                                         _ptr(beta[2]), None if sigma is None else _ptr(sigma),
                                         ctypes.byref(o), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(self._ctx)), "pp_setup_general")
        else:
            L.check(lib.pp_setup(ctypes.byref(self.grid), _ptr(beta[0]), _ptr(beta[1]), _ptr(beta[2]),
                                 ctypes.byref(o), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(self._ctx)), "pp_setup")
        self.last_stats = None

    # -- lifetime ---------------------------------------------------------
    def close(self) -> None:
        if self._ctx:
            self._lib.pp_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries ----------------------------------------------------------
    @property
    def levels(self) -> int:
        n = ctypes.c_int32()
        L.check(self._lib.pp_levels(self._ctx, ctypes.byref(n)), "pp_levels")
        return n.value

    def level_dims(self, level: int) -> Tuple[int, int, int]:
        d = (ctypes.c_int32 * 3)()
        L.check(self._lib.pp_level_dims(self._ctx, level, d), "pp_level_dims")
        return (d[0], d[1], d[2])

    @property
    def memory_bytes(self) -> int:
        b = ctypes.c_int64()
        L.check(self._lib.pp_memory(self._ctx, ctypes.byref(b)), "pp_memory")
        return b.value

    # -- operations -------------------------------------------------------
    def _field(self, t, name):
        _check_field(t, self.shape, name)
        return _ptr(t)

    def update_coeffs(self, beta: Sequence[torch.Tensor],
                      sigma: Optional[torch.Tensor] = None) -> None:
        if self.general:
            L.check(self._lib.pp_update_general(self._ctx, *(self._field(b, "beta") for b in beta),
                                                None if sigma is None else self._field(sigma, "sigma")),
                    "pp_update_general")
        else:
            if sigma is not None:
                raise ValueError("sigma needs a context made with sigma or general=True")
            L.check(self._lib.pp_update_coeffs(self._ctx, *(self._field(b, "beta") for b in beta)),
                    "pp_update_coeffs")

    def update_density(self, rho: torch.Tensor) -> None:
        """New face coefficients beta = 2 / (rho_L + rho_R) computed from the
        cell densities on the device, with the hierarchy rebuild, in one pass."""
        if self.general:
            raise ValueError("a general context takes its coefficients from update_coeffs")
        L.check(self._lib.pp_update_density(self._ctx, self._field(rho, "rho")),
                "pp_update_density")

    def divergence(self, u: Sequence[torch.Tensor], scale: float = 1.0,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=u[0].device)
        L.check(self._lib.pp_divergence(self._ctx, *(self._field(v, "u") for v in u), float(scale),
                                        self._field(out, "out")), "pp_divergence")
        return out

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(x)
        L.check(self._lib.pp_apply(self._ctx, self._field(x, "x"), self._field(out, "out")), "pp_apply")
        return out

    def solve(self, rhs: torch.Tensor, tol: float = 1e-8, p: Optional[torch.Tensor] = None,
              check: bool = True) -> torch.Tensor:
        """Mean-zero p with A p = rhs - mean(rhs); stats in self.last_stats."""
        if p is None:
            p = torch.empty_like(rhs)
        st = L.Stats()
        rc = self._lib.pp_solve(self._ctx, self._field(rhs, "rhs"), self._field(p, "p"), float(tol),
                                ctypes.byref(st))
        self.last_stats = st.as_dict()
        if check or rc not in (L.PP_OK, L.PP_ENOCONV):
            L.check(rc, "pp_solve")
        return p

    def project(self, us: Sequence[torch.Tensor], p: torch.Tensor, dt: float,
                out: Optional[Sequence[torch.Tensor]] = None):
        if out is None:
            out = tuple(torch.empty_like(p) for _ in range(3))
        L.check(self._lib.pp_project(self._ctx, *(self._field(v, "us") for v in us),
                                     self._field(p, "p"), float(dt),
                                     *(self._field(v, "u") for v in out)), "pp_project")
        return out

    def step(self, rho: torch.Tensor, us: Sequence[torch.Tensor], dt: float, tol: float = 1e-8,
             p: Optional[torch.Tensor] = None, rhs: Optional[torch.Tensor] = None,
             out: Optional[Sequence[torch.Tensor]] = None, check: bool = True):
        """One projection step in one call (pp_step): coefficients from rho,
        rhs = D us / dt, p from the solve, u projected; returns (p, u).  The
        same results as update_density, divergence, solve and project."""
        if self.general:
            raise ValueError("a general context takes its coefficients from update_coeffs")
        if p is None:
            p = torch.empty_like(rho)
        if rhs is None:
            rhs = torch.empty_like(rho)
        if out is None:
            out = tuple(torch.empty_like(rho) for _ in range(3))
        st = L.Stats()
        rc = self._lib.pp_step(self._ctx, self._field(rho, "rho"),
                               *(self._field(v, "us") for v in us), float(dt), float(tol),
                               self._field(rhs, "rhs"), self._field(p, "p"),
                               *(self._field(v, "u") for v in out), ctypes.byref(st))
        self.last_stats = st.as_dict()
        if check or rc not in (L.PP_OK, L.PP_ENOCONV):
            L.check(rc, "pp_step")
        return p, out

    def adjoint(self, p: torch.Tensor, g_p: torch.Tensor, tol: float = 1e-8,
                check: bool = True):
        """Returns (g_rhs, (g_beta_x, g_beta_y, g_beta_z)) for L with dL/dp = g_p."""
        g_rhs = torch.empty_like(p)
        g_b = tuple(torch.empty_like(p) for _ in range(3))
        st = L.Stats()
        rc = self._lib.pp_solve_adjoint(self._ctx, self._field(p, "p"), self._field(g_p, "g_p"),
                                        float(tol), _ptr(g_rhs), _ptr(g_b[0]), _ptr(g_b[1]),
                                        _ptr(g_b[2]), ctypes.byref(st))
        self.last_stats = st.as_dict()
        if check or rc not in (L.PP_OK, L.PP_ENOCONV):
            L.check(rc, "pp_solve_adjoint")
        return g_rhs, g_b

    def vcycle(self, r: torch.Tensor) -> torch.Tensor:
        e = torch.empty_like(r)
        L.check(self._lib.pp_vcycle(self._ctx, self._field(r, "r"), self._field(e, "e")), "pp_vcycle")
        return e

    # -- kernel timing ----------------------------------------------------
    def timing(self, on, kinds=None) -> None:
        """Time fine-level launches of the given kinds (all kinds by default)."""
        if not on:
            mask = 0
        elif kinds is None:
            mask = (1 << L.PP_KT_COUNT) - 1
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << int(k)
        L.check(self._lib.pp_timing_enable(self._ctx, mask), "pp_timing_enable")

    def timing_reset(self) -> None:
        L.check(self._lib.pp_timing_reset(self._ctx), "pp_timing_reset")

    def timing_get(self, kind: int) -> Tuple[int, float]:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        L.check(self._lib.pp_timing_get(self._ctx, kind, ctypes.byref(n), ctypes.byref(ms)),
                "pp_timing_get")
        return n.value, ms.value


class PressureSolve(torch.autograd.Function):
    """p = S(rhs; beta): the mean-zero solution of D(beta G p) = rhs - mean(rhs).

    backward returns dL/d rhs (one transposed solve; the operator is symmetric)
    and dL/d beta on every face (the face product G lambda * G p).
    """

    @staticmethod
    def forward(ctx, rhs, beta_x, beta_y, beta_z, solver: Solver, tol: float, adj_tol: float):
        p = solver.solve(rhs, tol=tol)
        ctx.solver = solver
        ctx.adj_tol = adj_tol
        ctx.save_for_backward(p)
        return p

    @staticmethod
    def backward(ctx, g_p):
        (p,) = ctx.saved_tensors
        g_rhs, g_b = ctx.solver.adjoint(p, g_p.contiguous(), tol=ctx.adj_tol)
        return g_rhs, g_b[0], g_b[1], g_b[2], None, None, None


def pressure_solve(rhs: torch.Tensor, beta: Sequence[torch.Tensor], solver: Solver,
                   tol: float = 1e-8, adj_tol: Optional[float] = None) -> torch.Tensor:
    """Differentiable solve; `solver` must have been built from these beta."""
    return PressureSolve.apply(rhs, beta[0], beta[1], beta[2], solver, tol,
                               tol if adj_tol is None else adj_tol)


# -- single-kernel entry points -----------------------------------------------

def k_smooth(shape, h, bc, beta, r, e, sweeps=1, zero_init=False, omega=1.0):
    lib = L.load()
    g = make_grid(shape, h, bc)
    L.check(lib.pp_k_smooth(ctypes.byref(g), *(_ptr(b) for b in beta), _ptr(r), _ptr(e), sweeps,
                            int(zero_init), float(omega), _stream_handle(None)), "pp_k_smooth")
    return e


def k_smooth_fused(shape, h, bc, beta, r, e_in, e_out, first_colour=0, zero_init=False,
                   omega=1.0):
    lib = L.load()
    g = make_grid(shape, h, bc)
    L.check(lib.pp_k_smooth_fused(ctypes.byref(g), *(_ptr(b) for b in beta), _ptr(r), _ptr(e_in),
                                  _ptr(e_out), int(first_colour), int(zero_init), float(omega),
                                  _stream_handle(None)), "pp_k_smooth_fused")
    return e_out


def k_smooth2_fused_f32(shape, h, bc, beta, r, e_in, e_out, first_colour=0, zero_init=False,
                        omega=1.0):
    """Two fused sweeps on float32 device tensors (the FP32 V-cycle's kernel)."""
    lib = L.load()
    g = make_grid(shape, h, bc)
    for t in (*beta, r, e_in, e_out):
        if t.dtype != torch.float32:
            raise TypeError("k_smooth2_fused_f32 takes float32 tensors")
    L.check(lib.pp_k_smooth2_fused_f32(ctypes.byref(g), *(_ptr(b) for b in beta), _ptr(r),
                                       _ptr(e_in), _ptr(e_out), int(first_colour), int(zero_init),
                                       float(omega), _stream_handle(None)),
            "pp_k_smooth2_fused_f32")
    return e_out


def k_smooth2_fused_dot_f32(shape, h, bc, beta, r, e_in, e_out, first_colour=0, omega=1.0):
    """k_smooth2_fused_f32 that also returns sum(r * e_out), r the pass's own
    right-hand side (products and sum in FP64)."""
    lib = L.load()
    g = make_grid(shape, h, bc)
    for t in (*beta, r, e_in, e_out):
        if t.dtype != torch.float32:
            raise TypeError("k_smooth2_fused_dot_f32 takes float32 fields")
    dot = torch.empty(1, dtype=torch.float64, device=r.device)
    L.check(lib.pp_k_smooth2_fused_dot_f32(ctypes.byref(g), *(_ptr(b) for b in beta), _ptr(r),
                                           _ptr(e_in), _ptr(e_out), int(first_colour),
                                           float(omega), _ptr(dot), _stream_handle(None)),
            "pp_k_smooth2_fused_dot_f32")
    return float(dot[0].item())


def k_smooth2_fused_dot_f32_noalloc(shape, h, bc, beta, r, e_in, e_out, dot, first_colour=0,
                                    omega=1.0):
    """The pass of k_smooth2_fused_dot_f32 through the entry point that
    allocates nothing: its partial sums use the library's static device
    array, and the result goes to `dot` (a float64 device tensor of at least
    one element) on the current stream, without waiting."""
    lib = L.load()
    g = make_grid(shape, h, bc)
    for t in (*beta, r, e_in, e_out):
        if t.dtype != torch.float32:
            raise TypeError("k_smooth2_fused_dot_f32_noalloc takes float32 fields")
    if dot.dtype != torch.float64 or dot.numel() < 1:
        raise TypeError("dot must be a float64 tensor of at least one element")
    L.check(lib.pp_k_smooth2_fused_dot_f32_noalloc(ctypes.byref(g), *(_ptr(b) for b in beta),
                                                   _ptr(r), _ptr(e_in), _ptr(e_out),
                                                   int(first_colour), float(omega), _ptr(dot),
                                                   _stream_handle(None)),
            "pp_k_smooth2_fused_dot_f32_noalloc")
    return dot


def k_resid_restrict(shape, h, bc, beta, e, r, rH):
    lib = L.load()
    g = make_grid(shape, h, bc)
    L.check(lib.pp_k_resid_restrict(ctypes.byref(g), *(_ptr(b) for b in beta), _ptr(e), _ptr(r),
                                    _ptr(rH), _stream_handle(None)), "pp_k_resid_restrict")
    return rH


def k_prolong_add(shape, h, bc, eH, e):
    lib = L.load()
    g = make_grid(shape, h, bc)
    L.check(lib.pp_k_prolong_add(ctypes.byref(g), _ptr(eH), _ptr(e), _stream_handle(None)),
            "pp_k_prolong_add")
    return e


def k_prolong_weights(shape, h, bc, beta):
    """Prolongation weights of every cell (int32 tensor: the x, y and z
    weights as 8-bit fractions of 256 in bits 0-7, 8-15, 16-23), from the
    FP64 face coefficients."""
    lib = L.load()
    g = make_grid(shape, h, bc)
    w = torch.empty(tuple(shape), dtype=torch.int32, device=beta[0].device)
    L.check(lib.pp_k_prolong_weights(ctypes.byref(g), *(_ptr(b) for b in beta), _ptr(w),
                                     _stream_handle(None)), "pp_k_prolong_weights")
    return w


def k_prolong_add_weighted(shape, h, bc, eH, w, e):
    lib = L.load()
    g = make_grid(shape, h, bc)
    L.check(lib.pp_k_prolong_add_weighted(ctypes.byref(g), _ptr(eH), _ptr(w), _ptr(e),
                                          _stream_handle(None)), "pp_k_prolong_add_weighted")
    return e


def k_coarsen_beta(shape, h, bc, beta, out):
    lib = L.load()
    g = make_grid(shape, h, bc)
    L.check(lib.pp_k_coarsen_beta(ctypes.byref(g), *(_ptr(b) for b in beta), *(_ptr(o) for o in out),
                                  _stream_handle(None)), "pp_k_coarsen_beta")
    return out


def k_copy(src: torch.Tensor, dst: torch.Tensor):
    lib = L.load()
    L.check(lib.pp_k_copy(_ptr(src), _ptr(dst), src.numel(), _stream_handle(None)), "pp_k_copy")
    return dst
