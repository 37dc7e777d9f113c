"""Plain FP64 CPU oracle for the pressure-projection step (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never touches it, and the two share no code.

Functions (all arrays are float64 numpy arrays in the (nz, ny, nx) layout, face
arrays use the low-face convention, bc is (bc_x, bc_y, bc_z) with 0 = periodic
and 1 = wall):

  face_coeffs(rho, bc)              beta = 1/rho on faces (Sec. 3.7.1)
  divergence(u, bc, h, scale)       scale * D u (eq. cont2)
  apply(beta, bc, h, x)             A x = D beta G x (Sec. 3.7.1 system)
  solve(beta, bc, h, rhs, tol)      mean-zero p with A p = rhs - mean(rhs)
  project(beta, bc, h, dt, us, p)   u = u* - dt beta G p (eq. fotm)
  rbsor(...)                        the paper's red-black SOR (eq. beta_pressure)
  adjoint(beta, bc, h, p, gp, tol)  dL/d rhs and dL/d beta for L = <gp, p>

General operator A_g x = A x - sigma x (closed links beta = 0 on interior
faces, Sec. 3.8; a diagonal sigma from the implicit viscous step, Sec. 3.2.3,
or from free-surface Dirichlet branches, Sec. 3.7.5):

  diagonal(beta, sigma, bc, h)      diagonal of -A_g
  active(beta, sigma, bc, h)        cells with a positive diagonal
  apply_gen(beta, sigma, bc, h, x)  A_g x
  solve_gen(beta, sigma, bc, h, rhs, tol)
                                    A_g p = rhs on the active cells (Jacobi CG)
  project_gen(beta, bc, h, dt, us, p)
                                    eq. fotm with closed links held at u = 0
  divergence_gen(beta, u, bc, h, scale)
                                    D u with closed links carrying no flux

`dense` holds the brute-force dense solve used on tiny grids.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pp_oracle.c")
_LIB = os.path.join(_HERE, "libpp_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("PP_ORACLE_LIB")  # a mutated build, for the mutation tests
        if path is None:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64P = ctypes.POINTER(ctypes.c_int64)
        IP = ctypes.POINTER(ctypes.c_int)
        D = ctypes.c_double
        lib.ppo_face_coeffs.argtypes = [I64P, IP, P, P, P, P]
        lib.ppo_face_coeffs.restype = None
        lib.ppo_divergence.argtypes = [I64P, IP, D, P, P, P, D, P]
        lib.ppo_divergence.restype = None
        lib.ppo_apply.argtypes = [I64P, IP, D, P, P, P, P, P]
        lib.ppo_apply.restype = None
        lib.ppo_project.argtypes = [I64P, IP, D, D, P, P, P, P, P, P, P, P, P, P]
        lib.ppo_project.restype = None
        lib.ppo_rbsor.argtypes = [I64P, IP, D, P, P, P, P, P, D, ctypes.c_int, D, ctypes.c_int,
                                  ctypes.POINTER(D)]
        lib.ppo_rbsor.restype = ctypes.c_int
        lib.ppo_solve.argtypes = [I64P, IP, D, P, P, P, P, P, D, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(D)]
        lib.ppo_solve.restype = ctypes.c_int
        lib.ppo_adjoint.argtypes = [I64P, IP, D, P, P, P, P, P, D, ctypes.c_int, P, P, P, P,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(D)]
        lib.ppo_adjoint.restype = ctypes.c_int
        lib.ppo_apply_gen.argtypes = [I64P, IP, D, P, P, P, P, P, P]
        lib.ppo_apply_gen.restype = None
        lib.ppo_solve_gen.argtypes = [I64P, IP, D, P, P, P, P, P, P, D, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(D)]
        lib.ppo_solve_gen.restype = ctypes.c_int
        lib.ppo_threads.argtypes = []
        lib.ppo_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().ppo_threads())


def set_threads(n: int) -> None:
    """Run later oracle calls (from this Python thread) on n OpenMP threads."""
    lib = _load()
    lib.ppo_set_threads.argtypes = [ctypes.c_int]
    lib.ppo_set_threads.restype = None
    lib.ppo_set_threads(int(n))


def _grid(shape, bc):
    nz, ny, nx = shape
    n = (ctypes.c_int64 * 3)(nx, ny, nz)
    b = (ctypes.c_int * 3)(*[int(v) for v in bc])
    return n, b


def _c(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def face_coeffs(rho: np.ndarray, bc: Sequence[int]) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    rho = _c(rho)
    n, b = _grid(rho.shape, bc)
    out = [np.empty_like(rho) for _ in range(3)]
    _load().ppo_face_coeffs(n, b, _p(rho), _p(out[0]), _p(out[1]), _p(out[2]))
    return out[0], out[1], out[2]


def divergence(u, bc, h: float, scale: float = 1.0) -> np.ndarray:
    ux, uy, uz = (_c(v) for v in u)
    n, b = _grid(ux.shape, bc)
    out = np.empty_like(ux)
    _load().ppo_divergence(n, b, h, _p(ux), _p(uy), _p(uz), scale, _p(out))
    return out


def apply(beta, bc, h: float, x: np.ndarray) -> np.ndarray:
    bx, by, bz = (_c(v) for v in beta)
    x = _c(x)
    n, b = _grid(x.shape, bc)
    y = np.empty_like(x)
    _load().ppo_apply(n, b, h, _p(bx), _p(by), _p(bz), _p(x), _p(y))
    return y


def project(beta, bc, h: float, dt: float, us, p: np.ndarray):
    bx, by, bz = (_c(v) for v in beta)
    usx, usy, usz = (_c(v) for v in us)
    p = _c(p)
    n, b = _grid(p.shape, bc)
    u = [np.empty_like(p) for _ in range(3)]
    _load().ppo_project(n, b, h, dt, _p(bx), _p(by), _p(bz), _p(usx), _p(usy), _p(usz), _p(p),
                        _p(u[0]), _p(u[1]), _p(u[2]))
    return u[0], u[1], u[2]


def rbsor(beta, bc, h: float, rhs: np.ndarray, p0: np.ndarray = None, omega: float = 1.3,
          sweeps: int = 100000, tol: float = 0.0, first_colour: int = 0):
    """The paper's red-black SOR; returns (p, sweeps_done, rel_residual).

    rhs is used as given; remove its mean first for a consistent system.
    first_colour 0 updates red ((i+j+k) even) first, as the paper does.
    """
    bx, by, bz = (_c(v) for v in beta)
    rhs = _c(rhs)
    p = np.zeros_like(rhs) if p0 is None else _c(p0).copy()
    n, b = _grid(rhs.shape, bc)
    rel = ctypes.c_double(0.0)
    s = _load().ppo_rbsor(n, b, h, _p(bx), _p(by), _p(bz), _p(rhs), _p(p), omega, sweeps, tol,
                          int(first_colour), ctypes.byref(rel))
    return p, s, rel.value


def solve(beta, bc, h: float, rhs: np.ndarray, tol: float = 1e-13, maxit: int = 5000,
          p0: np.ndarray = None, check: bool = True):
    """Mean-zero p with A p = rhs - mean(rhs); returns (p, iterations, rel_residual)."""
    bx, by, bz = (_c(v) for v in beta)
    rhs = _c(rhs)
    p = np.zeros_like(rhs) if p0 is None else _c(p0).copy()
    n, b = _grid(rhs.shape, bc)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = _load().ppo_solve(n, b, h, _p(bx), _p(by), _p(bz), _p(rhs), _p(p), tol, maxit,
                           ctypes.byref(it), ctypes.byref(rel))
    if rc < 0:
        raise ValueError("oracle: grid cannot be coarsened to a small enough coarsest level")
    if check and rc != 0:
        raise RuntimeError(f"oracle solve did not reach tol={tol}: rel={rel.value:.3e} "
                           f"after {it.value} iterations")
    return p, it.value, rel.value


def adjoint(beta, bc, h: float, p: np.ndarray, gp: np.ndarray, tol: float = 1e-13,
            maxit: int = 5000):
    """Returns (g_rhs, (g_bx, g_by, g_bz), iterations, rel_residual) for L = <gp, p>."""
    bx, by, bz = (_c(v) for v in beta)
    p = _c(p)
    gp = _c(gp)
    n, b = _grid(p.shape, bc)
    grhs = np.empty_like(p)
    gb = [np.empty_like(p) for _ in range(3)]
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = _load().ppo_adjoint(n, b, h, _p(bx), _p(by), _p(bz), _p(p), _p(gp), tol, maxit,
                             _p(grhs), _p(gb[0]), _p(gb[1]), _p(gb[2]), ctypes.byref(it),
                             ctypes.byref(rel))
    if rc != 0:
        raise RuntimeError(f"oracle adjoint solve did not reach tol={tol}: rel={rel.value:.3e}")
    return grhs, tuple(gb), it.value, rel.value


def rhs_from_velocity(us, bc, h: float, dt: float) -> np.ndarray:
    """b = D u* / dt with its mean removed (eq. poisson right-hand side)."""
    b = divergence(us, bc, h, 1.0 / dt)
    return b - b.mean()


# ---------------------------------------------------------------------------
# general operator: closed links, diagonal term, excluded cells
# ---------------------------------------------------------------------------

def _sig(sigma, shape):
    return None if sigma is None else _c(np.broadcast_to(np.asarray(sigma, dtype=np.float64), shape))


def apply_gen(beta, sigma, bc, h: float, x: np.ndarray) -> np.ndarray:
    """A_g x = A x - sigma x (sigma None means 0)."""
    bx, by, bz = (_c(v) for v in beta)
    x = _c(x)
    sg = _sig(sigma, x.shape)
    n, b = _grid(x.shape, bc)
    y = np.empty_like(x)
    _load().ppo_apply_gen(n, b, h, _p(bx), _p(by), _p(bz), None if sg is None else _p(sg), _p(x),
                          _p(y))
    return y


def open_faces(beta, bc):
    """Boolean masks of the open faces per direction: non-wall faces with beta > 0."""
    out = []
    for m, bm in enumerate(beta):
        o = np.asarray(bm) > 0.0
        if bc[m] == 1:
            idx = [slice(None)] * 3
            idx[2 - m] = 0
            o = o.copy()
            o[tuple(idx)] = False
        out.append(o)
    return out


def diagonal(beta, sigma, bc, h: float) -> np.ndarray:
    """Diagonal of -A_g: the open face coefficients of each cell / h^2 + sigma."""
    shape = np.asarray(beta[0]).shape
    o = open_faces(beta, bc)
    d = np.zeros(shape)
    for m in range(3):
        ax = 2 - m
        low = np.where(o[m], np.asarray(beta[m], dtype=np.float64), 0.0)
        if bc[m] == 0:
            high = np.roll(low, -1, axis=ax)          # low face of the next cell, wrapped
        else:
            high = np.zeros(shape)
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            src[ax] = slice(1, None)
            dst[ax] = slice(0, -1)
            high[tuple(dst)] = low[tuple(src)]        # the upper wall face is closed
        d += low + high
    d /= h * h
    if sigma is not None:
        d = d + np.broadcast_to(np.asarray(sigma, dtype=np.float64), shape)
    return d


def active(beta, sigma, bc, h: float) -> np.ndarray:
    """Cells with a positive diagonal (an open face or sigma > 0)."""
    return diagonal(beta, sigma, bc, h) > 0.0


def solve_gen(beta, sigma, bc, h: float, rhs: np.ndarray, tol: float = 1e-13,
              maxit: int = 1000000, p0: np.ndarray = None, check: bool = True):
    """A_g p = rhs on the active cells; returns (p, iterations, rel_residual).

    Singular when sigma vanishes on every active cell: then the mean of rhs
    over the active cells is removed and p has zero mean there."""
    bx, by, bz = (_c(v) for v in beta)
    rhs = _c(rhs)
    sg = _sig(sigma, rhs.shape)
    p = np.zeros_like(rhs) if p0 is None else _c(p0).copy()
    n, b = _grid(rhs.shape, bc)
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = _load().ppo_solve_gen(n, b, h, _p(bx), _p(by), _p(bz), None if sg is None else _p(sg),
                               _p(rhs), _p(p), tol, maxit, ctypes.byref(it), ctypes.byref(rel))
    if check and rc != 0:
        raise RuntimeError(f"oracle general solve did not reach tol={tol}: rel={rel.value:.3e} "
                           f"after {it.value} iterations")
    return p, it.value, rel.value


def project_gen(beta, bc, h: float, dt: float, us, p: np.ndarray):
    """eq. fotm on open faces; closed links (beta = 0) and walls carry u = 0
    (the link flags of Sec. 3.8 multiply the velocity)."""
    u = project(beta, bc, h, dt, us, p)
    o = open_faces(beta, bc)
    return tuple(np.where(o[m], u[m], 0.0) for m in range(3))


def divergence_gen(beta, u, bc, h: float, scale: float = 1.0) -> np.ndarray:
    """scale * D u with the velocity on closed links taken as 0 (Sec. 3.8)."""
    o = open_faces(beta, bc)
    return divergence(tuple(np.where(o[m], u[m], 0.0) for m in range(3)), bc, h, scale)
