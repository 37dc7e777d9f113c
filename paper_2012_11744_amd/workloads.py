"""Seeded synthetic inputs for the pressure-projection step.

This module only *draws* inputs: a cell density field, staggered predicted
velocities u* and (for gradient checks) a loss weight field.  It holds none of
the projection method's arithmetic (no face coefficients, no divergence, no
solve); both the HIP path and the CPU oracle receive the same arrays from here
and compute everything else on their own.

Layout (shared by every consumer):
  * cell arrays have shape (nz, ny, nx), C order, x fastest;
  * a face array for direction m has the same shape; entry c is the *low*
    face of cell c in direction m (position c - e_m/2);
  * in a wall direction the entry with c_m == 0 is the wall face; its normal
    velocity is 0.  The upper wall face is implicit.

Density fields follow the one-fluid law (rho = rho_l C + rho_g (1 - C), Sec. 2.1
eq. muH) with C the liquid volume fraction obtained by the "subgrid" lego
initialisation of Sec. 3.5.3: each cell is split into n_I^3 sub-cells and C is
the fraction of sub-cell centres that lie in the liquid.  Cells far from every
interface are uniform and are filled from the cell-centre test; only cells in
a band around an interface are sub-sampled (the band is wide enough that the
result equals sub-sampling every cell, which a test checks on small grids).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

PERIODIC = 0
WALL = 1

N_SUB = 4  # sub-cells per direction for the volume fractions


@dataclasses.dataclass
class Workload:
    name: str
    n: Tuple[int, int, int]          # (nx, ny, nz)
    bc: Tuple[int, int, int]         # per direction: PERIODIC or WALL
    h: float
    dt: float
    tol: float
    rho: np.ndarray                  # (nz, ny, nx) float64 cell densities
    us: Tuple[np.ndarray, np.ndarray, np.ndarray]  # u*_x, u*_y, u*_z faces
    w: Optional[np.ndarray] = None   # loss weights for L = sum(w * p)
    rho_l: float = 1.0
    rho_g: float = 1.0
    liquid_fraction: Optional[np.ndarray] = None
    geometry: Optional[dict] = None  # the drawn shapes, for checking the fractions

    @property
    def shape(self) -> Tuple[int, int, int]:
        nx, ny, nz = self.n
        return (nz, ny, nx)

    @property
    def cells(self) -> int:
        nx, ny, nz = self.n
        return nx * ny * nz


# ---------------------------------------------------------------------------
# geometry: each piece is described by a function inside(x, y, z) -> bool array
# and a conservative band test on cell centres.
# ---------------------------------------------------------------------------

def _centres(n: int, h: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def _sub_offsets(h: float) -> np.ndarray:
    """Offsets of the N_SUB sub-cell centres from a cell's low corner."""
    return (np.arange(N_SUB, dtype=np.float64) + 0.5) * (h / N_SUB)


def _bits_for_cells(idx_k, idx_j, idx_i, h, inside: Callable) -> np.ndarray:
    """64-bit masks of sub-cell centres inside a region, for the listed cells.

    Bit s of the mask is sub-cell s = (sk*N_SUB + sj)*N_SUB + si.
    """
    assert N_SUB ** 3 == 64
    off = _sub_offsets(h)
    masks = np.zeros(idx_k.shape[0], dtype=np.uint64)
    x0 = idx_i * h
    y0 = idx_j * h
    z0 = idx_k * h
    bit = 0
    for sk in range(N_SUB):
        z = z0 + off[sk]
        for sj in range(N_SUB):
            y = y0 + off[sj]
            for si in range(N_SUB):
                x = x0 + off[si]
                ins = inside(x, y, z)
                masks |= ins.astype(np.uint64) << np.uint64(bit)
                bit += 1
    return masks


def _periodic_delta(d: np.ndarray, length: float, periodic: bool) -> np.ndarray:
    if not periodic:
        return d
    return d - length * np.round(d / length)


class _Spheres:
    """Union of balls; minimum-image distances in periodic directions."""

    def __init__(self, centres, radii, box, periodic):
        self.c = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
        self.r = np.asarray(radii, dtype=np.float64).reshape(-1)
        self.box = box
        self.per = periodic

    def cells_near(self, n, h):
        """Per ball: cell index ranges covering the ball plus a 2-cell margin."""
        out = []
        nx, ny, nz = n
        for (cx, cy, cz), r in zip(self.c, self.r):
            rng = []
            for cval, nn, per in ((cx, nx, self.per[0]), (cy, ny, self.per[1]), (cz, nz, self.per[2])):
                lo = int(math.floor((cval - r) / h)) - 2
                hi = int(math.floor((cval + r) / h)) + 2
                idx = np.arange(lo, hi + 1)
                if per:
                    idx = np.unique(np.mod(idx, nn))
                else:
                    idx = idx[(idx >= 0) & (idx < nn)]
                rng.append(idx)
            out.append(rng)
        return out

    def inside_one(self, b):
        cx, cy, cz = self.c[b]
        r = self.r[b]
        Lx, Ly, Lz = self.box
        px, py, pz = self.per

        def f(x, y, z):
            dx = _periodic_delta(x - cx, Lx, px)
            dy = _periodic_delta(y - cy, Ly, py)
            dz = _periodic_delta(z - cz, Lz, pz)
            return dx * dx + dy * dy + dz * dz < r * r
        return f


def _union_masks(n, h, spheres: _Spheres):
    """Return (linear cell index, 64-bit mask) for cells touched by any ball."""
    nx, ny, nz = n
    all_idx = []
    all_mask = []
    for b, (ii, jj, kk) in enumerate(spheres.cells_near(n, h)):
        K, J, I = np.meshgrid(kk, jj, ii, indexing="ij")
        K = K.ravel()
        J = J.ravel()
        I = I.ravel()
        m = _bits_for_cells(K, J, I, h, spheres.inside_one(b))
        keep = m != 0
        all_idx.append((K[keep] * ny + J[keep]) * nx + I[keep])
        all_mask.append(m[keep])
    if not all_idx:
        return np.zeros(0, np.int64), np.zeros(0, np.uint64)
    idx = np.concatenate(all_idx).astype(np.int64)
    msk = np.concatenate(all_mask)
    order = np.argsort(idx, kind="stable")
    idx = idx[order]
    msk = msk[order]
    if idx.size == 0:
        return idx, msk
    starts = np.flatnonzero(np.r_[True, idx[1:] != idx[:-1]])
    return idx[starts], np.bitwise_or.reduceat(msk, starts)


def _fraction_from_masks(masks: np.ndarray) -> np.ndarray:
    return np.bitwise_count(masks).astype(np.float64) / 64.0


def _level_set_fraction(n, h, phi_centre: Callable, inside: Callable, band: float) -> np.ndarray:
    """Liquid fraction of the region inside(x,y,z), sub-sampled in a band.

    phi_centre(x, y, z) must be negative inside and Lipschitz with a constant
    L such that |phi| > band guarantees a whole cell lies on one side.
    """
    nx, ny, nz = n
    C = np.empty((nz, ny, nx), dtype=np.float64)
    xc = _centres(nx, h)
    yc = _centres(ny, h)
    for k in range(nz):
        z = (k + 0.5) * h
        X, Y = np.meshgrid(xc, yc, indexing="xy")
        phi = phi_centre(X, Y, np.full_like(X, z))
        plane = (phi < 0).astype(np.float64)
        near = np.abs(phi) <= band
        if near.any():
            jj, ii = np.nonzero(near)
            kk = np.full_like(jj, k)
            plane[jj, ii] = _fraction_from_masks(_bits_for_cells(kk, jj, ii, h, inside))
        C[k] = plane
    return C


# ---------------------------------------------------------------------------
# velocities
# ---------------------------------------------------------------------------

def _draw_velocities(rng, n, bc) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    nx, ny, nz = n
    shape = (nz, ny, nx)
    us = [rng.uniform(-1.0, 1.0, shape) for _ in range(3)]
    # axis m of a (nz,ny,nx) array is 2 - m
    for m in range(3):
        if bc[m] == WALL:
            sl = [slice(None)] * 3
            sl[2 - m] = 0
            us[m][tuple(sl)] = 0.0
    return us[0], us[1], us[2]


def _density(C, rho_l, rho_g):
    return rho_l * C + rho_g * (1.0 - C)


# ---------------------------------------------------------------------------
# the five workloads (sizes can be overridden for small parity cases)
# ---------------------------------------------------------------------------

def config1(N: int = 32) -> Workload:
    """Periodic cube, one liquid sphere R=0.25 (rho 10) in gas (rho 1), seed 0."""
    n = (N, N, N)
    h = 1.0 / N
    bc = (PERIODIC,) * 3
    rng = np.random.default_rng(0)
    sph = _Spheres([[0.5, 0.5, 0.5]], [0.25], (1.0, 1.0, 1.0), (True, True, True))
    idx, msk = _union_masks(n, h, sph)
    C = np.zeros(N ** 3)
    C[idx] = _fraction_from_masks(msk)
    C = C.reshape(N, N, N)
    us = _draw_velocities(rng, n, bc)
    return Workload("sphere-periodic", n, bc, h, 1e-3, 1e-10, _density(C, 10.0, 1.0), us,
                    rho_l=10.0, rho_g=1.0, liquid_fraction=C)


def config2(N: int = 128) -> Workload:
    """Walled cube of liquid (rho 1000) with 20 gas bubbles (rho 1), seed 1."""
    n = (N, N, N)
    h = 1.0 / N
    bc = (WALL,) * 3
    rng = np.random.default_rng(1)
    centres = rng.uniform(0.15, 0.85, (20, 3))
    radii = rng.uniform(0.05, 0.15, 20)
    sph = _Spheres(centres, radii, (1.0, 1.0, 1.0), (False, False, False))
    idx, msk = _union_masks(n, h, sph)
    gas = np.zeros(N ** 3)
    gas[idx] = _fraction_from_masks(msk)
    C = 1.0 - gas.reshape(N, N, N)
    ux, uy, uz = _draw_velocities(rng, n, bc)
    dt = 1e-3
    uz[1:, :, :] -= 9.81 * dt  # gravity on every interior z face
    return Workload("bubbles-walls", n, bc, h, dt, 1e-8, _density(C, 1000.0, 1.0), (ux, uy, uz),
                    rho_l=1000.0, rho_g=1.0, liquid_fraction=C,
                    geometry={"centres": centres, "radii": radii})


def _layer_phi(x, y, z):
    return z - (0.5 + 0.05 * np.sin(2.0 * np.pi * x / 0.25))


def config3(N: int = 256, rho_l: float = 1000.0, rho_g: float = 1.2) -> Workload:
    """Liquid layer with a sinusoidal surface plus 200 droplets in gas, seed 2.

    Periodic in x and y, walls in z.  rho_l=10 gives the low-ratio variant.
    """
    n = (N, N, N)
    h = 1.0 / N
    bc = (PERIODIC, PERIODIC, WALL)
    rng = np.random.default_rng(2)
    u = rng.uniform(0.0, 1.0, (200, 3))
    centres = np.empty_like(u)
    centres[:, 0] = u[:, 0]
    centres[:, 1] = u[:, 1]
    centres[:, 2] = 0.58 + (0.97 - 0.58) * u[:, 2]
    radii = rng.uniform(0.01, 0.03, 200)
    # the layer: |d phi| <= sqrt(1 + (0.05*2pi/0.25)^2) ~ 1.61 per unit length
    lip = math.sqrt(1.0 + (0.05 * 2.0 * math.pi / 0.25) ** 2)
    band = lip * 0.87 * h * 1.5
    C = _level_set_fraction(n, h, _layer_phi, lambda x, y, z: _layer_phi(x, y, z) < 0, band)
    sph = _Spheres(centres, radii, (1.0, 1.0, 1.0), (True, True, False))
    idx, msk = _union_masks(n, h, sph)
    if idx.size:
        kk = idx // (N * N)
        jj = (idx // N) % N
        ii = idx % N
        layer_bits = _bits_for_cells(kk, jj, ii, h, lambda x, y, z: _layer_phi(x, y, z) < 0)
        Cf = C.reshape(-1)
        Cf[idx] = _fraction_from_masks(msk | layer_bits)
    us = _draw_velocities(rng, n, bc)
    return Workload("layer-droplets" if rho_l == 1000.0 else "layer-droplets-lowratio", n, bc, h,
                    1e-3, 1e-8, _density(C, rho_l, rho_g), us, rho_l=rho_l, rho_g=rho_g,
                    liquid_fraction=C, geometry={"centres": centres, "radii": radii})


def config4(N: int = 64) -> Workload:
    """Periodic cube, one drop R=0.25 (rho 100) in gas (rho 1), seed 3, with weights."""
    n = (N, N, N)
    h = 1.0 / N
    bc = (PERIODIC,) * 3
    rng = np.random.default_rng(3)
    sph = _Spheres([[0.5, 0.5, 0.5]], [0.25], (1.0, 1.0, 1.0), (True, True, True))
    idx, msk = _union_masks(n, h, sph)
    C = np.zeros(N ** 3)
    C[idx] = _fraction_from_masks(msk)
    C = C.reshape(N, N, N)
    us = _draw_velocities(rng, n, bc)
    w = rng.uniform(-1.0, 1.0, (N, N, N))
    return Workload("drop-adjoint", n, bc, h, 1e-3, 1e-8, _density(C, 100.0, 1.0), us, w=w,
                    rho_l=100.0, rho_g=1.0, liquid_fraction=C)


def _jet_params(rng):
    k = rng.integers(1, 9, 5)
    nmode = rng.integers(0, 3, 5)
    ph = rng.uniform(0.0, 2.0 * np.pi, 5)
    return k, nmode, ph


def _jet_radius(x, theta, k, nmode, ph):
    r = np.full_like(x, 0.1)
    for m in range(5):
        r = r + 0.01 * np.cos(2.0 * np.pi * k[m] * x + nmode[m] * theta + ph[m])
    return r


def config5(N: int = 512) -> Workload:
    """Walled cube with a perturbed liquid jet along x (rho 800) in gas (rho 1), seed 4."""
    n = (N, N, N)
    h = 1.0 / N
    bc = (WALL,) * 3
    rng = np.random.default_rng(4)
    k, nmode, ph = _jet_params(rng)

    def phi(x, y, z):
        dy = y - 0.5
        dz = z - 0.5
        rr = np.sqrt(dy * dy + dz * dz)
        th = np.arctan2(dz, dy)
        return rr - _jet_radius(x, th, k, nmode, ph)

    # Lipschitz bound: radial 1, axial sum 0.01*2*pi*k <= 2.52, angular
    # sum 0.01*n / r <= 0.1 / 0.05 near the surface (r >= 0.05)
    band = math.sqrt(1.0 + 2.52 ** 2 + 2.0 ** 2) * 0.87 * h * 1.5
    C = _level_set_fraction(n, h, phi, lambda x, y, z: phi(x, y, z) < 0, band)
    us = _draw_velocities(rng, n, bc)
    w = rng.uniform(-1.0, 1.0, (N, N, N))
    return Workload("jet-walls", n, bc, h, 1e-3, 1e-8, _density(C, 800.0, 1.0), us, w=w,
                    rho_l=800.0, rho_g=1.0, liquid_fraction=C,
                    geometry={"k": k, "n": nmode, "phase": ph})


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def make(config: int, N: Optional[int] = None, **kw) -> Workload:
    """Build one of the five workloads, optionally at a reduced size N."""
    f = CONFIGS[config]
    return f(**kw) if N is None else f(N, **kw)


# ---------------------------------------------------------------------------
# generic random cases for parity tests (any shape, any boundary mix)
# ---------------------------------------------------------------------------

def random_case(n: Sequence[int], bc: Sequence[int], seed: int, ratio: float = 1000.0,
                h: Optional[float] = None, blobs: int = 6, dt: float = 1e-3) -> Workload:
    """Random blobs of heavy fluid in light fluid on an (nx, ny, nz) grid.

    Densities are 1 (light) and `ratio` (heavy); the blob boundaries are
    sub-sampled like the named workloads.  u* is uniform[-1, 1] with wall
    faces set to 0, and w is uniform[-1, 1].
    """
    nx, ny, nz = (int(v) for v in n)
    if h is None:
        h = 1.0 / max(nx, ny, nz)
    rng = np.random.default_rng(seed)
    box = (nx * h, ny * h, nz * h)
    centres = rng.uniform(0.0, 1.0, (blobs, 3)) * np.array(box)
    radii = rng.uniform(0.08, 0.25, blobs) * min(box)
    per = tuple(b == PERIODIC for b in bc)
    sph = _Spheres(centres, radii, box, per)
    idx, msk = _union_masks((nx, ny, nz), h, sph)
    C = np.zeros(nx * ny * nz)
    C[idx] = _fraction_from_masks(msk)
    C = C.reshape(nz, ny, nx)
    us = _draw_velocities(rng, (nx, ny, nz), tuple(bc))
    w = rng.uniform(-1.0, 1.0, (nz, ny, nx))
    return Workload(f"random-{nx}x{ny}x{nz}", (nx, ny, nz), tuple(bc), h, dt, 1e-10,
                    _density(C, ratio, 1.0), us, w=w, rho_l=ratio, rho_g=1.0, liquid_fraction=C,
                    geometry={"centres": centres, "radii": radii})


def brute_force_fraction(n, h, inside: Callable) -> np.ndarray:
    """Sub-sample every cell (slow; for checking the banded generators)."""
    nx, ny, nz = n
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = _bits_for_cells(K.ravel(), J.ravel(), I.ravel(), h, inside)
    return _fraction_from_masks(m).reshape(nz, ny, nx)
