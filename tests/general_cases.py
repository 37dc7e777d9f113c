"""Seeded inputs for the general operator A x - sigma x (test infrastructure).

These build what a caller of the library builds: face coefficients with
closed links, a diagonal term, and for the free-surface case the Dirichlet
branches of the pressure discretisation (Sec. 3.7.5, eq. mod_branches) with
a matching right-hand side.  Both the oracle pins and the GPU tests use them;
they call neither side.
"""
import math

import numpy as np


def rand_case(shape, bc, seed, frac_closed=0.2, frac_sigma=0.5):
    """Random beta in [0.5, 2] with a fraction of closed links, sigma >= 0 on a
    fraction of the cells, one cell held only by sigma (every link closed) at
    (1, 1, 1) and one excluded cell (every link closed, sigma 0) at (2, 2, 3)."""
    rng = np.random.default_rng(seed)
    beta = [rng.uniform(0.5, 2.0, shape) for _ in range(3)]
    for m in range(3):
        beta[m][rng.random(shape) < frac_closed] = 0.0
    sigma = rng.uniform(0.0, 3.0, shape) * (rng.random(shape) < frac_sigma)
    for (k, j, i), sg in (((1, 1, 1), 2.5), ((2, 2, 3), 0.0)):
        beta[0][k, j, i] = 0.0
        beta[0][k, j, (i + 1) % shape[2]] = 0.0
        beta[1][k, j, i] = 0.0
        beta[1][k, (j + 1) % shape[1], i] = 0.0
        beta[2][k, j, i] = 0.0
        beta[2][(k + 1) % shape[0], j, i] = 0.0
        sigma[k, j, i] = sg
    return beta, sigma


def close_links_of(beta, solid, bc):
    """Close every link that touches a solid cell: a link is open only if both
    of its cells are fluid (the product of the two cell flags; a link of Sec.
    3.8 sits between two cells).  Modifies beta in place."""
    for m in range(3):
        ax = 2 - m
        below = np.roll(solid, 1, axis=ax)        # the cell on the low side of the face
        beta[m][solid | below] = 0.0
    return beta


def _sphere_distance(xc, s, m, centre, R):
    """Distance t > 0 from xc along s e_m to the sphere surface."""
    d = np.asarray(xc) - centre
    perp = sum(d[q] ** 2 for q in range(3) if q != m)
    root = math.sqrt(R * R - perp)
    ts = [s * (-d[m] + root), s * (-d[m] - root)]
    return min(t for t in ts if t > 0)


def bubble_dirichlet_case(shape=(16, 20, 24), h=1.0 / 16, centre=(0.71, 0.62, 0.47), R=0.27,
                          g=(0.3, -1.1, 0.7), p0=2.0, beta0=1e-3):
    """Walled box, a spherical gas bubble (cells whose centre is inside are
    excluded) and the linear pressure p = p0 + g.x in the liquid.  A liquid
    cell next to the bubble takes the one-sided gradient (p_s - p_c)/delta to
    the interface: its link is closed, sigma_c += beta/(h delta) and the rhs
    gets -beta p_s/(h delta), p_s being the exact pressure there.  Wall
    fluxes of the linear field enter the rhs as sources.  Every branch is then
    exact for the linear field, so it solves the system.

    Returns (bc, beta, sigma, rhs, p_exact, gas)."""
    nz, ny, nx = shape
    bc = (1, 1, 1)
    centre = np.asarray(centre, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    idx = np.indices(shape)
    X = np.stack([(idx[2] + 0.5) * h, (idx[1] + 0.5) * h, (idx[0] + 0.5) * h], axis=-1)
    gas = np.sum((X - centre) ** 2, axis=-1) < R * R
    beta = close_links_of([np.full(shape, beta0) for _ in range(3)], gas, bc)
    sigma = np.zeros(shape)
    rhs = np.zeros(shape)
    n = (nx, ny, nz)
    exact = lambda x: p0 + float(g @ x)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if gas[k, j, i]:
                    continue
                c = [i, j, k]
                xc = X[k, j, i]
                for m in range(3):
                    for s in (-1, 1):
                        q = list(c)
                        q[m] += s
                        if q[m] < 0 or q[m] >= n[m]:
                            rhs[k, j, i] -= s * beta0 * g[m] / h        # wall flux as a source
                        elif gas[q[2], q[1], q[0]]:
                            t = _sphere_distance(xc, s, m, centre, R)
                            assert 0.0 < t <= h
                            xs = xc.copy()
                            xs[m] += s * t
                            sigma[k, j, i] += beta0 / (h * t)
                            rhs[k, j, i] -= beta0 * exact(xs) / (h * t)
    p_exact = p0 + X @ g
    return bc, beta, sigma, rhs, p_exact, gas


def mode(shape, bc, k):
    """Product of 1D eigenvectors of the unit-coefficient Laplacian: periodic
    cos(2 pi k i / n), walled (Neumann, cell centred) cos(pi k (i + 1/2) / n);
    returns (v, lam) with A v = lam / h^2 v."""
    nz, ny, nx = shape
    n = (nx, ny, nz)
    out = np.ones(shape)
    lam = 0.0
    for m in range(3):
        i = np.arange(n[m])
        if bc[m] == 0:
            v = np.cos(2 * math.pi * k[m] * i / n[m])
            lam -= 4 * math.sin(math.pi * k[m] / n[m]) ** 2
        else:
            v = np.cos(math.pi * k[m] * (i + 0.5) / n[m])
            lam -= 4 * math.sin(math.pi * k[m] / (2 * n[m])) ** 2
        sh = [1, 1, 1]
        sh[2 - m] = n[m]
        out = out * v.reshape(sh)
    return out, lam
