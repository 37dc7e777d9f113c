"""Brute-force dense solve of the pressure system on tiny grids (TEST INFRASTRUCTURE).

The matrix is assembled face by face, straight from the finite-volume
statement of Sec. 3.7.1: every non-wall face f between cells L and R with
coefficient beta_f contributes the flux beta_f (p_R - p_L) / h^2 to row R
with a minus sign and to row L with a plus sign... written out below as the
four matrix entries of a graph Laplacian.  Walls contribute no face
(Sec. 3.8: the link coefficient is zeroed).

The singular system (constants in the null space) is solved through the
bordered matrix [[A, 1], [1^T, 0]] [p; mu] = [b - mean(b); 0], which fixes
mean(p) = 0, with numpy's LAPACK-backed dense solver.
"""
from __future__ import annotations

import numpy as np


def faces(shape, bc):
    """Yield (direction m, low cell index L, high cell index R) for every
    non-wall face of an (nz, ny, nx) grid; the face is stored at entry R."""
    nz, ny, nx = shape
    n = (nx, ny, nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                R = (k * ny + j) * nx + i
                ijk = [i, j, k]
                for m in range(3):
                    q = list(ijk)
                    q[m] -= 1
                    if q[m] < 0:
                        if bc[m] == 1:
                            continue
                        q[m] += n[m]
                    L = (q[2] * ny + q[1]) * nx + q[0]
                    yield m, L, R


def matrix(beta, bc, h):
    """Dense A with (A p)_c = sum over faces of c of beta_f (p_other - p_c) / h^2."""
    shape = beta[0].shape
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    flat = [np.asarray(b, dtype=np.float64).reshape(-1) for b in beta]
    for m, L, R in faces(shape, bc):
        w = flat[m][R] / (h * h)
        A[R, R] -= w
        A[R, L] += w
        A[L, L] -= w
        A[L, R] += w
    return A


def solve(beta, bc, h, rhs):
    """Mean-zero p with A p = rhs - mean(rhs), by the bordered dense system."""
    A = matrix(beta, bc, h)
    N = A.shape[0]
    b = np.asarray(rhs, dtype=np.float64).reshape(-1)
    b = b - b.mean()
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = A
    M[:N, N] = 1.0
    M[N, :N] = 1.0
    x = np.linalg.solve(M, np.concatenate([b, [0.0]]))
    return x[:N].reshape(beta[0].shape)


def matrix_gen(beta, sigma, bc, h):
    """Dense A_g = A - diag(sigma): faces as in `matrix` (a closed link has
    beta = 0 and adds nothing), the diagonal term straight from its definition."""
    A = matrix(beta, bc, h)
    if sigma is not None:
        sg = np.broadcast_to(np.asarray(sigma, dtype=np.float64), beta[0].shape).reshape(-1)
        A[np.diag_indices_from(A)] -= sg
    return A


def solve_gen(beta, sigma, bc, h, rhs):
    """A_g p = rhs restricted to the active cells (nonzero diagonal of A_g);
    excluded cells get 0.  If sigma vanishes on the active cells the system
    is singular: the bordered system fixes the mean of p over the active
    cells to 0 after removing the mean of rhs there."""
    A = matrix_gen(beta, sigma, bc, h)
    act = np.abs(np.diag(A)) > 0.0
    idx = np.nonzero(act)[0]
    Aa = A[np.ix_(idx, idx)]
    b = np.asarray(rhs, dtype=np.float64).reshape(-1)[idx]
    sg = (np.zeros(A.shape[0]) if sigma is None else
          np.broadcast_to(np.asarray(sigma, dtype=np.float64), beta[0].shape).reshape(-1))
    out = np.zeros(A.shape[0])
    if np.all(sg[idx] == 0.0):
        b = b - b.mean()
        n = len(idx)
        M = np.zeros((n + 1, n + 1))
        M[:n, :n] = Aa
        M[:n, n] = 1.0
        M[n, :n] = 1.0
        out[idx] = np.linalg.solve(M, np.concatenate([b, [0.0]]))[:n]
    else:
        out[idx] = np.linalg.solve(Aa, b)
    return out.reshape(beta[0].shape)
