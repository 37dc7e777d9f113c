"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the property it checks and where it comes from: closed forms of
the discrete operator, the paper's own solver (red-black SOR, Sec. 3.7.1), a
brute-force dense solve, a 1D reduction integrated by cumulative sums, the
discrete Helmholtz-Hodge decomposition, and the adjoint identities.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.dense as dense
from paper_2012_11744_amd import workloads as W

BCS = [(0, 0, 0), (1, 1, 1), (0, 0, 1), (1, 0, 1)]


def _case(n, bc, seed, ratio=1000.0):
    w = W.random_case(n, bc, seed=seed, ratio=ratio)
    beta = oracle.face_coeffs(w.rho, bc)
    return w, beta


def _centres(n, h):
    return (np.arange(n) + 0.5) * h


# --------------------------------------------------------------------------
# P1: operator invariants and the face-by-face assembly
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [(8, 8, 8), (6, 10, 4)])
def test_operator_matches_facewise_assembly(n, bc):
    """The stencil apply equals the matrix assembled face by face (Sec. 3.7.1)."""
    w, beta = _case(n, bc, seed=11)
    A = dense.matrix(beta, bc, w.h)
    x = np.random.default_rng(1).standard_normal(w.shape)
    y = oracle.apply(beta, bc, w.h, x).ravel()
    ref = A @ x.ravel()
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("bc", BCS)
def test_operator_symmetric_nullspace_semidefinite(bc):
    """<Ax,y> = <x,Ay>, A 1 = 0 and x^T A x = -sum_f beta_f (dx_f)^2 / h^2 <= 0."""
    n = (12, 8, 10)
    w, beta = _case(n, bc, seed=12)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(w.shape)
    y = rng.standard_normal(w.shape)
    Ax = oracle.apply(beta, bc, w.h, x)
    Ay = oracle.apply(beta, bc, w.h, y)
    assert abs(np.vdot(Ax, y) - np.vdot(x, Ay)) <= 1e-12 * abs(np.vdot(Ax, y))
    A1 = oracle.apply(beta, bc, w.h, np.ones(w.shape))
    assert np.abs(A1).max() <= 1e-12 * np.abs(Ax).max()
    # energy: sum over faces of beta * (jump)^2 / h^2
    energy = 0.0
    for m in range(3):
        ax = 2 - m
        jump = x - np.roll(x, 1, axis=ax)
        b = beta[m].copy()
        if bc[m] == 1:
            sl = [slice(None)] * 3
            sl[ax] = 0
            b[tuple(sl)] = 0.0
        energy += np.sum(b * jump * jump) / w.h ** 2
    assert np.vdot(x, Ax) <= 0
    assert abs(np.vdot(x, Ax) + energy) <= 1e-12 * energy


def test_face_coeffs_two_phase_block():
    """beta = 2/(rho_L + rho_R) on a face, 0 on wall faces (Sec. 3.7.1, Sec. 3.8)."""
    nz, ny, nx = 4, 4, 6
    rho = np.ones((nz, ny, nx))
    rho[:, :, 3:] = 1000.0
    bx, by, bz = oracle.face_coeffs(rho, (1, 0, 1))
    assert np.all(bx[:, :, 0] == 0.0)                     # x walls
    assert np.allclose(bx[:, :, 1:3], 1.0)
    assert np.allclose(bx[:, :, 3], 2.0 / 1001.0)         # the interface face
    assert np.allclose(bx[:, :, 4:], 1e-3)
    assert np.allclose(by[:, :, :3], 1.0)                 # periodic y: no walls
    assert np.allclose(by[:, :, 3:], 1e-3)
    assert np.all(bz[0] == 0.0)                           # z walls
    # periodic x with the same field: the wrap face between i=5 and i=0
    bxp, _, _ = oracle.face_coeffs(rho, (0, 0, 0))
    assert np.allclose(bxp[:, :, 0], 2.0 / 1001.0)


def test_divergence_closed_form():
    """D of u_x = sin(2 pi x) sampled on the faces x = i h is
    2 cos(2 pi x_c) sin(pi h) / h at the cell centres (eq. cont2)."""
    n = 16
    h = 1.0 / n
    xf = np.arange(n) * h
    ux = np.broadcast_to(np.sin(2 * np.pi * xf), (n, n, n)).copy()
    zero = np.zeros((n, n, n))
    d = oracle.divergence((ux, zero, zero), (0, 0, 0), h)
    exact = 2.0 * np.cos(2 * np.pi * _centres(n, h)) * np.sin(np.pi * h) / h
    assert np.abs(d - exact[None, None, :]).max() <= 1e-12
    # the same field along z, with the z walls: faces 0 are walls and ignored
    uz = np.broadcast_to(np.sin(2 * np.pi * xf)[:, None, None], (n, n, n)).copy()
    uz[0] = 123.0
    d = oracle.divergence((zero, zero, uz), (0, 0, 1), h)
    ref = np.empty(n)
    for k in range(n):
        lo = 0.0 if k == 0 else np.sin(2 * np.pi * k * h)
        hi = 0.0 if k == n - 1 else np.sin(2 * np.pi * (k + 1) * h)
        ref[k] = (hi - lo) / h
    assert np.abs(d - ref[:, None, None]).max() <= 1e-12


# --------------------------------------------------------------------------
# P2: manufactured solution, exact discrete answer
# --------------------------------------------------------------------------

# max|p_h - p| / max|p| = (pi h)^2 / sin^2(pi h) - 1 (closed form, see below)
CLOSED_FORM_ERR = {8: 5.3029e-2, 16: 1.2951e-2, 32: 3.2190e-3, 64: 8.0358e-4}


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (0, 1, 0)])
@pytest.mark.parametrize("n", [8, 16, 32])
def test_manufactured_cosine(n, bc):
    """p = cos 2pi x cos 2pi y cos 2pi z, rho constant: cos(2 pi x_i) at cell
    centres is an eigenvector of the 3-point second difference with
    eigenvalue -4 sin^2(pi h)/h^2, for periodic rows and for Neumann rows
    (its mirror images across x = 0 and x = 1 are equal), so the discrete
    solution of A p_h = -12 pi^2 p / rho is p (pi h)^2 / sin^2(pi h)."""
    rho0 = 3.0
    h = 1.0 / n
    x = _centres(n, h)
    c = np.cos(2 * np.pi * x)
    p = c[None, None, :] * c[None, :, None] * c[:, None, None]
    rho = np.full((n, n, n), rho0)
    beta = oracle.face_coeffs(rho, bc)
    rhs = -12.0 * np.pi ** 2 * p / rho0
    ph, it, rel = oracle.solve(beta, bc, h, rhs, tol=1e-13)
    factor = (np.pi * h) ** 2 / np.sin(np.pi * h) ** 2
    assert np.abs(ph - p * factor).max() <= 1e-11
    err = np.abs(ph - p).max() / np.abs(p).max()
    assert abs(err - (factor - 1.0)) <= 1e-10
    if n in CLOSED_FORM_ERR:
        assert abs(err - CLOSED_FORM_ERR[n]) <= 5e-5 * CLOSED_FORM_ERR[n] + 1e-8


def test_manufactured_second_order_ratio():
    """Halving h divides the error by -> 4 (second-order operator)."""
    errs = []
    for n in (8, 16, 32):
        h = 1.0 / n
        c = np.cos(2 * np.pi * _centres(n, h))
        p = c[None, None, :] * c[None, :, None] * c[:, None, None]
        beta = oracle.face_coeffs(np.ones((n, n, n)), (0, 0, 0))
        ph, _, _ = oracle.solve(beta, (0, 0, 0), h, -12.0 * np.pi ** 2 * p, tol=1e-13)
        errs.append(np.abs(ph - p).max() / np.abs(p).max())
    r1 = errs[0] / errs[1]
    r2 = errs[1] / errs[2]
    assert 4.05 < r1 < 4.15 and 4.0 < r2 < 4.05


# --------------------------------------------------------------------------
# P3: discrete Helmholtz-Hodge decomposition (exact for any beta)
# --------------------------------------------------------------------------

def discrete_curl(psi, bc, h):
    """MAC curl of an edge-centred potential (psi_x, psi_y, psi_z), each stored
    at the low edge of its cell; tangential potential on wall planes is 0."""
    px, py, pz = (a.copy() for a in psi)
    for m in range(3):
        if bc[m] == 1:
            ax = 2 - m
            for comp in range(3):
                if comp == m:
                    continue
                sl = [slice(None)] * 3
                sl[ax] = 0
                (px, py, pz)[comp][tuple(sl)] = 0.0

    def dplus(a, ax):
        return (np.roll(a, -1, axis=ax) - a) / h
    ux = dplus(pz, 1) - dplus(py, 0)
    uy = dplus(px, 0) - dplus(pz, 2)
    uz = dplus(py, 2) - dplus(px, 1)
    return ux, uy, uz


@pytest.mark.parametrize("bc", BCS)
def test_hodge_projection_exact(bc):
    """u* = u_df + dt beta G q with D u_df = 0 projects to u = u_df and
    p = q - mean(q) (eqs. fotm / poisson), at density ratio 1000."""
    n = (16, 12, 8)
    w, beta = _case(n, bc, seed=21)
    rng = np.random.default_rng(3)
    psi = [rng.standard_normal(w.shape) for _ in range(3)]
    udf = discrete_curl(psi, bc, w.h)
    assert np.abs(oracle.divergence(udf, bc, w.h)).max() <= 1e-11
    q = rng.standard_normal(w.shape)
    zero = np.zeros(w.shape)
    # dt beta G q via the oracle's projection of a zero field: u = -dt beta G q
    g = oracle.project(beta, bc, w.h, w.dt, (zero, zero, zero), q)
    us = tuple(udf[m] - g[m] for m in range(3))
    rhs = oracle.rhs_from_velocity(us, bc, w.h, w.dt)
    p, _, _ = oracle.solve(beta, bc, w.h, rhs, tol=1e-13)
    qq = q - q.mean()
    assert np.abs(p - qq).max() <= 1e-9 * np.abs(qq).max()
    u = oracle.project(beta, bc, w.h, w.dt, us, p)
    for m in range(3):
        assert np.abs(u[m] - udf[m]).max() <= 1e-8 * np.abs(udf[m]).max()


def test_hydrostatic_column():
    """rho = rho(z), walls in z, u* = -g dt on interior z faces: the pressure
    balances gravity, p[k] - p[k-1] = -g h (rho[k-1] + rho[k]) / 2, and the
    projected velocity is zero."""
    n = 16
    h = 1.0 / n
    dt = 1e-3
    g = 9.81
    rng = np.random.default_rng(4)
    prof = np.where(rng.uniform(size=n) < 0.5, 1000.0, 1.2)
    rho = np.broadcast_to(prof[:, None, None], (n, n, n)).copy()
    bc = (0, 0, 1)
    beta = oracle.face_coeffs(rho, bc)
    uz = np.full((n, n, n), -g * dt)
    uz[0] = 0.0
    zero = np.zeros((n, n, n))
    rhs = oracle.rhs_from_velocity((zero, zero, uz), bc, h, dt)
    # the rhs lives in the two wall layers and p ~ g rho z is large: the FP64
    # residual floor is a few 1e-13 here
    p, _, _ = oracle.solve(beta, bc, h, rhs, tol=1e-12)
    dp = p[1:, 0, 0] - p[:-1, 0, 0]
    exact = -g * h * (prof[:-1] + prof[1:]) / 2.0
    assert np.abs(dp - exact).max() <= 1e-8 * np.abs(exact).max()
    u = oracle.project(beta, bc, h, dt, (zero, zero, uz), p)
    assert max(np.abs(c).max() for c in u) <= 1e-9


# --------------------------------------------------------------------------
# P4 / P8: dense solve and the paper's red-black SOR
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [(8, 8, 8), (6, 4, 10)])
def test_solve_matches_dense(n, bc):
    """MG-PCG equals the bordered dense solve on tiny grids at ratio 1000."""
    w, beta = _case(n, bc, seed=31)
    rhs = oracle.rhs_from_velocity(w.us, bc, w.h, w.dt)
    pd = dense.solve(beta, bc, w.h, rhs)
    p, _, rel = oracle.solve(beta, bc, w.h, rhs, tol=1e-13)
    assert rel <= 1e-13
    assert np.abs(p - pd).max() <= 1e-11 * np.abs(pd).max()


def test_solve_matches_dense_multilevel():
    """16^3 needs a coarsened hierarchy: checks the V-cycle preconditioned path."""
    bc = (0, 0, 1)
    w, beta = _case((16, 16, 16), bc, seed=32)
    rhs = oracle.rhs_from_velocity(w.us, bc, w.h, w.dt)
    pd = dense.solve(beta, bc, w.h, rhs)
    p, it, rel = oracle.solve(beta, bc, w.h, rhs, tol=1e-13)
    assert it > 1
    assert np.abs(p - pd).max() <= 1e-10 * np.abs(pd).max()


@pytest.mark.parametrize("bc", BCS)
def test_paper_rb_sor_matches_dense(bc):
    """The paper's GS with over-relaxation 1.3 (eq. beta_pressure, red first)
    converges to the dense solution: our operator is its A1..A7 system."""
    w, beta = _case((8, 8, 8), bc, seed=41, ratio=10.0)
    rhs = oracle.rhs_from_velocity(w.us, bc, w.h, w.dt)
    pd = dense.solve(beta, bc, w.h, rhs)
    p, sweeps, rel = oracle.rbsor(beta, bc, w.h, rhs, omega=1.3, tol=1e-13)
    assert rel <= 1e-13 and sweeps < 100000
    p = p - p.mean()
    assert np.abs(p - pd).max() <= 1e-10 * np.abs(pd).max()


@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("omega", [1.0, 1.3])
def test_rb_sor_single_sweep_by_hand(omega, first):
    """One sweep of eq. beta_pressure, red first, checked against a direct loop
    over cells of the face-assembled matrix."""
    n = (4, 4, 4)
    bc = (0, 1, 0)
    w, beta = _case(n, bc, seed=42, ratio=50.0)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(w.shape)
    p0 = rng.standard_normal(w.shape)
    p1, _, _ = oracle.rbsor(beta, bc, w.h, rhs, p0=p0, omega=omega, sweeps=1, first_colour=first)
    A = dense.matrix(beta, bc, w.h)
    ref = p0.ravel().copy()
    nz, ny, nx = w.shape
    for colour in (first, 1 - first):
        for c in range(nz * ny * nx):
            i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
            if (i + j + k) % 2 != colour:
                continue
            off = A[c] @ ref - A[c, c] * ref[c]
            ref[c] = (1 - omega) * ref[c] + omega * (rhs.ravel()[c] - off) / A[c, c]
    assert np.abs(p1.ravel() - ref).max() <= 1e-13 * np.abs(ref).max()


# --------------------------------------------------------------------------
# P5: 1D reduction, integrated in closed form
# --------------------------------------------------------------------------

def _solve_1d(beta_f, b, h, periodic):
    """Flux form: F_{i+1/2} - F_{i-1/2} = h b_i, F = beta (p_{i+1} - p_i)/h.
    Walls: F_{-1/2} = 0.  Periodic: the constant flux makes p periodic.
    beta_f[i] is the coefficient of the face between cells i-1 and i."""
    n = b.size
    S = np.cumsum(h * b)                  # F_{i+1/2} - F_{-1/2}
    up = np.roll(beta_f, -1)              # face i+1/2 for i = 0..n-1
    if periodic:
        F0 = -np.sum(h * S / up) / np.sum(h / up)
    else:
        F0 = 0.0
    F = F0 + S                            # F_{i+1/2}
    p = np.zeros(n)
    for i in range(n - 1):
        p[i + 1] = p[i] + h * F[i] / up[i]
    return p - p.mean()


@pytest.mark.parametrize("bcx", [0, 1])
def test_one_dimensional_reduction(bcx):
    """beta_x and b depend on x only (beta_y, beta_z arbitrary): the 3D
    solution is the 1D flux-integrated solution in every row."""
    nx, ny, nz = 32, 6, 4
    h = 1.0 / nx
    rng = np.random.default_rng(6)
    rho_x = np.where(rng.uniform(size=nx) < 0.5, 1000.0, 1.0)
    rho = np.broadcast_to(rho_x[None, None, :], (nz, ny, nx)).copy()
    bc = (bcx, 0, 1)
    bx, by, bz = oracle.face_coeffs(rho, bc)
    by = by * rng.uniform(0.5, 2.0, by.shape)   # arbitrary transverse beta
    bz = bz * rng.uniform(0.5, 2.0, bz.shape)
    b1 = rng.standard_normal(nx)
    b1 -= b1.mean()
    rhs = np.broadcast_to(b1[None, None, :], (nz, ny, nx)).copy()
    # p swings by ~1/beta_min across the heavy cells: the FP64 residual floor
    # is ~1e-12 here
    p, _, _ = oracle.solve((bx, by, bz), bc, h, rhs, tol=1e-11)
    p1 = _solve_1d(bx[0, 0, :], b1, h, periodic=(bcx == 0))
    assert np.abs(p - p1[None, None, :]).max() <= 1e-9 * np.abs(p1).max()


# --------------------------------------------------------------------------
# P6: projection identity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bc", BCS)
def test_projection_identity(bc):
    """D u = D u* - dt A p for any p, so D u = dt (b - A p) with b = D u*/dt."""
    w, beta = _case((10, 8, 12), bc, seed=51)
    p = np.random.default_rng(7).standard_normal(w.shape)
    u = oracle.project(beta, bc, w.h, w.dt, w.us, p)
    lhs = oracle.divergence(u, bc, w.h)
    rhs = oracle.divergence(w.us, bc, w.h) - w.dt * oracle.apply(beta, bc, w.h, p)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()
    for m in range(3):
        if bc[m] == 1:
            sl = [slice(None)] * 3
            sl[2 - m] = 0
            assert np.all(u[m][tuple(sl)] == 0.0)


# --------------------------------------------------------------------------
# P7: adjoint
# --------------------------------------------------------------------------

def test_adjoint_dot_product():
    """<w, S b> = <S w, b>: the solve operator is self-adjoint."""
    bc = (0, 1, 0)
    w, beta = _case((16, 8, 8), bc, seed=61)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(w.shape)
    b -= b.mean()
    g = rng.standard_normal(w.shape)
    g -= g.mean()
    Sb, _, _ = oracle.solve(beta, bc, w.h, b)
    Sg, _, _ = oracle.solve(beta, bc, w.h, g)
    assert abs(np.vdot(g, Sb) - np.vdot(Sg, b)) <= 1e-10 * abs(np.vdot(g, Sb))


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1)])
def test_adjoint_finite_differences(bc):
    """Central differences of L = <w, p> in rhs entries and in face betas."""
    w, beta = _case((8, 8, 8), bc, seed=62, ratio=100.0)
    rhs = oracle.rhs_from_velocity(w.us, bc, w.h, w.dt)
    p, _, _ = oracle.solve(beta, bc, w.h, rhs)
    grhs, gbeta, _, _ = oracle.adjoint(beta, bc, w.h, p, w.w)
    rng = np.random.default_rng(9)

    def loss(rhs_, beta_):
        pp, _, _ = oracle.solve(beta_, bc, w.h, rhs_, tol=1e-14, check=False)
        return np.vdot(w.w, pp)

    d = 1e-6 * np.sqrt(np.mean(rhs ** 2))
    for _ in range(6):
        c = tuple(rng.integers(0, s) for s in w.shape)
        rp = rhs.copy(); rp[c] += d
        rm = rhs.copy(); rm[c] -= d
        fd = (loss(rp, beta) - loss(rm, beta)) / (2 * d)
        assert abs(fd - grhs[c]) <= 1e-6 * np.abs(grhs).max()
    for _ in range(6):
        m = int(rng.integers(0, 3))
        c = tuple(rng.integers(0, s) for s in w.shape)
        if bc[m] == 1 and c[2 - m] == 0:
            assert gbeta[m][c] == 0.0
            continue
        bp = [b.copy() for b in beta]; bp[m][c] += 1e-6
        bm = [b.copy() for b in beta]; bm[m][c] -= 1e-6
        fd = (loss(rhs, bp) - loss(rhs, bm)) / 2e-6
        assert abs(fd - gbeta[m][c]) <= 1e-5 * np.abs(gbeta[m]).max()


def test_adjoint_constant_density_closed_form():
    """rho = 1, w = the cosine eigenvector: lambda = w h^2 / (-12 sin^2(pi h))
    ... i.e. lambda = A^-1 w in closed form, and g_beta = G lambda * G p."""
    n = 16
    h = 1.0 / n
    c = np.cos(2 * np.pi * _centres(n, h))
    wv = c[None, None, :] * c[None, :, None] * c[:, None, None]
    beta = oracle.face_coeffs(np.ones((n, n, n)), (0, 0, 0))
    lam_exact = wv * h * h / (-12.0 * np.sin(np.pi * h) ** 2)
    p = np.random.default_rng(10).standard_normal((n, n, n))
    grhs, gb, _, _ = oracle.adjoint(beta, (0, 0, 0), h, p, wv)
    assert np.abs(grhs - lam_exact).max() <= 1e-11 * np.abs(lam_exact).max()
    for m in range(3):
        ax = 2 - m
        gl = (lam_exact - np.roll(lam_exact, 1, axis=ax)) / h
        gp = (p - np.roll(p, 1, axis=ax)) / h
        assert np.abs(gb[m] - gl * gp).max() <= 1e-9 * np.abs(gl * gp).max()


def test_solve_ignores_rhs_mean():
    """The system is only solvable for mean-zero data; the solve removes the
    mean of the right-hand side, so adding a constant changes nothing."""
    bc = (1, 1, 0)
    w, beta = _case((8, 12, 8), bc, seed=71)
    rhs = oracle.rhs_from_velocity(w.us, bc, w.h, w.dt)
    p1, _, _ = oracle.solve(beta, bc, w.h, rhs)
    p2, _, _ = oracle.solve(beta, bc, w.h, rhs + 1234.5)
    assert abs(p1.mean()) <= 1e-12 * np.abs(p1).max()
    assert np.abs(p1 - p2).max() <= 1e-10 * np.abs(p1).max()
