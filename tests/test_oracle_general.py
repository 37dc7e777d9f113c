"""Pins of the oracle's general operator A_g x = A x - sigma x (CPU only).

Closed links (Sec. 3.8: the link flags zero the coefficients of a blocked
link), a diagonal term (Sec. 3.2.3: the implicit viscous step divided by
tau mu; Sec. 3.7.5: Dirichlet branches of the free-surface discretisation)
and excluded cells.  Each pin checks the oracle against something it does not
compute itself: a dense matrix assembled face by face, a closed-form
eigenvalue, a discretely exact solution, or an identity of the projection.
"""
import numpy as np
import pytest

import oracle
from oracle import dense

from general_cases import bubble_dirichlet_case, close_links_of, mode, rand_case


CASES = [((6, 4, 8), (1, 0, 1)), ((4, 6, 6), (0, 0, 0)), ((5, 6, 4), (1, 1, 1))]


@pytest.mark.parametrize("shape,bc", CASES)
def test_apply_gen_matches_dense_assembly(shape, bc):
    beta, sigma = rand_case(shape, bc, 1)
    h = 0.1
    x = np.random.default_rng(2).standard_normal(shape)
    A = dense.matrix_gen(beta, sigma, bc, h)
    ref = (A @ x.reshape(-1)).reshape(shape)
    y = oracle.apply_gen(beta, sigma, bc, h, x)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()
    # the diagonal helper is the dense diagonal, and an excluded cell has none
    assert np.allclose(oracle.diagonal(beta, sigma, bc, h).reshape(-1), -np.diag(A), rtol=1e-14,
                       atol=0.0)
    act = oracle.active(beta, sigma, bc, h)
    assert act[1, 1, 1] and not act[2, 2, 3]


@pytest.mark.parametrize("shape,bc", CASES)
def test_solve_gen_matches_dense_nonsingular(shape, bc):
    beta, sigma = rand_case(shape, bc, 3)
    h = 0.1
    rhs = np.random.default_rng(4).standard_normal(shape)
    p, it, rel = oracle.solve_gen(beta, sigma, bc, h, rhs, tol=1e-13)
    ref = dense.solve_gen(beta, sigma, bc, h, rhs)
    assert np.abs(p - ref).max() <= 1e-10 * np.abs(ref).max()
    assert p[2, 2, 3] == 0.0                      # excluded cell


def test_solve_gen_matches_dense_singular_with_solid():
    """sigma = 0: the constants on the fluid cells span the null space; a solid
    block (every link of its cells closed) is excluded."""
    shape, bc = (6, 6, 8), (0, 1, 0)
    rng = np.random.default_rng(5)
    beta = [rng.uniform(0.5, 2.0, shape) for _ in range(3)]
    solid = np.zeros(shape, dtype=bool)
    solid[2:4, 1:3, 3:6] = True
    close_links_of(beta, solid, bc)
    rhs = rng.standard_normal(shape)
    p, it, rel = oracle.solve_gen(beta, None, bc, 0.2, rhs, tol=1e-13)
    ref = dense.solve_gen(beta, None, bc, 0.2, rhs)
    assert np.abs(p - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(p[solid] == 0.0)
    assert abs(p[~solid].mean()) <= 1e-13 * np.abs(p).max()


@pytest.mark.parametrize("bc", [(0, 1, 0), (1, 1, 1), (0, 0, 0)])
def test_helmholtz_eigenmode_closed_form(bc):
    """Unit coefficients and constant sigma: A_g v = (lam / h^2 - sigma) v for
    every product of 1D eigenvectors, so the solve divides by that number."""
    shape = (8, 12, 16)
    h, s = 1.0 / 16, 37.0
    beta = [np.ones(shape) for _ in range(3)]
    v, lam = mode(shape, bc, (3, 2, 1))
    ev = lam / (h * h) - s
    y = oracle.apply_gen(beta, s, bc, h, v)
    assert np.abs(y - ev * v).max() <= 1e-12 * abs(ev)
    p, it, rel = oracle.solve_gen(beta, s, bc, h, v, tol=1e-13)
    assert np.abs(p - v / ev).max() <= 1e-11 * np.abs(v / ev).max()


def test_implicit_viscous_step_damping():
    """Sec. 3.2.3, eq. muelliptic: U* = U^n + tau mu lap U*.  Divided by
    tau mu it is A_g U* = -U^n / (tau mu) with beta = 1, sigma = 1/(tau mu);
    an eigenmode of the Laplacian is damped by 1 / (1 + tau mu |lam|)."""
    shape, bc = (8, 8, 8), (0, 0, 0)
    h, tau, mu = 1.0 / 8, 1e-3, 2.5
    beta = [np.ones(shape) for _ in range(3)]
    v, lam = mode(shape, bc, (1, 2, 3))
    sig = 1.0 / (tau * mu)
    u, it, rel = oracle.solve_gen(beta, sig, bc, h, -v / (tau * mu), tol=1e-14)
    expect = v / (1.0 + tau * mu * abs(lam) / (h * h))
    assert np.abs(u - expect).max() <= 1e-12


def test_solid_block_projection():
    """Sec. 3.8: with the links of a solid closed, the projected velocity is 0
    on those links and discretely divergence-free on every fluid cell, and the
    solid cells drop out of the pressure system."""
    shape, bc = (12, 12, 12), (0, 0, 1)
    h, dt = 1.0 / 12, 1e-3
    rng = np.random.default_rng(7)
    beta = [rng.uniform(0.001, 1.0, shape) for _ in range(3)]
    solid = np.zeros(shape, dtype=bool)
    solid[3:7, 4:9, 2:6] = True
    close_links_of(beta, solid, bc)
    us = [rng.uniform(-1, 1, shape) for _ in range(3)]
    b = oracle.divergence_gen(beta, us, bc, h, 1.0 / dt)
    p, it, rel = oracle.solve_gen(beta, None, bc, h, b, tol=1e-13)
    u = oracle.project_gen(beta, bc, h, dt, us, p)
    opened = oracle.open_faces(beta, bc)
    for m in range(3):
        assert np.all(u[m][~opened[m]] == 0.0)
    div = oracle.divergence_gen(beta, u, bc, h)
    scale = np.abs(oracle.divergence_gen(beta, us, bc, h)).max()
    assert np.abs(div[~solid]).max() <= 1e-10 * scale
    assert np.all(p[solid] == 0.0)
    # projection identity for any p: D u = D u* - dt A_g p (on every cell)
    q = rng.standard_normal(shape)
    uq = oracle.project_gen(beta, bc, h, dt, us, q)
    lhs = oracle.divergence_gen(beta, uq, bc, h)
    rhs = oracle.divergence_gen(beta, us, bc, h) - dt * oracle.apply_gen(beta, None, bc, h, q)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_free_surface_dirichlet_branches_exact_for_linear_pressure():
    """Sec. 3.7.5, eq. mod_branches: a liquid cell next to an excluded (gas)
    cell takes the gradient (p_s - p_c) / delta to the interface.  In A_g form
    the face's coefficient moves to sigma_c += beta / (h delta) and
    -beta p_s / (h delta) to the right-hand side.  For a linear pressure, with
    its wall fluxes as sources, every branch is exact, so the discrete
    solution is the linear function at every liquid cell centre."""
    h = 1.0 / 16
    bc, beta, sigma, rhs, pe, gas = bubble_dirichlet_case(h=h)
    p, it, rel = oracle.solve_gen(beta, sigma, bc, h, rhs, tol=1e-14)
    err = np.abs(p - pe)[~gas].max() / np.abs(pe).max()
    assert err <= 1e-10
    assert np.all(p[gas] == 0.0)
