"""GPU parity for the general operator A x - sigma x (pp_setup_general) against
the oracle, through the C ABI.

Closed links (Sec. 3.8 link flags), a diagonal term (Sec. 3.2.3 implicit
viscous step; Sec. 3.7.5 free-surface Dirichlet branches) and excluded cells.
Tolerances follow test_gpu_parity: single passes are the same FP64 arithmetic
in another order (relative 1e-13); solves are checked through the oracle's own
FP64 residual of the GPU answer and against the oracle's solution or a
discretely exact one.
"""
import sys

import numpy as np
import pytest

import oracle
from general_cases import bubble_dirichlet_case, close_links_of, mode, rand_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRECISIONS = ["fp64", "fp32", "fp16"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_2012_11744_amd import solver
    return solver


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def rel_res(beta, sigma, bc, h, rhs, p):
    """The oracle's FP64 residual of p for A_g p = rhs on the active cells
    (rhs mean over them removed when sigma vanishes)."""
    act = oracle.active(beta, sigma, bc, h)
    b = np.where(act, rhs, 0.0)
    if sigma is None or not np.any(np.broadcast_to(sigma, rhs.shape)[act] > 0):
        b = np.where(act, b - b[act].mean(), 0.0)
    r = np.where(act, b - oracle.apply_gen(beta, sigma, bc, h, p), 0.0)
    return np.linalg.norm(r) / np.linalg.norm(b)


GRIDS = [((8, 8, 8), (0, 0, 0)), ((40, 20, 56), (1, 0, 1)), ((48, 36, 24), (1, 1, 1))]


@pytest.mark.parametrize("n,bc", GRIDS)
def test_apply_divergence_project_general(S, n, bc):
    """Single passes with closed links and sigma against the oracle."""
    _say(f"general apply/div/project n={n} bc={bc}")
    shape = (n[2], n[1], n[0])
    beta, sigma = rand_case(shape, bc, 11)
    h, dt = 1.0 / n[0], 1e-3
    rng = np.random.default_rng(12)
    x = rng.standard_normal(shape)
    us = [rng.uniform(-1, 1, shape) for _ in range(3)]
    with S.Solver([dev(b) for b in beta], h, bc, precision="fp64", sigma=dev(sigma)) as sol:
        y = host(sol.apply(dev(x)))
        d = host(sol.divergence([dev(u) for u in us], 1.0 / dt))
        u = [host(c) for c in sol.project([dev(u) for u in us], dev(x), dt)]
    assert relmax(y, oracle.apply_gen(beta, sigma, bc, h, x)) <= 1e-13
    assert relmax(d, oracle.divergence_gen(beta, us, bc, h, 1.0 / dt)) <= 1e-13
    ref = oracle.project_gen(beta, bc, h, dt, us, x)
    for m in range(3):
        assert relmax(u[m], ref[m]) <= 1e-14
        assert np.all(u[m][~oracle.open_faces(beta, bc)[m]] == 0.0)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("n,bc", GRIDS)
def test_solve_general_nonsingular(S, n, bc, precision):
    """Random closed links and sigma (one cell held only by sigma, one
    excluded cell): the GPU answer against the oracle's."""
    _say(f"general solve (sigma) n={n} bc={bc} {precision}")
    shape = (n[2], n[1], n[0])
    beta, sigma = rand_case(shape, bc, 21, frac_closed=0.1)
    sigma = sigma * 400.0                  # a diagonal of the size of the link terms
    h = 1.0 / n[0]
    rhs = np.random.default_rng(22).standard_normal(shape)
    p_o, it, rel = oracle.solve_gen(beta, sigma, bc, h, rhs, tol=1e-13)
    with S.Solver([dev(b) for b in beta], h, bc, precision=precision, sigma=dev(sigma)) as sol:
        p = host(sol.solve(dev(rhs), tol=1e-11))
    assert rel_res(beta, sigma, bc, h, rhs, p) <= 1.05e-11
    assert relmax(p, p_o) <= 1e-8
    assert p[2, 2, 3] == 0.0


@pytest.mark.parametrize("precision", PRECISIONS)
def test_solve_general_singular_solid(S, precision):
    """sigma absent, a solid block with its links closed: singular on the
    fluid cells; the solve removes the rhs mean there and returns a mean-zero
    p; solid cells are excluded; the projection is divergence-free on the
    fluid and zero on the closed links."""
    _say(f"general solve (solid) {precision}")
    shape, bc = (24, 20, 32), (0, 1, 1)
    h, dt = 1.0 / 32, 1e-3
    rng = np.random.default_rng(31)
    beta = [rng.uniform(0.05, 1.0, shape) for _ in range(3)]
    solid = np.zeros(shape, dtype=bool)
    solid[6:15, 5:13, 8:20] = True
    close_links_of(beta, solid, bc)
    us = [rng.uniform(-1, 1, shape) for _ in range(3)]
    b = oracle.divergence_gen(beta, us, bc, h, 1.0 / dt)
    p_o, it, rel = oracle.solve_gen(beta, None, bc, h, b, tol=1e-13)
    with S.Solver([dev(x) for x in beta], h, bc, precision=precision, general=True) as sol:
        usd = [dev(u) for u in us]
        bd = sol.divergence(usd, 1.0 / dt)
        p = sol.solve(bd, tol=1e-11)
        u = [host(c) for c in sol.project(usd, p, dt)]
        p = host(p)
    assert rel_res(beta, None, bc, h, b, p) <= 1.05e-11
    assert relmax(p, p_o) <= 1e-8
    assert np.all(p[solid] == 0.0)
    assert abs(p[~solid].mean()) <= 1e-12 * np.abs(p).max()
    div = oracle.divergence_gen(beta, u, bc, h)
    scale = np.abs(oracle.divergence_gen(beta, us, bc, h)).max()
    assert np.abs(div[~solid]).max() <= 1e-8 * scale
    for m in range(3):
        assert np.all(u[m][~oracle.open_faces(beta, bc)[m]] == 0.0)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_free_surface_dirichlet_exact_on_gpu(S, precision):
    """The bubble case of the oracle pins on the GPU: the solution is the
    linear pressure at every liquid cell (the discretisation is exact)."""
    _say(f"bubble Dirichlet branches {precision}")
    h = 1.0 / 16
    bc, beta, sigma, rhs, pe, gas = bubble_dirichlet_case(h=h)
    with S.Solver([dev(b) for b in beta], h, bc, precision=precision, sigma=dev(sigma)) as sol:
        p = host(sol.solve(dev(rhs), tol=1e-12))
    assert np.abs(p - pe)[~gas].max() / np.abs(pe).max() <= 1e-9
    assert np.all(p[gas] == 0.0)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_helmholtz_eigenmode_and_viscous_step_128(S, precision):
    """128^3 (fused sweeps with the diagonal term): a Laplacian eigenmode
    under the implicit viscous step is damped by 1 / (1 + tau mu |lam|)."""
    _say(f"implicit viscous step 128^3 {precision}")
    shape, bc = (128, 128, 128), (0, 1, 0)
    h, tau, mu = 1.0 / 128, 1e-3, 0.05
    v, lam = mode(shape, bc, (3, 2, 5))
    ones = dev(np.ones(shape))
    sig = dev(np.full(shape, 1.0 / (tau * mu)))
    with S.Solver([ones, ones, ones], h, bc, precision=precision, sigma=sig) as sol:
        u = host(sol.solve(dev(-v / (tau * mu)), tol=1e-11))
        it = sol.last_stats["outer_iters"]
    expect = v / (1.0 + tau * mu * abs(lam) / (h * h))
    _say(f"  {it} iterations")
    assert relmax(u, expect) <= 1e-9


def test_general_solid_and_sigma_128(S):
    """128^3 mixed FP32 with closed links and a variable sigma: the oracle's
    FP64 residual of the GPU answer at the solve tolerance."""
    _say("general 128^3 fp32")
    shape, bc = (128, 128, 128), (1, 0, 1)
    h = 1.0 / 128
    rng = np.random.default_rng(41)
    beta = [rng.uniform(0.01, 1.0, shape) for _ in range(3)]
    solid = np.zeros(shape, dtype=bool)
    solid[40:70, 30:90, 50:100] = True
    close_links_of(beta, solid, bc)
    sigma = rng.uniform(0.0, 50.0, shape)
    sigma[solid] = 0.0
    rhs = rng.standard_normal(shape)
    with S.Solver([dev(b) for b in beta], h, bc, precision="fp32", sigma=dev(sigma)) as sol:
        p = host(sol.solve(dev(rhs), tol=1e-10))
        it = sol.last_stats["outer_iters"]
    _say(f"  {it} iterations")
    assert rel_res(beta, sigma, bc, h, rhs, p) <= 1.05e-10
    assert np.all(p[solid] == 0.0)


def test_general_update_warm_start_and_graph(S):
    """update_general replaces beta and sigma in place; a warm start with
    garbage on excluded cells ignores it; the graph-replayed coarse cycle
    gives the same bits as the eager one."""
    _say("general update / warm start / graph")
    n, bc = (40, 20, 56), (1, 0, 1)
    shape = (n[2], n[1], n[0])
    h = 1.0 / n[0]
    beta, sigma = rand_case(shape, bc, 51, frac_closed=0.1)
    beta2, sigma2 = rand_case(shape, bc, 52, frac_closed=0.1)
    sigma, sigma2 = sigma * 300.0, sigma2 * 300.0
    rhs = np.random.default_rng(53).standard_normal(shape)
    bt = [dev(b) for b in beta]
    with S.Solver(bt, h, bc, precision="fp32", sigma=dev(sigma), warm_start=True) as sol:
        p0 = torch.zeros(shape, dtype=torch.float64, device="cuda")
        p0[2, 2, 3] = float("nan")                     # an excluded cell
        pa = host(sol.solve(dev(rhs), tol=1e-11, p=p0))
        assert rel_res(beta, sigma, bc, h, rhs, pa) <= 1.05e-11
        assert pa[2, 2, 3] == 0.0
        sol.update_coeffs([dev(b) for b in beta2], dev(sigma2))
        pb = host(sol.solve(dev(rhs), tol=1e-11, p=torch.zeros_like(p0)))
        assert rel_res(beta2, sigma2, bc, h, rhs, pb) <= 1.05e-11
    # graph vs eager coarse cycle: same kernels in the same order, same bits
    with S.Solver(bt, h, bc, precision="fp32", sigma=dev(sigma)) as g, \
            S.Solver(bt, h, bc, precision="fp32", sigma=dev(sigma), coarse_graph=False) as e:
        pg = host(g.solve(dev(rhs), tol=1e-9))
        pe = host(e.solve(dev(rhs), tol=1e-9))
        assert np.array_equal(pg, pe)


def test_general_adjoint(S):
    """The adjoint of the general solve: lambda solves A_g lambda = g_p;
    g_beta = G lambda . G p on open faces and 0 on closed links and walls;
    dL/d sigma = lambda p checked by a central difference along a direction."""
    _say("general adjoint")
    n, bc = (24, 16, 20), (0, 1, 1)
    shape = (n[2], n[1], n[0])
    h = 1.0 / n[0]
    beta, sigma = rand_case(shape, bc, 61, frac_closed=0.1)
    sigma = sigma * 200.0
    rng = np.random.default_rng(62)
    rhs = rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    with S.Solver([dev(b) for b in beta], h, bc, precision="fp64", sigma=dev(sigma)) as sol:
        p = sol.solve(dev(rhs), tol=1e-13)
        lam, gb = sol.adjoint(p, dev(w), tol=1e-13)
        ph, lh = host(p), host(lam)
        gbh = [host(g) for g in gb]
    lam_o, _, _ = oracle.solve_gen(beta, sigma, bc, h, w, tol=1e-14)
    assert relmax(lh, lam_o) <= 1e-9
    opened = oracle.open_faces(beta, bc)
    for m in range(3):
        ax = 2 - m
        ref = (lh - np.roll(lh, 1, axis=ax)) * (ph - np.roll(ph, 1, axis=ax)) / (h * h)
        ref = np.where(opened[m], ref, 0.0)
        assert relmax(gbh[m], ref) <= 1e-12
    # dL/d sigma_c = lambda_c p_c, along a random direction on active cells
    act = oracle.active(beta, sigma, bc, h)
    dsg = rng.uniform(0.0, 1.0, shape) * (sigma > 0)
    eps = 1e-4 * sigma.max()
    vals = []
    for sgn in (1, -1):
        p2, _, _ = oracle.solve_gen(beta, sigma + sgn * eps * dsg, bc, h, rhs, tol=1e-14)
        vals.append(float(np.vdot(w, p2)))
    fd = (vals[0] - vals[1]) / (2 * eps)
    ad = float(np.sum(lh * ph * dsg))
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    assert np.all(lh[~act] == 0.0)


def test_general_rejects_bad_coefficients(S):
    from paper_2012_11744_amd import _lib as L
    shape, bc = (8, 8, 8), (0, 0, 0)
    h = 1.0 / 8
    ones = [dev(np.ones(shape)) for _ in range(3)]
    bad = np.ones(shape)
    bad[3, 3, 3] = -1.0
    with pytest.raises(L.PPError, match="non-negative"):
        S.Solver([dev(bad), ones[1], ones[2]], h, bc, general=True)
    sg = np.ones(shape)
    sg[1, 2, 3] = float("nan")
    with pytest.raises(L.PPError, match="sigma"):
        S.Solver(ones, h, bc, sigma=dev(sg))
    zero = [dev(np.zeros(shape)) for _ in range(3)]
    with pytest.raises(L.PPError, match="no cell"):
        S.Solver(zero, h, bc, general=True)
    with S.Solver(ones, h, bc, sigma=dev(np.ones(shape))) as sol:
        with pytest.raises(L.PPError, match="sigma must be given"):
            sol.update_coeffs(ones)
    with S.Solver(ones, h, bc, general=True) as sol:
        with pytest.raises(L.PPError, match="sigma must be NULL"):
            sol.update_coeffs(ones, dev(np.ones(shape)))
