"""pp_update_density: face coefficients computed from the cell densities
together with the hierarchy rebuild (GPU, through the C ABI).

beta = 2 / (rho_L + rho_R) is the interpolation of pp_face_coeffs (pinned
against the oracle's face coefficients in test_gpu_parity), so the density
path must load the same coefficients bit for bit: the tests compare whole
solves and projections with those of pp_face_coeffs + pp_update_coeffs
bitwise, on the one-pass kernel (aligned rho, several levels) and on the
fallback path (a single-level grid; a misaligned rho), and check that bad
densities are rejected.  After a density update the search direction's
image and the projection form beta from a copy of rho instead of reading the
three coefficient arrays; the bitwise comparisons cover them, and
further tests check that the copy is the library's own (the caller may
overwrite rho), that a later coefficient update stops its use, that z
chunks which do not divide the grid wrap correctly, and the adjoint.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2012_11744_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _two_ways(S, w, precision, rho_t):
    """(p, u) from face_coeffs + update_coeffs and from update_density, on
    one context each, after a first update with unrelated coefficients."""
    out = []
    beta0 = S.face_coeffs(dev(np.full(w.shape, 3.0)), w.h, w.bc)
    us = [dev(u) for u in w.us]
    for mode in ("beta", "rho"):
        with S.Solver(beta0, w.h, w.bc, precision=precision) as sol:
            if mode == "beta":
                sol.update_coeffs(S.face_coeffs(rho_t, w.h, w.bc))
            else:
                sol.update_density(rho_t)
            b = sol.divergence(us, 1.0 / w.dt)
            p = sol.solve(b, tol=1e-10)
            u = sol.project(us, p, w.dt)
            out.append((host(p).copy(), [host(c).copy() for c in u],
                        sol.last_stats["outer_iters"]))
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp16"])
def test_density_update_matches_face_coeffs_bitwise(S, precision):
    w = W.config3(64)
    _say(f"density update config3 64^3 {precision}")
    (p1, u1, i1), (p2, u2, i2) = _two_ways(S, w, precision, dev(w.rho))
    assert i1 == i2
    assert np.array_equal(p1, p2)
    for a, b in zip(u1, u2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,bc", [((40, 20, 56), (1, 0, 1)), ((48, 36, 24), (1, 1, 1))])
def test_density_update_ragged_and_misaligned(S, n, bc):
    """Ragged grids with walls; then rho handed as a view one element into a
    larger buffer (8-byte aligned only): the fallback path, same bits."""
    w = W.random_case(n, bc, seed=131, ratio=1000.0)
    _say(f"density update n={n} bc={bc}")
    (p1, u1, _), (p2, u2, _) = _two_ways(S, w, "fp32", dev(w.rho))
    assert np.array_equal(p1, p2)
    big = torch.empty(w.rho.size + 1, dtype=torch.float64, device="cuda")
    big[1:] = dev(w.rho).reshape(-1)
    view = big[1:].view(w.shape)
    assert view.data_ptr() % 16 == 8
    (p3, u3, _), (p4, u4, _) = _two_ways(S, w, "fp32", view)
    assert np.array_equal(p3, p1) and np.array_equal(p4, p1)
    for a, b in zip(u1, u4):
        assert np.array_equal(a, b)


def test_density_update_single_level(S):
    """A 4^3 grid has one level: the fallback path (face coefficients, then
    the separate checks)."""
    n, bc = (4, 4, 4), (0, 1, 0)
    w = W.random_case(n, bc, seed=132, ratio=100.0)
    (p1, _, _), (p2, _, _) = _two_ways(S, w, "fp64", dev(w.rho))
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("bad", [-1.0, 0.0, float("nan"), float("inf")])
def test_density_update_rejects_bad_rho(S, bad):
    from paper_2012_11744_amd import _lib as L
    w = W.config3(32)
    rho = w.rho.copy()
    rho[3, 5, 7] = bad
    beta = S.face_coeffs(dev(w.rho), w.h, w.bc)
    with S.Solver(beta, w.h, w.bc) as sol:
        with pytest.raises(L.PPError):
            sol.update_density(dev(rho))
        # a later good update recovers the context
        sol.update_density(dev(w.rho))
        p = sol.solve(sol.divergence([dev(u) for u in w.us], 1.0 / w.dt), tol=1e-8)
        assert np.isfinite(host(p)).all()
    # fallback path (misaligned) rejects it too
    big = torch.empty(rho.size + 1, dtype=torch.float64, device="cuda")
    big[1:] = dev(rho).reshape(-1)
    with S.Solver(beta, w.h, w.bc) as sol:
        with pytest.raises(L.PPError):
            sol.update_density(big[1:].view(w.shape))


def test_density_update_refused_for_general_context(S):
    from paper_2012_11744_amd import _lib as L
    w = W.config3(32)
    beta = S.face_coeffs(dev(w.rho), w.h, w.bc)
    with S.Solver(beta, w.h, w.bc, general=True) as sol:
        with pytest.raises((L.PPError, ValueError)):
            sol.update_density(dev(w.rho))


@pytest.mark.parametrize("n,bc", [((36, 28, 20), (0, 0, 0)), ((40, 24, 28), (0, 1, 1)),
                                  ((10, 10, 9), (0, 1, 0))])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_density_update_partial_z_chunks(S, n, bc, precision):
    """nz not a multiple of the 8-plane column walk of the outer kernels, with
    periodic z (the carried plane below wraps) and walls; nz = 9 takes the
    fallback load (one level) and its copy of rho."""
    w = W.random_case(n, bc, seed=133, ratio=500.0)
    _say(f"density update partial z chunks n={n} bc={bc} {precision}")
    (p1, u1, i1), (p2, u2, i2) = _two_ways(S, w, precision, dev(w.rho))
    assert i1 == i2
    assert np.array_equal(p1, p2)
    for a, b in zip(u1, u2):
        assert np.array_equal(a, b)


def test_density_copy_is_owned_and_dropped_by_coefficient_update(S):
    """The library keeps its own copy of rho: overwriting the caller's tensor
    after the update changes nothing.  A later pp_update_coeffs makes the
    stored coefficients the operator again (the copy of rho is stale)."""
    w = W.config3(32)
    us = [dev(u) for u in w.us]
    beta_a = S.face_coeffs(dev(w.rho), w.h, w.bc)
    rho_b = np.where(w.rho > 500.0, 2.0, 700.0)
    beta_b = S.face_coeffs(dev(rho_b), w.h, w.bc)

    def solve_with(setup):
        with S.Solver(beta_a, w.h, w.bc, precision="fp32") as sol:
            setup(sol)
            b = sol.divergence(us, 1.0 / w.dt)
            return host(sol.solve(b, tol=1e-10)).copy()

    p_a = solve_with(lambda sol: sol.update_coeffs(beta_a))
    p_b = solve_with(lambda sol: sol.update_coeffs(beta_b))

    def overwrite(sol):
        r = dev(w.rho)
        sol.update_density(r)
        r.fill_(5.0)
        torch.cuda.synchronize()

    assert np.array_equal(solve_with(overwrite), p_a)
    assert np.array_equal(
        solve_with(lambda sol: (sol.update_density(dev(w.rho)), sol.update_coeffs(beta_b))), p_b)
    assert np.array_equal(
        solve_with(lambda sol: (sol.update_coeffs(beta_b), sol.update_density(dev(w.rho)))), p_a)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_density_update_adjoint_bitwise(S, precision):
    """The adjoint solve runs the same outer kernels: g_rhs and g_beta agree
    bit for bit between the two ways of loading the coefficients."""
    w = W.random_case((40, 24, 32), (1, 0, 1), seed=134, ratio=1000.0)
    us = [dev(u) for u in w.us]
    g = dev(np.random.default_rng(135).standard_normal(w.shape))
    beta0 = S.face_coeffs(dev(np.full(w.shape, 3.0)), w.h, w.bc)
    outs = []
    for mode in ("beta", "rho"):
        with S.Solver(beta0, w.h, w.bc, precision=precision) as sol:
            if mode == "beta":
                sol.update_coeffs(S.face_coeffs(dev(w.rho), w.h, w.bc))
            else:
                sol.update_density(dev(w.rho))
            p = sol.solve(sol.divergence(us, 1.0 / w.dt), tol=1e-10)
            g_rhs, g_b = sol.adjoint(p, g, tol=1e-10)
            outs.append([host(g_rhs).copy()] + [host(t).copy() for t in g_b])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
