"""pp_step: the whole projection step in one call (GPU, through the C ABI).

The call chains the density load, the divergence, the solve and the
projection with the same kernels in the same order as the four separate
calls, and only moves the density check's read-back to the solve's first
wait, so its results must equal theirs bit for bit: p, u, the right-hand
side and the iteration count, over several steps (each rebuilds the
hierarchy and the coarsest pseudo-inverse), in every precision, with a warm
start and with u written in place over u*.  A rejected density is reported
by the step, and a later good step recovers the context.
"""
import sys

import numpy as np
import pytest

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
    return t.detach().cpu().numpy().copy()


def _densities(w, steps):
    """the workload's density, then shifted copies of it (a moving interface)"""
    return [np.roll(w.rho, 3 * s, axis=0) for s in range(steps)]


def _run(S, w, precision, mode, steps=3, warm=False, in_place=False):
    beta0 = S.face_coeffs(dev(np.full(w.shape, 2.0)), w.h, w.bc)
    res = []
    with S.Solver(beta0, w.h, w.bc, precision=precision, warm_start=warm) as sol:
        p = torch.zeros(w.shape, dtype=torch.float64, device="cuda")
        rhs = torch.empty_like(p)
        for rho in _densities(w, steps):
            rho_t = dev(rho)
            us = [dev(u) for u in w.us]
            out = us if in_place else [torch.empty_like(p) for _ in range(3)]
            if mode == "calls":
                sol.update_density(rho_t)
                sol.divergence(us, 1.0 / w.dt, out=rhs)
                sol.solve(rhs, tol=1e-9, p=p)
                sol.project(us, p, w.dt, out=out)
            else:
                sol.step(rho_t, us, w.dt, tol=1e-9, p=p, rhs=rhs, out=out)
            res.append((host(p), host(rhs), [host(c) for c in out],
                        sol.last_stats["outer_iters"], sol.last_stats["rel_res"]))
    return res


def _same(a, b):
    for (p1, r1, u1, i1, e1), (p2, r2, u2, i2, e2) in zip(a, b):
        assert i1 == i2 and e1 == e2
        assert np.array_equal(r1, r2)
        assert np.array_equal(p1, p2)
        for x, y in zip(u1, u2):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp16"])
def test_step_matches_four_calls_bitwise(S, precision):
    w = W.config3(64)
    _say(f"step config3 64^3 {precision}")
    a = _run(S, w, precision, "calls")
    b = _run(S, w, precision, "step")
    assert all(np.isfinite(x[0]).all() for x in a)
    _same(a, b)


@pytest.mark.parametrize("n,bc", [((40, 20, 56), (1, 0, 1)), ((48, 36, 24), (1, 1, 1))])
def test_step_ragged_warm_in_place(S, n, bc):
    w = W.random_case(n, bc, seed=141, ratio=1000.0)
    _say(f"step ragged n={n} bc={bc} warm, in place")
    _same(_run(S, w, "fp32", "calls", warm=True, in_place=True),
          _run(S, w, "fp32", "step", warm=True, in_place=True))


@pytest.mark.parametrize("bad", [0.0, float("nan")])
def test_step_rejects_bad_density_then_recovers(S, bad):
    from paper_2012_11744_amd import _lib as L
    w = W.config3(32)
    rho = w.rho.copy()
    rho[5, 6, 7] = bad
    beta = S.face_coeffs(dev(w.rho), w.h, w.bc)
    us = [dev(u) for u in w.us]
    _say(f"step bad density {bad}")
    with S.Solver(beta, w.h, w.bc) as sol:
        with pytest.raises(L.PPError, match="rho"):
            sol.step(dev(rho), us, w.dt, tol=1e-8)
        p, u = sol.step(dev(w.rho), us, w.dt, tol=1e-8)
        got = (host(p), [host(c) for c in u])
    with S.Solver(beta, w.h, w.bc) as sol:
        p, u = sol.step(dev(w.rho), us, w.dt, tol=1e-8)
        want = (host(p), [host(c) for c in u])
    assert np.array_equal(got[0], want[0])
    for x, y in zip(got[1], want[1]):
        assert np.array_equal(x, y)


def test_step_rejects_aliasing_and_general_contexts(S):
    from paper_2012_11744_amd import _lib as L
    w = W.config3(32)
    beta = S.face_coeffs(dev(w.rho), w.h, w.bc)
    rho = dev(w.rho)
    us = [dev(u) for u in w.us]
    t = [torch.empty_like(rho) for _ in range(5)]
    P = S._ptr
    with S.Solver(beta, w.h, w.bc) as sol:
        lib = sol._lib

        def call(rhs, p, u, dt=w.dt, tol=1e-8):
            return lib.pp_step(sol._ctx, P(rho), *(P(v) for v in us), dt, tol, P(rhs), P(p),
                               *(P(v) for v in u), None)
        assert call(t[0], t[0], t[2:5]) == L.PP_EINVAL          # rhs = p
        assert call(t[0], t[1], [t[1], t[3], t[4]]) == L.PP_EINVAL   # p = u_x
        assert call(us[0], t[1], t[2:5]) == L.PP_EINVAL         # rhs = us_x
        assert call(t[0], t[1], [us[1], t[3], t[4]]) == L.PP_EINVAL  # u_x = us_y
        assert call(t[0], t[1], t[2:5], dt=0.0) == L.PP_EINVAL
        assert call(t[0], t[1], t[2:5], tol=1.0) == L.PP_EINVAL
        assert call(t[0], t[1], [us[0], us[1], us[2]]) == L.PP_OK   # u in place over u*
    with S.Solver(beta, w.h, w.bc, general=True) as sol:
        with pytest.raises(ValueError):
            sol.step(rho, us, w.dt)
        rc = sol._lib.pp_step(sol._ctx, P(rho), *(P(v) for v in us), w.dt, 1e-8, P(t[0]),
                              P(t[1]), *(P(v) for v in t[2:5]), None)
        assert rc == L.PP_EINVAL and "general" in sol._lib.pp_last_error().decode()
