"""Parity at the full workload sizes, in the configuration bench.py times.

* 256^3 layer + droplets (density ratio 833): element-wise parity with the
  oracle's converged solution, and the oracle's own FP64 residual of the GPU
  answer at the timing tolerance, for the three V-cycle precisions.
* 512^3 jet (walls, ratio 800), forward and backward: properties that hold at
  any size (oracle residual of the GPU p, projection identity, adjoint
  dot-product identity, the face-product formula on sampled faces) and central
  differences of L = <w, p> along random full-field directions.
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


def rel_res(beta, bc, h, rhs, p):
    b = rhs - rhs.mean()
    return np.linalg.norm(b - oracle.apply(beta, bc, h, p)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def layer256():
    _say("generating the 256^3 layer+droplets workload")
    w = W.config3(256)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    _say("oracle solve at 256^3 (tol 1e-13)")
    p_o, it, rel = oracle.solve(beta, w.bc, w.h, rhs, tol=1e-13)
    _say(f"  oracle: {it} iterations, rel {rel:.2e}")
    return w, beta, rhs, p_o


@pytest.mark.parametrize("precision", ["fp32", "fp64", "fp16"])
def test_layer256_parity(S, layer256, precision):
    w, beta, rhs, p_o = layer256
    _say(f"256^3 {precision}")
    rho = dev(w.rho)
    bt = S.face_coeffs(rho, w.h, w.bc)
    with S.Solver(bt, w.h, w.bc, precision=precision) as sol:
        us = [dev(u) for u in w.us]
        b = sol.divergence(us, 1.0 / w.dt)
        # the timed configuration: tol 1e-8
        p8 = host(sol.solve(b, tol=1e-8)).copy()
        it8 = sol.last_stats["outer_iters"]
        r8 = rel_res(beta, w.bc, w.h, rhs, p8)
        # parity configuration: tol 1e-11
        p11 = sol.solve(b, tol=1e-11)
        u = sol.project(us, p11, w.dt)
        p11h = host(p11)
        uh = [host(c) for c in u]
    err8 = np.abs(p8 - p_o).max() / np.abs(p_o).max()
    err11 = np.abs(p11h - p_o).max() / np.abs(p_o).max()
    u_o = oracle.project(beta, w.bc, w.h, w.dt, w.us, p_o)
    div = oracle.divergence(uh, w.bc, w.h)
    div_o = oracle.divergence(u_o, w.bc, w.h)
    ds = np.abs(oracle.divergence(w.us, w.bc, w.h)).max()
    err_div = np.abs(div - div_o).max() / ds
    err_u = max(np.abs(uh[m] - u_o[m]).max() for m in range(3)) / max(np.abs(c).max() for c in w.us)
    _say(f"  tol 1e-8: {it8} iterations, oracle residual {r8:.2e}, p error {err8:.2e}; "
         f"tol 1e-11: p error {err11:.2e}, div(u) error {err_div:.2e}, u error {err_u:.2e}")
    assert r8 <= 1.05e-8
    # measured 3.3e-8 (FP32 and FP64: 7 iterations, final residual 4.0e-9)
    # and 3.7e-9 (FP16 storage, 8 iterations); the residual tolerance does
    # not bound the p error by itself (condition number ~1e8), so the bound
    # leaves a margin of 3 over the largest measured value
    assert err8 <= 1e-7
    # iteration counts of the timed configuration (measured 7, 7 and 8 with
    # the default over-relaxation): a mistake in a preconditioner kernel, or
    # a smoother that lost its relaxation, shows up here first
    assert it8 <= (9 if precision == "fp16" else 8)
    assert err11 <= 1e-8
    assert err_div <= 1e-8
    assert err_u <= 1e-8


def test_layer256_low_ratio_fp16(S):
    """The same layer and droplets with liquid density 10 (ratio 8.3), where
    FP16 storage of the V-cycle is meant to hold: element-wise parity at tol
    1e-11 and the oracle's FP64 residual of the answer at the timing
    tolerance."""
    _say("generating the 256^3 layer+droplets workload at density ratio 8.3")
    w = W.config3(256, rho_l=10.0)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    _say("oracle solve at 256^3, ratio 8.3 (tol 1e-13)")
    p_o, it_o, rel_o = oracle.solve(beta, w.bc, w.h, rhs, tol=1e-13)
    _say(f"  oracle: {it_o} iterations, rel {rel_o:.2e}")
    rho = dev(w.rho)
    bt = S.face_coeffs(rho, w.h, w.bc)
    with S.Solver(bt, w.h, w.bc, precision="fp16") as sol:
        sol.update_density(rho)
        us = [dev(u) for u in w.us]
        b = sol.divergence(us, 1.0 / w.dt)
        p8 = host(sol.solve(b, tol=1e-8)).copy()
        st8 = dict(sol.last_stats)
        p11 = host(sol.solve(b, tol=1e-11)).copy()
        st11 = dict(sol.last_stats)
    r8 = rel_res(beta, w.bc, w.h, rhs, p8)
    err8 = np.abs(p8 - p_o).max() / np.abs(p_o).max()
    err11 = np.abs(p11 - p_o).max() / np.abs(p_o).max()
    _say(f"  fp16 tol 1e-8: {st8['outer_iters']} iterations (fell back: {st8['fell_back']}), "
         f"oracle residual {r8:.2e}, p error {err8:.2e}; tol 1e-11: {st11['outer_iters']} "
         f"iterations, p error {err11:.2e}")
    assert not st8["fell_back"] and not st11["fell_back"]
    assert r8 <= 1.05e-8
    assert err11 <= 1e-8


@pytest.fixture(scope="module")
def jet512():
    _say("generating the 512^3 jet workload")
    return W.config5(512)


def test_jet512_forward_backward(S, jet512):
    w = jet512
    _say("512^3 forward (mixed FP32, tol 1e-8)")
    rho = dev(w.rho)
    bt = S.face_coeffs(rho, w.h, w.bc)
    with S.Solver(bt, w.h, w.bc, precision="fp32") as sol:
        us = [dev(u) for u in w.us]
        b = sol.divergence(us, 1.0 / w.dt)
        p = sol.solve(b, tol=1e-8)
        it = sol.last_stats["outer_iters"]
        u = sol.project(us, p, w.dt)
        wt = dev(w.w)
        _say("512^3 backward")
        lam, gb = sol.adjoint(p, wt, tol=1e-8)
        ita = sol.last_stats["outer_iters"]
        ph, lh_, bh = host(p), host(lam), host(b)
        uh = [host(c) for c in u]
        gbh = [host(g) for g in gb]
        betah = [host(x) for x in bt]
        del us, u, gb
    _say(f"  forward {it} iterations, backward {ita} iterations")
    rhs = bh
    # oracle residual of the GPU pressure (FP64)
    assert rel_res(betah, w.bc, w.h, rhs, ph) <= 1.05e-8
    assert abs(ph.mean()) <= 1e-12 * np.abs(ph).max()
    # projection identity, by the oracle: D u = D u* - dt A p
    du = oracle.divergence(uh, w.bc, w.h)
    dus = oracle.divergence(w.us, w.bc, w.h)
    ref = dus - w.dt * oracle.apply(betah, w.bc, w.h, ph)
    # the two sides cancel to ~1e-8 of |D u*|: compare at the scale of D u*
    assert np.abs(du - ref).max() <= 1e-12 * np.abs(dus).max()
    # adjoint: lambda solves A lambda = w - mean w (oracle residual), mean zero
    assert rel_res(betah, w.bc, w.h, w.w, lh_) <= 1.05e-8
    # dot-product identity <w, S b> = <S w, b> (both sides at tol 1e-8)
    bm = rhs - rhs.mean()
    lhs = np.vdot(w.w - w.w.mean(), ph)
    rhs_ = np.vdot(lh_, bm)
    assert abs(lhs - rhs_) <= 1e-6 * abs(lhs)
    # face products on sampled faces: g_beta_m[c] = G lambda * G p, 0 on walls
    rng = np.random.default_rng(5)
    h = w.h
    nz, ny, nx = w.shape
    for _ in range(200):
        m = int(rng.integers(0, 3))
        k, j, i = (int(v) for v in rng.integers(0, 512, 3))
        c = (k, j, i)
        lo = [k, j, i]
        lo[2 - m] -= 1
        if lo[2 - m] < 0:
            assert gbh[m][c] == 0.0
            continue
        lo = tuple(lo)
        ref = (lh_[c] - lh_[lo]) * (ph[c] - ph[lo]) / (h * h)
        assert abs(gbh[m][c] - ref) <= 1e-12 * max(abs(ref), np.abs(gbh[m]).max() * 1e-6)


def test_jet512_directional_derivatives(S, jet512):
    """Central differences of L = <w, p> at 512^3 along random full-field
    directions (single-entry differences drown in solver noise at 1.3e8
    cells): in beta, dL = <g_beta, dbeta>; in rhs, L is linear, so the
    difference quotient must equal <g_rhs, v>.  Perturbed solves run in FP64
    to 1e-12 from the unperturbed solution."""
    w = jet512
    _say("512^3 directional derivatives")
    rho = dev(w.rho)
    bt = S.face_coeffs(rho, w.h, w.bc)
    wt = dev(w.w)
    us = [dev(u) for u in w.us]
    with S.Solver(bt, w.h, w.bc, precision="fp32") as sol:
        b = sol.divergence(us, 1.0 / w.dt)
        p = sol.solve(b, tol=1e-11)
        g_rhs, g_b = sol.adjoint(p, wt, tol=1e-11)
    del us
    gen = torch.Generator(device="cuda").manual_seed(7)
    with S.Solver(bt, w.h, w.bc, precision="fp64", warm_start=True) as s64:
        p0 = torch.zeros_like(b)
        s64.solve(b, tol=1e-12, p=p0)

        def L(rhs_t, solver):
            pp = p0.clone()
            solver.solve(rhs_t, tol=1e-12, p=pp)
            return float((wt * pp).sum())

        v = (torch.rand(b.shape, generator=gen, device="cuda", dtype=torch.float64) * 2 - 1) * b.abs().max()
        eps = 1e-3
        fd = (L(b + eps * v, s64) - L(b - eps * v, s64)) / (2 * eps)
        ad = float((g_rhs * v).sum())
        _say(f"  rhs direction: fd {fd:.9e} adjoint {ad:.9e}")
        assert abs(fd - ad) <= 1e-6 * abs(ad)
    dirs = []
    for m in range(3):
        dv = torch.rand(b.shape, generator=gen, device="cuda", dtype=torch.float64) * 2 - 1
        dv[(slice(None),) * (2 - m) + (0,)] = 0.0          # wall faces stay walls
        dirs.append(dv * bt[m])
    eps = 1e-5
    vals = []
    for sgn in (1, -1):
        bb = [bt[m] + sgn * eps * dirs[m] for m in range(3)]
        with S.Solver(bb, w.h, w.bc, precision="fp64", warm_start=True) as s2:
            pp = p0.clone()
            s2.solve(b, tol=1e-12, p=pp)
            vals.append(float((wt * pp).sum()))
    fd = (vals[0] - vals[1]) / (2 * eps)
    ad = sum(float((g_b[m] * dirs[m]).sum()) for m in range(3))
    _say(f"  beta direction: fd {fd:.9e} adjoint {ad:.9e}")
    assert abs(fd - ad) <= 1e-5 * abs(ad)
