"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances:
  * single passes (face coefficients, divergence, operator, projection, one
    Gauss-Seidel sweep, transfers) are the same FP64 arithmetic in another
    order: relative 1e-14..1e-13 of the field's scale;
  * solves: both sides converge to a relative residual; the p error is then
    bounded by the conditioning, so parity is asserted at a tight tolerance
    (GPU 1e-11, oracle 1e-13) with max|p - p_o| / max|p_o| <= 1e-8, and at
    the timing tolerance 1e-8 through the oracle's own FP64 residual of the
    GPU answer (<= 1.05e-8) plus a looser p bound.
"""
import hashlib
import math
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


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


RAGGED = [((8, 8, 8), (0, 0, 0)), ((40, 20, 56), (1, 0, 1)), ((144, 80, 32), (0, 1, 1)),
          ((48, 36, 24), (1, 1, 1))]


# ---------------------------------------------------------------------------
# single passes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,bc", RAGGED)
def test_face_coeffs(S, n, bc):
    _say(f"face_coeffs n={n} bc={bc}")
    w = W.random_case(n, bc, seed=101)
    ref = oracle.face_coeffs(w.rho, bc)
    got = S.face_coeffs(dev(w.rho), w.h, bc)
    for m in range(3):
        assert relmax(host(got[m]), ref[m]) <= 2e-16


@pytest.mark.parametrize("n,bc", RAGGED)
def test_divergence_apply_project(S, n, bc):
    _say(f"divergence/apply/project n={n} bc={bc}")
    w = W.random_case(n, bc, seed=102)
    beta = oracle.face_coeffs(w.rho, bc)
    with S.Solver([dev(b) for b in beta], w.h, bc, precision="fp64") as sol:
        us = [dev(u) for u in w.us]
        d = sol.divergence(us, 1.0 / w.dt)
        assert relmax(host(d), oracle.divergence(w.us, bc, w.h, 1.0 / w.dt)) <= 1e-14
        x = np.random.default_rng(1).standard_normal(w.shape)
        y = sol.apply(dev(x))
        assert relmax(host(y), oracle.apply(beta, bc, w.h, x)) <= 1e-13
        u = sol.project(us, dev(x), w.dt)
        ref = oracle.project(beta, bc, w.h, w.dt, w.us, x)
        for m in range(3):
            assert relmax(host(u[m]), ref[m]) <= 1e-14
        # in place (u aliases u*)
        sol.project(us, dev(x), w.dt, out=us)
        for m in range(3):
            assert relmax(host(us[m]), ref[m]) <= 1e-14


@pytest.mark.parametrize("n,bc", RAGGED)
@pytest.mark.parametrize("omega", [1.0, 1.3])
def test_one_gauss_seidel_sweep_matches_paper_sor(S, n, bc, omega):
    """One red-black sweep (relaxation omega) equals the oracle's sweep of eq.
    beta_pressure: same-colour updates are independent, so order-free."""
    _say(f"rbgs sweep n={n} bc={bc} omega={omega}")
    w = W.random_case(n, bc, seed=103)
    beta = oracle.face_coeffs(w.rho, bc)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(w.shape)
    e0 = rng.standard_normal(w.shape)
    ref, _, _ = oracle.rbsor(beta, bc, w.h, r, p0=e0, omega=omega, sweeps=1)
    e = dev(e0)
    S.k_smooth(w.shape, w.h, bc, [dev(b) for b in beta], dev(r), e, sweeps=1, omega=omega)
    assert relmax(host(e), ref) <= 1e-14
    # two sweeps from zero (zero_init reads neither e nor, in the first sweep,
    # the second colour's old values)
    ref2, _, _ = oracle.rbsor(beta, bc, w.h, r, p0=np.zeros(w.shape), omega=omega, sweeps=2)
    e = dev(np.full(w.shape, np.nan))
    S.k_smooth(w.shape, w.h, bc, [dev(b) for b in beta], dev(r), e, sweeps=2, zero_init=True,
               omega=omega)
    assert relmax(host(e), ref2) <= 1e-14


# grids whose z chunks are long enough for the march in whole unrolled blocks
# (the last block running past the chunk), with a ragged last chunk: FP64
# single sweep (128 x 8 tiles, chunks of 47 planes) and FP32 two-sweep pass
# (64 x 8 tiles, chunks of 48 planes)
WHOLE_F64 = ((256, 128, 370), (1, 0, 0))
WHOLE_F32 = ((256, 128, 190), (0, 0, 1))


@pytest.mark.parametrize("n,bc", RAGGED + [((130, 12, 20), (0, 0, 1)), ((64, 16, 8), (1, 1, 0)),
                                  WHOLE_F64])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("omega", [1.0, 1.3])
def test_fused_sweep_matches_paper_sor(S, n, bc, first, omega):
    """One fused out-of-place sweep (tiles of 128 x 8 cells, z chunks, ring
    recomputation) equals the oracle's sweep of eq. beta_pressure with the
    same colour order and relaxation; also from a zero start (e_in not read)."""
    _say(f"fused rbgs sweep n={n} bc={bc} first={first} omega={omega}")
    w = W.random_case(n, bc, seed=113)
    beta = oracle.face_coeffs(w.rho, bc)
    bt = [dev(b) for b in beta]
    rng = np.random.default_rng(4)
    r = rng.standard_normal(w.shape)
    e0 = rng.standard_normal(w.shape)
    ref, _, _ = oracle.rbsor(beta, bc, w.h, r, p0=e0, omega=omega, sweeps=1, first_colour=first)
    out = dev(np.full(w.shape, np.nan))
    S.k_smooth_fused(w.shape, w.h, bc, bt, dev(r), dev(e0), out, first_colour=first, omega=omega)
    assert relmax(host(out), ref) <= 1e-14
    ref0, _, _ = oracle.rbsor(beta, bc, w.h, r, p0=np.zeros(w.shape), omega=omega, sweeps=1,
                              first_colour=first)
    out = dev(np.full(w.shape, np.nan))
    S.k_smooth_fused(w.shape, w.h, bc, bt, dev(r), dev(np.full(w.shape, np.nan)), out,
                     first_colour=first, zero_init=True, omega=omega)
    assert relmax(host(out), ref0) <= 1e-14


@pytest.mark.parametrize("n,bc", RAGGED + [((130, 12, 20), (0, 0, 1)), ((64, 16, 8), (1, 1, 0)),
                                  ((200, 72, 40), (0, 0, 0)), WHOLE_F32])
@pytest.mark.parametrize("first", [0, 1])
@pytest.mark.parametrize("omega", [1.0, 1.3])
def test_two_sweep_fused_f32_matches_paper_sor(S, n, bc, first, omega):
    """Two sweeps in one pass (FP32 storage and arithmetic; tiles of 64 x 8
    cells with a ring two pairs / three rows deep, z chunks marched three
    planes beyond their ends) against two of the oracle's sweeps of eq.
    beta_pressure on the same FP32-rounded inputs.  Tolerance: FP32 rounding
    of each update (a few ulps, the reciprocal within 1 ulp) carried through
    four colour passes, relative to max|e|: 2e-6 (with relaxation 1.3 each update
    also rounds (1 - omega) e and omega / diag, a few more ulps)."""
    _say(f"two-sweep fused f32 n={n} bc={bc} first={first} omega={omega}")
    w = W.random_case(n, bc, seed=117)
    beta = [b.astype(np.float32) for b in oracle.face_coeffs(w.rho, bc)]
    rng = np.random.default_rng(5)
    r = rng.standard_normal(w.shape).astype(np.float32)
    e0 = rng.standard_normal(w.shape).astype(np.float32)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    bt = [f32(b) for b in beta]
    b64 = [b.astype(np.float64) for b in beta]
    for zero in (False, True):
        p0 = np.zeros(w.shape) if zero else e0.astype(np.float64)
        ref, _, _ = oracle.rbsor(b64, bc, w.h, r.astype(np.float64), p0=p0, omega=omega,
                                 sweeps=2, first_colour=first)
        out = f32(np.full(w.shape, np.nan))
        ein = f32(np.full(w.shape, np.nan)) if zero else f32(e0)
        S.k_smooth2_fused_f32(w.shape, w.h, bc, bt, f32(r), ein, out, first_colour=first,
                              zero_init=zero, omega=omega)
        got = host(out).astype(np.float64)
        err = relmax(got, ref)
        _say(f"  zero={zero} err={err:.2e}")
        assert np.isfinite(got).all()
        assert err <= 2e-6


@pytest.mark.parametrize("n,bc", [((40, 20, 56), (1, 0, 1)), ((144, 80, 32), (0, 1, 1)),
                                  ((200, 72, 40), (0, 0, 0)), WHOLE_F32])
def test_two_sweep_fused_dot_product(S, n, bc):
    """The FP32 V-cycle's last fine pass also forms r . e_out for the outer
    iteration, r its own right-hand side: e_out equals the plain pass bit for
    bit.  Each product is formed from the FP32 h^2 r the sweep carries, so the
    dot product equals sum(fl32(h^2 r) e_out) / h^2 in FP64 up to summation
    order (relative 1e-12 of the sum of absolute terms), and sum(r e_out)
    within the FP32 rounding of h^2 r (2^-24 per term)."""
    _say(f"two-sweep fused dot n={n} bc={bc}")
    w = W.random_case(n, bc, seed=118)
    beta = [b.astype(np.float32) for b in oracle.face_coeffs(w.rho, bc)]
    rng = np.random.default_rng(6)
    r = rng.standard_normal(w.shape).astype(np.float32)
    e0 = rng.standard_normal(w.shape).astype(np.float32)
    h2f = np.float32(w.h * w.h)
    hr = (h2f * r).astype(np.float64)            # FP32 product, as the sweep forms it
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    bt = [f32(b) for b in beta]
    for first, omega in ((0, 1.0), (1, 1.0), (0, 1.3)):
        plain = f32(np.full(w.shape, np.nan))
        S.k_smooth2_fused_f32(w.shape, w.h, bc, bt, f32(r), f32(e0), plain, first_colour=first,
                              omega=omega)
        out = f32(np.full(w.shape, np.nan))
        dot = S.k_smooth2_fused_dot_f32(w.shape, w.h, bc, bt, f32(r), f32(e0), out,
                                        first_colour=first, omega=omega)
        eo = host(out).astype(np.float64)
        assert np.array_equal(host(plain), host(out))
        ref = float(np.sum(hr * eo)) / float(h2f)
        scale = float(np.sum(np.abs(hr * eo))) / float(h2f)
        plain_ref = float(np.sum(r.astype(np.float64) * eo))
        _say(f"  first={first} dot={dot:.15e} ref={ref:.15e} sum(r e)={plain_ref:.15e}")
        assert abs(dot - ref) <= 1e-12 * scale
        assert abs(dot - plain_ref) <= 2.0 ** -23 * scale


@pytest.mark.parametrize("count,offset", [(1, 0), (7, 0), (1 << 20, 0), ((1 << 20) + 3, 0),
                                          (1001, 1)])
def test_copy_kernel(S, count, offset):
    """The bandwidth-reference copy, exact for even and odd counts and for
    8-byte aligned (not 16-byte aligned) arrays."""
    src = torch.arange(count + offset, dtype=torch.float64, device="cuda")[offset:]
    dst = torch.full((count + offset,), -1.0, dtype=torch.float64, device="cuda")[offset:]
    S.k_copy(src, dst)
    assert torch.equal(src, dst)


def _restrict_ref(x):
    nz, ny, nx = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def _prolong_ref(eH, bc):
    """Cell-centred trilinear: 3/4 parent + 1/4 next coarse cell per axis."""
    out = eH
    for ax, m in ((2, 0), (1, 1), (0, 2)):
        nH = out.shape[ax]
        i = np.arange(2 * nH)
        par = i // 2
        oth = np.where(i % 2 == 0, par - 1, par + 1)
        if bc[m] == 1:
            oth = np.clip(oth, 0, nH - 1)
        else:
            oth = oth % nH
        out = 0.75 * np.take(out, par, axis=ax) + 0.25 * np.take(out, oth, axis=ax)
    return out


# grids whose coarse level takes the restriction's slab block order (a block
# count that divides by 8): two x-blocks of 64 coarse columns with a partial
# last one, two block rows (the second partial in the first case) and a
# multiple of 8 block planes
XCD_GROUPED = [((144, 12, 16), (0, 1, 1)), ((144, 16, 32), (1, 0, 0))]


@pytest.mark.parametrize("n,bc", RAGGED + XCD_GROUPED)
def test_transfers(S, n, bc):
    _say(f"transfers n={n} bc={bc}")
    w = W.random_case(n, bc, seed=104)
    beta = oracle.face_coeffs(w.rho, bc)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(w.shape)
    r = rng.standard_normal(w.shape)
    nz, ny, nx = w.shape
    cshape = (nz // 2, ny // 2, nx // 2)
    rH = dev(np.zeros(cshape))
    S.k_resid_restrict(w.shape, w.h, bc, [dev(b) for b in beta], dev(e), dev(r), rH)
    ref = _restrict_ref(r - oracle.apply(beta, bc, w.h, e))
    assert relmax(host(rH), ref) <= 1e-13
    eH = rng.standard_normal(cshape)
    ef = dev(e)
    S.k_prolong_add(w.shape, w.h, bc, dev(eH), ef)
    assert relmax(host(ef), e + _prolong_ref(eH, bc)) <= 1e-14
    out = [dev(np.zeros(cshape)) for _ in range(3)]
    S.k_coarsen_beta(w.shape, w.h, bc, [dev(b) for b in beta], out)
    ref = _coarse_beta_ref(beta, bc)
    for m in range(3):
        assert relmax(host(out[m]), ref[m]) <= 1e-14
    # operator-dependent prolongation: weights from the face coefficients,
    # then the interpolation with those weights
    wts = S.k_prolong_weights(w.shape, w.h, bc, [dev(b) for b in beta])
    packed = host(wts).astype(np.int64) & 0xFFFFFFFF
    wq = [_quantise(x) for x in _weights_ref(beta, bc)]
    assert np.array_equal(packed, wq[0] | (wq[1] << 8) | (wq[2] << 16))
    ef = dev(e)
    S.k_prolong_add_weighted(w.shape, w.h, bc, dev(eH), wts, ef)
    assert relmax(host(ef), e + _prolong_weighted_ref(eH, bc, [q / 256.0 for q in wq])) <= 1e-14


def _wall0(b, m, bc):
    """b with the wall entries (index 0 along direction m) set to 0."""
    b = b.copy()
    if bc[m] == 1:
        sl = [slice(None)] * 3
        sl[2 - m] = 0
        b[tuple(sl)] = 0.0
    return b


def _coarse_beta_ref(beta, bc):
    """Coarse face coefficient: 1/4 of (a) the mean of the 4 fine faces on the
    coarse face plus 3/4 of (b) the mean over the 4 rows of the series
    coefficient 2 / (1/(2 b[2I-1]) + 1/b[2I] + 1/(2 b[2I+1])) along the normal."""
    out = []
    for m in range(3):
        ax = 2 - m
        b = _wall0(beta[m], m, bc)
        lo = np.roll(b, 1, axis=ax)
        hi = np.roll(b, -1, axis=ax)
        with np.errstate(divide="ignore", invalid="ignore"):
            den = (b * hi + 2.0 * (lo * hi)) + lo * b
            ser = np.where(den > 0, (4.0 * lo) * (b * hi) / np.where(den > 0, den, 1.0), 0.0)
        sl = [slice(None)] * 3
        sl[ax] = slice(0, None, 2)
        par, srs = b[tuple(sl)], ser[tuple(sl)]
        for a in range(3):
            if a == ax:
                continue
            lo_ = [slice(None)] * 3
            hi_ = [slice(None)] * 3
            lo_[a] = slice(0, None, 2)
            hi_[a] = slice(1, None, 2)
            par = 0.5 * (par[tuple(lo_)] + par[tuple(hi_)])
            srs = 0.5 * (srs[tuple(lo_)] + srs[tuple(hi_)])
        f = 0.25 * par + 0.75 * srs
        if bc[m] == 1:
            s0 = [slice(None)] * 3
            s0[ax] = 0
            f[tuple(s0)] = 0.0
        out.append(f)
    return out


def _weights_ref(beta, bc):
    """Weight of the far coarse cell per fine cell and axis: the share of the
    half link to the parent's centre in the series resistance of the interval
    between the two coarse centres, g_m g_f / (g_m g_f + g_n (2 g_f + g_m))."""
    out = []
    for m in range(3):
        ax = 2 - m
        b = _wall0(beta[m], m, bc)
        n = b.shape[ax]
        f = {d: np.roll(b, -d, axis=ax) for d in (-1, 0, 1, 2)}   # face i + d
        idx = np.arange(n).reshape([n if a == ax else 1 for a in range(3)])
        odd = (idx % 2) == 1
        gn = np.where(odd, f[0], f[1])
        gm = np.where(odd, f[1], f[0])
        gf = np.where(odd, f[2], f[-1])
        den = gm * gf + gn * (2 * gf + gm)
        with np.errstate(invalid="ignore", divide="ignore"):
            out.append(np.where(den > 0, gm * gf / np.where(den > 0, den, 1.0), 0.0))
    return out


def _quantise(wt):
    """8-bit fraction of 256: min(255, floor(256 w + 1/2))."""
    return np.minimum(255, np.floor(wt * 256.0 + 0.5)).astype(np.int64)


def _prolong_weighted_ref(eH, bc, wts):
    """Per axis parent (1 - w) and next coarse cell (w), composed as a product."""
    shape = tuple(2 * v for v in eH.shape)
    maps = []
    for ax, m in ((0, 2), (1, 1), (2, 0)):
        nH = eH.shape[ax]
        i = np.arange(2 * nH)
        par = i // 2
        oth = np.where(i % 2 == 0, par - 1, par + 1)
        oth = np.clip(oth, 0, nH - 1) if bc[m] == 1 else oth % nH
        maps.append((par, oth))
    (pz, oz), (py, oy), (px, ox) = maps
    wz, wy, wx = wts[2], wts[1], wts[0]
    out = np.zeros(shape)
    for cz, fz in ((pz, 1 - wz), (oz, wz)):
        for cy, fy in ((py, 1 - wy), (oy, wy)):
            for cx, fx in ((px, 1 - wx), (ox, wx)):
                out += fz * fy * fx * eH[cz[:, None, None], cy[None, :, None], cx[None, None, :]]
    return out


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

_ORACLE_P = {}


def _oracle_p(w, beta, rhs, tol):
    # keyed on the inputs themselves: workloads of one name and size may
    # differ in seed or density ratio
    key = (w.name, w.n, w.bc, tol, hashlib.sha1(rhs.tobytes()).hexdigest(),
           hashlib.sha1(w.rho.tobytes()).hexdigest())
    if key not in _ORACLE_P:
        _ORACLE_P[key] = oracle.solve(beta, w.bc, w.h, rhs, tol=tol)[0]
    return _ORACLE_P[key]


def _parity_solve(S, w, precision, outer="pcg", tol=1e-11, tol_oracle=1e-13, ptol=1e-8,
                  max_outer=500, omega=None, cycle="v"):
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o = _oracle_p(w, beta, rhs, tol_oracle)
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision, outer=outer,
                  max_outer=max_outer, omega=omega, cycle=cycle) as sol:
        us = [dev(u) for u in w.us]
        b = sol.divergence(us, 1.0 / w.dt)
        p = sol.solve(b, tol=tol)
        st = sol.last_stats
        u = sol.project(us, p, w.dt)
        p_h = host(p)
        err_p = relmax(p_h, p_o)
        u_o = oracle.project(beta, w.bc, w.h, w.dt, w.us, p_o)
        du = oracle.divergence([host(c) for c in u], w.bc, w.h)
        du_o = oracle.divergence(u_o, w.bc, w.h)
        ds = oracle.divergence(w.us, w.bc, w.h)
        err_div = np.abs(du - du_o).max() / np.abs(ds).max()
        res = oracle.apply(beta, w.bc, w.h, p_h)
        bm = rhs - rhs.mean()
        rel_true = np.linalg.norm(bm - res) / np.linalg.norm(bm)
    _say(f"  {w.name} {precision}/{outer}/{cycle} tol={tol:g}: iters={st['outer_iters']} "
         f"rel={st['rel_res']:.2e} true={rel_true:.2e} err_p={err_p:.2e} err_div={err_div:.2e} "
         f"fell_back={st['fell_back']}")
    assert rel_true <= 1.05 * tol
    assert err_p <= ptol
    assert abs(p_h.mean()) <= 1e-12 * np.abs(p_h).max()
    return st, err_p, err_div


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_relaxation_reaches_the_smoothers(S, precision):
    """The smoother's over-relaxation (opts.omega) changes the preconditioner
    (different residual histories) and not the answer: 64^3 layer and droplets
    (two-sweep or fused passes on 64^3 and 32^3, the single-workgroup tail
    below) solved with plain Gauss-Seidel, the default and a strong
    over-relaxation all match the oracle."""
    _say(f"relaxation 64^3 {precision}")
    w = W.config3(64)
    hist = {}
    for om in (1.0, 1.2, 1.6):
        st, _, _ = _parity_solve(S, w, precision, tol=1e-11, ptol=1e-8, omega=om)
        hist[om] = list(st["res_hist"][:st["outer_iters"]])
    assert hist[1.0] != hist[1.2] and hist[1.2] != hist[1.6]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config1_sphere_periodic(S, precision):
    _say(f"config1 32^3 {precision}")
    w = W.config1(32)
    _parity_solve(S, w, precision, tol=1e-10, ptol=1e-8)


@pytest.mark.parametrize("n,bc", RAGGED)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_random_ratio1000_ragged(S, n, bc, precision):
    _say(f"random ratio1000 n={n} bc={bc} {precision}")
    w = W.random_case(n, bc, seed=105, ratio=1000.0)
    _parity_solve(S, w, precision, tol=1e-11, ptol=1e-8)


@pytest.mark.parametrize("n,bc", [((9, 10, 10), (1, 0, 1)), ((10, 9, 8), (0, 1, 0)),
                                  ((7, 11, 12), (0, 0, 1))])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_odd_grid_one_cell_direction_pass(S, n, bc, precision):
    """Odd nx or ny: the direction pass takes its one-cell form (pairs of
    cells need both counts even); single-level grids of at most 1024 cells."""
    _say(f"odd grid n={n} bc={bc} {precision}")
    w = W.random_case(n, bc, seed=136, ratio=1000.0)
    _parity_solve(S, w, precision, tol=1e-11, ptol=1e-8)


@pytest.mark.parametrize("load", ["beta", "rho"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_unaligned_iterate_one_cell_direction_pass(S, precision, load):
    """p handed as a view one element into a larger buffer (8-byte aligned):
    the direction pass updates the iterate one cell at a time, with the
    stored coefficients or (after a density update) beta formed from rho.
    Parity with the oracle as for an aligned p."""
    w = W.config3(64)
    _say(f"unaligned p config3 64^3 {precision} {load}")
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o = _oracle_p(w, beta, rhs, 1e-13)
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision) as sol:
        if load == "rho":
            sol.update_density(dev(w.rho))
        b = sol.divergence([dev(u) for u in w.us], 1.0 / w.dt)
        big = torch.zeros(w.rho.size + 1, dtype=torch.float64, device="cuda")
        p = big[1:].view(w.shape)
        assert p.data_ptr() % 16 == 8
        sol.solve(b, tol=1e-11, p=p)
        it_u = sol.last_stats["outer_iters"]
        p_a = sol.solve(b, tol=1e-11)
        it_a = sol.last_stats["outer_iters"]
        p_h, pa_h = host(p), host(p_a)
    res = oracle.apply(beta, w.bc, w.h, p_h)
    bm = rhs - rhs.mean()
    rel_true = np.linalg.norm(bm - res) / np.linalg.norm(bm)
    _say(f"  iters unaligned={it_u} aligned={it_a} true={rel_true:.2e} "
         f"err_p={relmax(p_h, p_o):.2e} vs aligned={relmax(p_h, pa_h):.2e}")
    assert rel_true <= 1.05e-11
    assert relmax(p_h, p_o) <= 1e-8
    assert relmax(p_h, pa_h) <= 1e-9
    assert abs(it_u - it_a) <= 1


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_density_load_then_fp64_coefficient_readers(S, precision):
    """After a density load in a mixed mode the FP64 fine-level coefficients
    are formed from rho only when something reads them: pp_apply gives the
    same bits as a context loaded with the coefficients themselves, and
    defect correction (whose residual reads them every iteration) and a
    second PCG solve reach parity with the oracle."""
    _say(f"density load then FP64 readers, config3 64^3 {precision}")
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o = _oracle_p(w, beta, rhs, 1e-13)
    x = dev(np.random.default_rng(5).standard_normal(w.shape))
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision) as ref:
        y_ref = host(ref.apply(x)).copy()
    flat = [dev(np.ones(w.shape)) for _ in range(3)]
    for outer in ("dc", "pcg"):
        with S.Solver(flat, w.h, w.bc, precision=precision, outer=outer) as sol:
            sol.update_density(dev(w.rho))
            p = sol.solve(dev(rhs), tol=1e-11)
            it = sol.last_stats["outer_iters"]
            p_h = host(p)
            if outer == "dc":
                assert np.array_equal(host(sol.apply(x)), y_ref)
        _say(f"  {outer}: iters={it} err_p={relmax(p_h, p_o):.2e}")
        assert relmax(p_h, p_o) <= 1e-8


@pytest.mark.parametrize("outer", ["pcg", "dc"])
def test_config3_layer_droplets_64(S, outer):
    _say(f"config3 geometry at 64^3, fp32, {outer}")
    w = W.config3(64)
    _parity_solve(S, w, "fp32", outer=outer, tol=1e-11, ptol=1e-8)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config2_bubbles_128(S, precision):
    _say(f"config2 128^3 {precision}")
    w = W.config2(128)
    _parity_solve(S, w, precision, tol=1e-10, ptol=1e-8)
    st, _, _ = _parity_solve(S, w, precision, tol=1e-8, ptol=1e-6)
    # gas bubbles in liquid at ratio 1000: the coefficient-dependent coarse
    # faces and prolongation take the outer CG from 57 iterations (averaged
    # faces, trilinear interpolation) to 23
    assert st["outer_iters"] <= 26


@pytest.mark.parametrize("cycle", ["w", "f"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_w_cycle_bubbles_128(S, precision, cycle):
    """W- and F-cycles (two coarse corrections per level above the
    single-workgroup tail, the second starting from the first's result)
    solve the bubbles at ratio 1000 to parity in fewer outer iterations
    than the V-cycle."""
    _say(f"{cycle.upper()}-cycle config2 128^3 {precision}")
    w = W.config2(128)
    _parity_solve(S, w, precision, tol=1e-10, ptol=1e-8, cycle=cycle)
    st_w, _, _ = _parity_solve(S, w, precision, tol=1e-8, ptol=1e-6, cycle=cycle)
    st_v, _, _ = _parity_solve(S, w, precision, tol=1e-8, ptol=1e-6, cycle="v")
    assert st_w["outer_iters"] < st_v["outer_iters"]


@pytest.mark.parametrize("cycle", ["w", "f"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("outer", ["pcg", "dc"])
def test_w_cycle_layer_droplets_64(S, precision, outer, cycle):
    """W- and F-cycles on the layer and droplets at 64^3 (two-sweep passes on 64^3
    and 32^3 entered from a non-zero correction, the tail entered warm):
    parity with the oracle under both outer iterations."""
    _say(f"{cycle.upper()}-cycle config3 64^3 {precision} {outer}")
    w = W.config3(64)
    _parity_solve(S, w, precision, outer=outer, tol=1e-11, ptol=1e-8, cycle=cycle)


@pytest.mark.parametrize("cycle", ["w", "f"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cycles_from_the_coarse_graph(S, precision, cycle):
    """W- and F-cycles with the coarse levels replayed from a HIP graph (the
    whole recursion below the fine level, warm-started tails included, is
    captured once): the same iterations and the same bits as the eager
    launches, on three solves in a row, and parity with the oracle."""
    _say(f"{cycle.upper()}-cycle coarse graph config3 64^3 {precision}")
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o = _oracle_p(w, beta, rhs, 1e-13)
    out = {}
    for graph in (False, True):
        with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision, cycle=cycle,
                      coarse_graph=graph) as sol:
            runs = []
            for _ in range(3):
                p = sol.solve(dev(rhs), tol=1e-11)
                runs.append((sol.last_stats["outer_iters"], host(p).copy()))
        out[graph] = runs
    for (ie, pe), (ig, pg) in zip(out[False], out[True]):
        assert ie == ig
        assert np.array_equal(pe, pg)
    _say(f"  iters={out[True][0][0]} err_p={relmax(out[True][0][1], p_o):.2e}")
    assert relmax(out[True][-1][1], p_o) <= 1e-8


@pytest.mark.parametrize("coarsest,dims", [(512, (8, 8, 8)), (1000, (8, 8, 8)), (200, (4, 4, 4)),
                                            (1, (4, 4, 4))])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coarsest_level_size(S, precision, coarsest, dims):
    """opts.coarsest stops the halving at a level of at most that many cells:
    on 64^3 a limit of 512 keeps 8^3 as the coarsest level (a 512 x 512
    pseudo-inverse read from global memory by the tail), 64 or less ends at
    4^3.  Parity with the oracle either way."""
    _say(f"coarsest={coarsest} config3 64^3 {precision}")
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o = _oracle_p(w, beta, rhs, 1e-13)
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision,
                  coarsest=coarsest) as sol:
        nl = sol.levels
        assert sol.level_dims(nl - 1) == dims
        p = sol.solve(dev(rhs), tol=1e-11)
        it = sol.last_stats["outer_iters"]
        p_h = host(p)
    _say(f"  levels={nl} iters={it} err_p={relmax(p_h, p_o):.2e}")
    assert relmax(p_h, p_o) <= 1e-8


@pytest.mark.parametrize("cycle", ["w", "f"])
@pytest.mark.parametrize("n,bc", RAGGED)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_w_cycle_ragged(S, n, bc, precision, cycle):
    """W- and F-cycles on ragged grids: 144 x 80 x 32 has a level of 5,760 cells
    that the per-colour sweep handles, entered warm for the second coarse
    correction."""
    _say(f"{cycle.upper()}-cycle random ratio1000 n={n} bc={bc} {precision}")
    w = W.random_case(n, bc, seed=171, ratio=1000.0)
    _parity_solve(S, w, precision, tol=1e-11, ptol=1e-8, cycle=cycle)


def test_config2_bubbles_128_defect_correction(S):
    """Defect correction (the V-cycle as a stationary iteration, FP64 outer
    residual) converges on the bubbles at ratio 1000, to parity: slowly
    (about 0.93 per cycle once the fast modes are gone; it stalled with
    averaged coarse faces and trilinear interpolation)."""
    _say("config2 128^3 fp32 defect correction")
    w = W.config2(128)
    st, _, _ = _parity_solve(S, w, "fp32", outer="dc", tol=1e-11, ptol=1e-8, max_outer=1000)
    assert not st["fell_back"]


def test_manufactured_cosine_gpu(S):
    """The GPU solve reproduces the closed-form discrete solution
    p (pi h)^2 / sin^2(pi h) of the cosine mode (walls)."""
    n = 64
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    c = np.cos(2 * np.pi * x)
    p = c[None, None, :] * c[None, :, None] * c[:, None, None]
    bc = (1, 1, 1)
    beta = oracle.face_coeffs(np.full((n, n, n), 2.0), bc)
    with S.Solver([dev(b) for b in beta], h, bc, precision="fp32") as sol:
        ph = host(sol.solve(dev(-12 * np.pi ** 2 * p / 2.0), tol=1e-12))
    assert np.abs(ph - p * (np.pi * h) ** 2 / np.sin(np.pi * h) ** 2).max() <= 1e-10


def test_deterministic_bitwise(S):
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = dev(oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt))
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision="fp32") as sol:
        p1 = host(sol.solve(rhs, tol=1e-9)).copy()
        p2 = host(sol.solve(rhs, tol=1e-9)).copy()
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_rhs_scale_bitwise_linear(S, precision):
    """The mixed-precision solve keeps everything held in FP32 / FP16 (the
    residual handed to the V-cycle, the search direction) in units of the
    residual's RMS, and the rest in FP64, so scaling the right-hand side by
    2^+-130 (beyond the FP32 range either way) scales the answer by exactly
    that power of two, bit for bit, with the same iterations."""
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision) as sol:
        p0 = host(sol.solve(dev(rhs), tol=1e-9)).copy()
        it0 = sol.last_stats["outer_iters"]
        for e in (130, -130):
            _say(f"rhs scale 2^{e} {precision}")
            pe = host(sol.solve(dev(np.ldexp(rhs, e)), tol=1e-9)).copy()
            assert sol.last_stats["outer_iters"] == it0
            assert np.array_equal(pe, np.ldexp(p0, e))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_coarse_graph_replays_match_eager(S, precision):
    """The coarse levels replayed from the captured HIP graph give, replay
    after replay and with eager work and synchronisations in between, the
    same bits as the same kernels launched one by one."""
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    bt = [dev(b) for b in beta]
    rhs = dev(oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt))
    rng = np.random.default_rng(11)
    with S.Solver(bt, w.h, w.bc, precision=precision, coarse_graph=True) as g, \
            S.Solver(bt, w.h, w.bc, precision=precision, coarse_graph=False) as e:
        for rep in range(4):
            r = dev(rng.standard_normal(w.shape))
            zg = host(g.vcycle(r)).copy()
            junk = torch.randn(w.shape, dtype=torch.float64, device="cuda") * 2.0   # eager work
            torch.cuda.synchronize()
            ze = host(e.vcycle(r)).copy()
            assert np.array_equal(zg, ze), f"replay {rep} differs"
            pg = host(g.solve(rhs, tol=1e-9)).copy()
            pe = host(e.solve(rhs, tol=1e-9)).copy()
            assert np.array_equal(pg, pe), f"solve {rep} differs"
            del junk


def test_smallest_grid_single_level(S):
    """4^3: the whole problem is the coarsest level (direct FP64 solve)."""
    w = W.random_case((4, 4, 4), (1, 0, 1), seed=106)
    st, err, _ = _parity_solve(S, w, "fp32", tol=1e-11, ptol=1e-10)
    assert st["outer_iters"] <= 2


def test_zero_rhs_and_constant_rhs(S):
    w = W.random_case((16, 16, 16), (0, 0, 0), seed=107)
    beta = oracle.face_coeffs(w.rho, w.bc)
    with S.Solver([dev(b) for b in beta], w.h, w.bc) as sol:
        p = sol.solve(dev(np.zeros(w.shape)), tol=1e-8)
        assert np.all(host(p) == 0.0) and sol.last_stats["outer_iters"] == 0
        p = sol.solve(dev(np.full(w.shape, 3.0)), tol=1e-8)   # mean removed -> zero
        assert np.all(host(p) == 0.0)


def test_warm_start_and_update_coeffs(S):
    w = W.config4(32)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o, _, _ = oracle.solve(beta, w.bc, w.h, rhs)
    with S.Solver([dev(np.ones(w.shape)) for _ in range(3)], w.h, w.bc, warm_start=True) as sol:
        sol.update_coeffs([dev(b) for b in beta])
        p = dev(np.zeros(w.shape))
        sol.solve(dev(rhs), tol=1e-11, p=p)
        cold = sol.last_stats["outer_iters"]
        sol.solve(dev(rhs), tol=1e-11, p=p)          # warm: already converged
        assert sol.last_stats["outer_iters"] <= 1 < cold
        assert relmax(host(p), p_o) <= 1e-8


def test_invalid_coefficients_rejected(S):
    from paper_2012_11744_amd import _lib as L
    n = 8
    b = np.ones((n, n, n))
    bad = b.copy()
    bad[3, 4, 5] = 0.0                      # an interior face with zero coefficient
    with pytest.raises(L.PPError) as ei:
        S.Solver([dev(b), dev(bad), dev(b)], 1.0 / n, (0, 0, 0))
    assert ei.value.code == L.PP_EINVAL and "non-wall faces" in ei.value.detail
    nanb = b.copy()
    nanb[0, 0, 1] = np.nan
    with pytest.raises(L.PPError):
        S.Solver([dev(nanb), dev(b), dev(b)], 1.0 / n, (0, 0, 0))
    # a zero on a wall face is fine (wall entries are ignored)
    wallb = b.copy()
    wallb[:, :, 0] = 0.0
    S.Solver([dev(wallb), dev(b), dev(b)], 1.0 / n, (1, 0, 0)).close()


def test_max_outer_reports_noconv(S):
    from paper_2012_11744_amd import _lib as L
    w = W.config3(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = dev(oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt))
    with S.Solver([dev(b) for b in beta], w.h, w.bc, max_outer=2) as sol:
        p = sol.solve(rhs, tol=1e-12, check=False)
        st = sol.last_stats
        assert st["status"] == L.PP_ENOCONV and st["outer_iters"] == 2
        assert np.isfinite(host(p)).all()
        with pytest.raises(L.PPError):
            sol.solve(rhs, tol=1e-12)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_matches_oracle(S, precision):
    _say(f"adjoint config4 64^3 {precision}")
    w = W.config4(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    p_o, _, _ = oracle.solve(beta, w.bc, w.h, rhs)
    g_o, gb_o, _, _ = oracle.adjoint(beta, w.bc, w.h, p_o, w.w)
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision=precision) as sol:
        p = sol.solve(dev(rhs), tol=1e-11)
        g, gb = sol.adjoint(p, dev(w.w), tol=1e-11)
        assert relmax(host(g), g_o) <= 1e-8
        for m in range(3):
            assert relmax(host(gb[m]), gb_o[m]) <= 1e-8


def test_adjoint_finite_differences_64(S):
    """Config 4 at its own size (64^3, drop of density ratio 100): the
    hand-written backward (mixed FP32 V-cycle, tol 1e-12) against central
    differences of L = sum(w p) in 50 right-hand-side entries and 50 face
    coefficients spread over the three directions.  The perturbed solves are
    FP64, warm-started from the unperturbed p, to 1e-13; the coefficient
    perturbations go through update_coeffs on one context.  Steps: 1e-6 of
    the RMS of the right-hand side, 1e-6 absolute for beta."""
    _say("adjoint FD config4 64^3")
    w = W.config4(64)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    wt = dev(w.w)
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision="fp32") as sol:
        p = sol.solve(dev(rhs), tol=1e-12)
        g, gb = sol.adjoint(p, wt, tol=1e-12)
        g_rhs = host(g)
        g_b = [host(x) for x in gb]
    rng = np.random.default_rng(3)
    n = 64
    with S.Solver([dev(b) for b in beta], w.h, w.bc, precision="fp64", warm_start=True) as s64:
        p0 = dev(np.zeros(w.shape))
        s64.solve(dev(rhs), tol=1e-13, p=p0)

        def L_of(rhs_):
            pp = p0.clone()
            s64.solve(rhs_, tol=1e-13, p=pp)
            return float((wt * pp).sum())

        d = 1e-6 * np.sqrt(np.mean(rhs ** 2))
        rt = dev(rhs)
        worst = 0.0
        for _ in range(50):
            c = tuple(int(v) for v in rng.integers(0, n, 3))
            rt[c] += d
            lp = L_of(rt)
            rt[c] -= 2 * d
            lm = L_of(rt)
            rt[c] += d
            fd = (lp - lm) / (2 * d)
            worst = max(worst, abs(fd - g_rhs[c]) / np.abs(g_rhs).max())
        _say(f"  rhs entries: worst |fd - adjoint| / max|g_rhs| = {worst:.2e}")
        assert worst <= 1e-5
        bdev = [dev(b) for b in beta]
        worst = 0.0
        for _ in range(50):
            m = int(rng.integers(0, 3))
            c = tuple(int(v) for v in rng.integers(0, n, 3))
            bdev[m][c] += 1e-6
            s64.update_coeffs(bdev)
            lp = L_of(rt)
            bdev[m][c] -= 2e-6
            s64.update_coeffs(bdev)
            lm = L_of(rt)
            bdev[m][c] += 1e-6
            fd = (lp - lm) / 2e-6
            worst = max(worst, abs(fd - g_b[m][c]) / np.abs(g_b[m]).max())
        _say(f"  face coefficients: worst |fd - adjoint| / max|g_beta| = {worst:.2e}")
        assert worst <= 1e-4


def test_autograd_finite_differences(S):
    """Backward of the autograd Function against central differences of
    L = sum(w p) in 50 rhs entries and 50 face coefficients (FP64 solves)."""
    _say("autograd FD config4 geometry at 32^3")
    w = W.config4(32)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rhs = oracle.divergence(w.us, w.bc, w.h, 1.0 / w.dt)
    bt = [dev(b).requires_grad_(True) for b in beta]
    rt = dev(rhs).requires_grad_(True)
    wt = dev(w.w)
    with S.Solver([b.detach() for b in bt], w.h, w.bc, precision="fp32") as sol:
        p = S.pressure_solve(rt, bt, sol, tol=1e-12)
        loss = (wt * p).sum()
        loss.backward()
    g_rhs = host(rt.grad)
    g_b = [host(b.grad) for b in bt]
    rng = np.random.default_rng(3)

    def L_of(rhs_, beta_):
        with S.Solver([dev(b) for b in beta_], w.h, w.bc, precision="fp64") as s2:
            return float((wt * s2.solve(dev(rhs_), tol=1e-13)).sum())

    d = 1e-6 * np.sqrt(np.mean(rhs ** 2))
    for _ in range(50):
        c = tuple(int(v) for v in rng.integers(0, 32, 3))
        rp = rhs.copy(); rp[c] += d
        rm = rhs.copy(); rm[c] -= d
        fd = (L_of(rp, beta) - L_of(rm, beta)) / (2 * d)
        assert abs(fd - g_rhs[c]) <= 1e-5 * np.abs(g_rhs).max()
    for _ in range(50):
        m = int(rng.integers(0, 3))
        c = tuple(int(v) for v in rng.integers(0, 32, 3))
        bp = [b.copy() for b in beta]; bp[m][c] += 1e-6
        bm = [b.copy() for b in beta]; bm[m][c] -= 1e-6
        fd = (L_of(rhs, bp) - L_of(rhs, bm)) / 2e-6
        assert abs(fd - g_b[m][c]) <= 1e-4 * np.abs(g_b[m]).max()
