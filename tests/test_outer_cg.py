"""The outer flexible conjugate-gradient bookkeeping of the GPU path (CPU).

The GPU outer loop keeps the search direction in units of the V-cycle's scale
s_k and never forms r_{k+1} . z_k from the vectors: since
alpha_k (D_k . A D_k) = r_k . z_k and D_k - z_k = beta_k D_{k-1},
r_{k+1} . z_k = alpha_k beta_k (D_{k-1} . A D_k), which the direction pass
sums as D_old . q.  These tests run that bookkeeping in FP64 numpy, slot for
slot, with a preconditioner that changes from one iteration to the next (red-
black sweeps of the paper's relaxation, a different count each time), and
check it against the textbook flexible (Polak-Ribiere) iteration in true units
and against the direct dot products.
"""
import numpy as np

import oracle
from paper_2012_11744_amd import workloads as W


def _setup():
    w = W.random_case((12, 10, 8), (1, 0, 1), seed=141, ratio=1000.0)
    beta = oracle.face_coeffs(w.rho, w.bc)
    rng = np.random.default_rng(142)
    b = rng.standard_normal(w.shape)
    b -= b.mean()
    A = lambda x: oracle.apply(beta, w.bc, w.h, x)

    def M(k, r):   # linear in r for each k; differs between iterations
        z, _, _ = oracle.rbsor(beta, w.bc, w.h, r, omega=1.0, sweeps=2 + (k % 3))
        return z

    return A, M, b


def _textbook(A, M, b, iters):
    """Flexible CG in true units: beta = (r_k.z_k - r_k.z_{k-1}) / (r_{k-1}.z_{k-1})."""
    x = np.zeros_like(b)
    r = b.copy()
    d = z_old = rz_prev = None
    xs, rzold_direct = [], []
    for k in range(iters):
        z = M(k, r)
        rz = float(np.vdot(r, z))
        if k == 0:
            d = z.copy()
        else:
            bet = (rz - float(np.vdot(r, z_old))) / rz_prev
            d = z + bet * d
        q = A(d)
        alpha = rz / float(np.vdot(d, q))
        x = x + alpha * d
        r = r - alpha * q
        rzold_direct.append(float(np.vdot(r, z)))   # r_{k+1} . z_k
        z_old, rz_prev = z, rz
        xs.append(x.copy())
    return xs, rzold_direct


def _stored_units(A, M, b, iters):
    """The GPU's slots: S_USED = s_k (RMS of the residual), the V-cycle on
    r / s_k, D stored divided by s_k, alpha stored times s_k, S_RZOLD from
    D_old . q (the finalising steps OP_RZ, OP_ALPHA, OP_UPDATE)."""
    x = np.zeros_like(b)
    r = b.copy()
    s_used = float(np.sqrt(np.mean(r * r)))
    D = None
    RZ = RZOLD = DS = 0.0
    xs, rzold_slot, rzold_check, rzs = [], [], [], []
    for k in range(iters):
        zst = M(k, r / s_used)                          # V-cycle on the scaled residual
        rz = s_used * float(np.vdot(r, zst))            # OP_RZ
        gamma = 0.0 if k == 0 else (rz - RZOLD) / RZ * (DS / s_used)
        RZ = rz
        Dold = np.zeros_like(b) if D is None else D
        D = zst + gamma * Dold                          # direction pass
        q = A(D)
        s0 = float(np.vdot(D, q))
        s1 = float(np.vdot(Dold, q))
        alpha = RZ / (s_used * s0)                      # OP_ALPHA
        DS = s_used
        RZOLD = alpha * gamma * s_used * s1
        x = x + alpha * D
        r = r - alpha * q                               # residual update
        rzold_slot.append(RZOLD)
        rzs.append(RZ)
        rzold_check.append(s_used * float(np.vdot(r, zst)))   # r_{k+1} . z_k from the vectors
        s_used = float(np.sqrt(np.mean(r * r)))          # OP_UPDATE: the next scale
        xs.append(x.copy())
    return xs, rzold_slot, rzold_check, rzs


def test_rz_old_from_direction_pass_equals_direct_dot():
    A, M, b = _setup()
    _, slot, check, rzs = _stored_units(A, M, b, 8)
    assert slot[0] == 0.0
    for k, (a, c, rz) in enumerate(zip(slot, check, rzs)):
        # r_{k+1} . z_k is small against r_k . z_k, the size of the terms
        # either way forms it from: the two agree to rounding of that size
        assert abs(a - c) <= 1e-12 * abs(rz), (k, a, c, rz)
    # and it is not zero: the preconditioner changes between iterations
    assert max(abs(c) / abs(rz) for c, rz in zip(check[1:], rzs[1:])) > 1e-6


def test_stored_units_follow_the_textbook_iteration():
    A, M, b = _setup()
    xs_t, direct = _textbook(A, M, b, 8)
    xs_s, slot, _, _ = _stored_units(A, M, b, 8)
    for k, (xt, xsk) in enumerate(zip(xs_t, xs_s)):
        err = np.max(np.abs(xt - xsk)) / np.max(np.abs(xt))
        assert err < 1e-10, (k, err)
    # the slot's r_{k+1} . z_k is the textbook value in true units
    for a, c in zip(slot[1:], direct[1:]):
        assert abs(a - c) <= 1e-8 * abs(c) + 1e-14, (a, c)
    # the iteration converges (a plain check that it is a working solver)
    r_last = b - A(xs_s[-1])
    assert np.linalg.norm(r_last) < 1e-2 * np.linalg.norm(b)
