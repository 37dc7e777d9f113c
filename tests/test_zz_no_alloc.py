"""The entry point that allocates nothing, pp_k_smooth2_fused_dot_f32_noalloc,
against the allocating pp_k_smooth2_fused_dot_f32 through the C ABI: two calls
in a row on one GPU, the second on a smaller grid, each compared bit for bit
(e_out and the dot product) with the allocating entry point on the same
inputs.  Both launch the same kernel and the same fixed-order finalising sum,
so equality is exact."""
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


def _case(n, bc, seed):
    import oracle
    w = W.random_case(n, bc, seed=seed)
    beta = [b.astype(np.float32) for b in oracle.face_coeffs(w.rho, bc)]
    rng = np.random.default_rng(seed + 1)
    r = rng.standard_normal(w.shape).astype(np.float32)
    e0 = rng.standard_normal(w.shape).astype(np.float32)
    return w, beta, r, e0


def _f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_noalloc_matches_allocating_entry_two_calls(S):
    # the first grid fills several tiles and z chunks with a ragged last tile;
    # the second is smaller, so the second call reads fewer partial sums than
    # the first left in the shared array
    cases = [((200, 72, 40), (0, 1, 1), 0, 1.0), ((40, 20, 56), (1, 0, 1), 1, 1.3)]
    dot = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for n, bc, first, omega in cases:
        _say(f"no-alloc fused dot pass n={n} bc={bc} first_colour={first} omega={omega}")
        w, beta, r, e0 = _case(n, bc, seed=301 + n[0])
        bt = [_f32(b) for b in beta]
        ref_out = _f32(np.full(w.shape, np.nan))
        ref_dot = S.k_smooth2_fused_dot_f32(w.shape, w.h, bc, bt, _f32(r), _f32(e0), ref_out,
                                            first_colour=first, omega=omega)
        out = _f32(np.full(w.shape, np.nan))
        S.k_smooth2_fused_dot_f32_noalloc(w.shape, w.h, bc, bt, _f32(r), _f32(e0), out, dot,
                                          first_colour=first, omega=omega)
        torch.cuda.synchronize()
        got = float(dot[0].item())
        _say(f"  dot={got:.17e} allocating entry={ref_dot:.17e}")
        assert np.array_equal(out.cpu().numpy(), ref_out.cpu().numpy())
        assert got == ref_dot
