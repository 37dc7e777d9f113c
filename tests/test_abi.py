"""The C-ABI library loads and exports every declared entry point, and its
host-side validation rejects bad arguments before any GPU work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("pp.h", "pp_kernels.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(pp_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2012_11744_amd import _lib as L
    return L.load()


def test_headers_declare_the_core_calls():
    names = declared_functions()
    for core in ("pp_setup", "pp_solve", "pp_project", "pp_solve_adjoint", "pp_divergence",
                 "pp_destroy", "pp_strerror", "pp_face_coeffs", "pp_update_coeffs"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2012_11744_amd import _lib as L
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(declared_functions()) <= set(L.EXPORTS)


def test_strerror_names(lib):
    assert lib.pp_strerror(0) == b"ok"
    assert lib.pp_strerror(-1) == b"invalid argument"
    assert lib.pp_strerror(-4) == b"not converged"
    assert lib.pp_strerror(12345) == b"unknown status"


def test_opts_default(lib):
    from paper_2012_11744_amd import _lib as L
    o = L.Opts()
    lib.pp_opts_default(ctypes.byref(o))
    assert (o.precision, o.outer, o.nu_pre, o.nu_post, o.max_outer, o.warm_start, o.fallback,
            o.coarse_graph, o.nu_coarse, o.omega, o.cycle, o.coarsest) == (
                L.PP_MIXED_FP32, L.PP_OUTER_PCG, 2, 2, 500, 0, 1, 0, 4, 1.2, L.PP_CYCLE_V, 64)


def _grid(n=(8, 8, 8), h=0.125, bc=(0, 0, 0)):
    from paper_2012_11744_amd import _lib as L
    g = L.Grid()
    for m in range(3):
        g.n[m] = n[m]
        g.bc[m] = bc[m]
    g.h = h
    return g


@pytest.mark.parametrize("n,h,bc,why", [
    ((0, 8, 8), 0.1, (0, 0, 0), ">= 4"),            # empty grid
    ((3, 8, 8), 0.1, (0, 0, 0), ">= 4"),
    ((8, 8, 8), 0.0, (0, 0, 0), "h must be"),
    ((8, 8, 8), float("nan"), (0, 0, 0), "h must be"),
    ((8, 8, 8), 0.1, (0, 2, 0), "bc"),
    ((66, 66, 66), 0.1, (0, 0, 0), "1024"),          # 33^3 coarsest level
    ((256, 256, 4), 0.1, (0, 0, 0), "1024"),         # cannot coarsen a thin slab
])
def test_setup_rejects_bad_grids_without_gpu(lib, n, h, bc, why):
    from paper_2012_11744_amd import _lib as L
    g = _grid(n, h, bc)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    rc = lib.pp_setup(ctypes.byref(g), fake, fake, fake, None, None, ctypes.byref(ctx))
    assert rc == L.PP_EINVAL
    assert why in lib.pp_last_error().decode()
    assert not ctx.value


def test_setup_rejects_null_and_bad_options(lib):
    from paper_2012_11744_amd import _lib as L
    g = _grid()
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert lib.pp_setup(ctypes.byref(g), None, fake, fake, None, None, ctypes.byref(ctx)) == L.PP_EINVAL
    assert lib.pp_setup(None, fake, fake, fake, None, None, ctypes.byref(ctx)) == L.PP_EINVAL
    assert lib.pp_setup(ctypes.byref(g), fake, fake, fake, None, None, None) == L.PP_EINVAL
    for field, bad in (("precision", 7), ("outer", 3), ("nu_pre", 0), ("nu_post", 17),
                       ("max_outer", 0), ("warm_start", 2), ("coarse_graph", 5),
                       ("nu_coarse", 0), ("nu_coarse", 17), ("omega", 0.0), ("omega", 2.0),
                       ("omega", float("nan")), ("cycle", 3), ("cycle", -1),
                       ("coarsest", 0), ("coarsest", 1025)):
        o = L.Opts()
        lib.pp_opts_default(ctypes.byref(o))
        setattr(o, field, bad)
        rc = lib.pp_setup(ctypes.byref(g), fake, fake, fake, ctypes.byref(o), None, ctypes.byref(ctx))
        assert rc == L.PP_EINVAL, field
        assert "opts." + field.split("_")[0] in lib.pp_last_error().decode()


def test_calls_reject_null_context(lib):
    from paper_2012_11744_amd import _lib as L
    fake = ctypes.c_void_p(0x1000)
    assert lib.pp_solve(None, fake, fake, 1e-8, None) == L.PP_EINVAL
    assert lib.pp_project(None, fake, fake, fake, fake, 1e-3, fake, fake, fake) == L.PP_EINVAL
    assert lib.pp_solve_adjoint(None, fake, fake, 1e-8, fake, fake, fake, fake, None) == L.PP_EINVAL
    assert lib.pp_divergence(None, fake, fake, fake, 1.0, fake) == L.PP_EINVAL
    assert lib.pp_update_density(None, fake) == L.PP_EINVAL
    assert lib.pp_step(None, fake, fake, fake, fake, 1e-3, 1e-8, fake, fake, fake, fake, fake,
                       None) == L.PP_EINVAL
    lib.pp_destroy(None)  # no-op


def test_kernel_entries_validate(lib):
    from paper_2012_11744_amd import _lib as L
    fake = ctypes.c_void_p(0x1000)
    g = _grid((10, 8, 8), 0.1, (0, 0, 0))   # periodic x with an even count is fine,
    g2 = _grid((9, 8, 8), 0.1, (0, 0, 0))   # an odd periodic count is not
    assert lib.pp_k_smooth(ctypes.byref(g2), fake, fake, fake, fake, fake, 1, 0, 1.0,
                           None) == L.PP_EINVAL
    assert lib.pp_k_smooth(ctypes.byref(g), fake, fake, fake, fake, fake, 0, 0, 1.0,
                           None) == L.PP_EINVAL
    for om in (0.0, 2.0, -1.0, float("nan")):                # SOR needs 0 < omega < 2
        assert lib.pp_k_smooth(ctypes.byref(g), fake, fake, fake, fake, fake, 1, 0, om,
                               None) == L.PP_EINVAL
    g3 = _grid((9, 8, 8), 0.1, (1, 0, 0))   # the fused sweep needs even nx even with walls
    other = ctypes.c_void_p(0x2000)
    assert lib.pp_k_smooth_fused(ctypes.byref(g3), fake, fake, fake, fake, fake, other, 0, 0,
                                 1.0, None) == L.PP_EINVAL
    assert lib.pp_k_smooth_fused(ctypes.byref(g), fake, fake, fake, fake, fake, fake, 0, 0,
                                 1.0, None) == L.PP_EINVAL      # e_in aliases e_out
    assert lib.pp_k_smooth_fused(ctypes.byref(g), fake, fake, fake, fake, fake, other, 2, 0,
                                 1.0, None) == L.PP_EINVAL      # bad colour
    assert lib.pp_k_smooth_fused(ctypes.byref(g), fake, fake, fake, fake, fake, other, 0, 0,
                                 2.5, None) == L.PP_EINVAL      # bad omega
    for gg in (g3, _grid((10, 8, 6), 0.1, (1, 1, 1))):    # odd nx; a count below 8
        assert lib.pp_k_smooth2_fused_f32(ctypes.byref(gg), fake, fake, fake, fake, fake, other, 0,
                                          0, 1.0, None) == L.PP_EINVAL
    assert lib.pp_k_smooth2_fused_f32(ctypes.byref(g), fake, fake, fake, fake, fake, fake, 0, 0,
                                      1.0, None) == L.PP_EINVAL      # e_in aliases e_out
    assert lib.pp_k_smooth2_fused_f32(ctypes.byref(g), fake, fake, fake, fake, fake, other, 0, 0,
                                      0.0, None) == L.PP_EINVAL      # bad omega
    assert lib.pp_k_smooth2_fused_dot_f32(ctypes.byref(g), fake, fake, fake, fake, fake, other, 0,
                                          1.0, None, None) == L.PP_EINVAL      # no dot
    assert lib.pp_k_smooth2_fused_dot_f32(ctypes.byref(g), fake, fake, fake, fake, fake, other, 0,
                                          1.0, ctypes.c_void_p(0x1004), None) == L.PP_EINVAL   # dot misaligned
    assert lib.pp_k_smooth2_fused_dot_f32(ctypes.byref(g), fake, fake, fake, fake, fake, fake, 0,
                                          1.0, other, None) == L.PP_EINVAL     # aliasing
    assert lib.pp_k_smooth2_fused_dot_f32(ctypes.byref(g), fake, fake, fake, fake, fake, other, 0,
                                          2.0, ctypes.c_void_p(0x3000), None) == L.PP_EINVAL   # bad omega
    # the entry point that allocates nothing checks the same arguments, and
    # rejects grids whose partial sums would not fit its static array
    assert lib.pp_k_smooth2_fused_dot_f32_noalloc(ctypes.byref(g), fake, fake, fake, fake, fake,
                                                  other, 0, 1.0, None, None) == L.PP_EINVAL
    assert lib.pp_k_smooth2_fused_dot_f32_noalloc(ctypes.byref(g), fake, fake, fake, fake, fake,
                                                  fake, 0, 1.0, other, None) == L.PP_EINVAL
    assert lib.pp_k_smooth2_fused_dot_f32_noalloc(ctypes.byref(g), fake, fake, fake, fake, fake,
                                                  other, 0, -0.5, ctypes.c_void_p(0x3000),
                                                  None) == L.PP_EINVAL
    big = _grid((1024, 1024, 1024), 1.0 / 1024, (0, 0, 0))   # 16 * 128 * 128 partial sums
    assert lib.pp_k_smooth2_fused_dot_f32_noalloc(ctypes.byref(big), fake, fake, fake, fake, fake,
                                                  other, 0, 1.0, ctypes.c_void_p(0x3000),
                                                  None) == L.PP_EINVAL
    assert b"65536" in lib.pp_last_error()
    assert lib.pp_k_resid_restrict(ctypes.byref(g2), fake, fake, fake, fake, fake, fake, None) == L.PP_EINVAL
    assert lib.pp_k_prolong_add(ctypes.byref(g2), fake, fake, None) == L.PP_EINVAL
    assert lib.pp_k_prolong_add(ctypes.byref(g), fake, ctypes.c_void_p(0x1008), None) == L.PP_EINVAL   # e misaligned
    assert lib.pp_k_copy(None, fake, 10, None) == L.PP_EINVAL
    assert lib.pp_k_copy(fake, fake, 0, None) == L.PP_OK   # nothing to do


def test_entry_module_imports():
    """The build and smoke entry points are importable Python (a syntax error there would
    only show when the build is driven through them)."""
    import importlib
    import sys
    sys.path.insert(0, ROOT)
    try:
        mod = importlib.import_module("__graft_entry__")
    finally:
        sys.path.remove(ROOT)
    assert callable(mod.build) and callable(mod.smoke)
