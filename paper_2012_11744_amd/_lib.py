"""ctypes view of the C ABI in include/pp.h and include/pp_kernels.h.

Loading fails loudly (ImportError) when the HIP library has not been built:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# PP_LIB names another build of the same library (a sanitizer build of the
# host code, for example); by default the in-tree libpp.so
LIB_PATH = os.environ.get("PP_LIB") or os.path.join(HERE, "libpp.so")

PP_OK = 0
PP_EINVAL = -1
PP_ENOMEM = -2
PP_EHIP = -3
PP_ENOCONV = -4
PP_EDIVERGED = -5

PP_PERIODIC = 0
PP_WALL = 1

PP_FP64 = 0
PP_MIXED_FP32 = 1
PP_MIXED_FP16 = 2

PP_OUTER_PCG = 0
PP_OUTER_DC = 1

PP_CYCLE_V = 0
PP_CYCLE_W = 1
PP_CYCLE_F = 2

PP_HIST = 128

PP_KT_SMOOTH = 0
PP_KT_RESTRICT = 1
PP_KT_PROLONG = 2
PP_KT_OUTER_APPLY = 3
PP_KT_OUTER_UPDATE = 4
PP_KT_COUNT = 5


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double), ("bc", ctypes.c_int32 * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("coarse_graph", ctypes.c_int32),
                ("nu_coarse", ctypes.c_int32), ("omega", ctypes.c_double),
                ("cycle", ctypes.c_int32), ("coarsest", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("vcycles", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("res_hist", ctypes.c_double * PP_HIST),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        n = min(self.outer_iters, PP_HIST)
        return {"outer_iters": self.outer_iters, "vcycles": self.vcycles,
                "fell_back": bool(self.fell_back), "status": self.status,
                "rel_res": self.rel_res, "res_hist": list(self.res_hist[:n]), "ms": self.ms}


EXPORTS = [
    "pp_opts_default", "pp_face_coeffs", "pp_setup", "pp_setup_general", "pp_update_coeffs", "pp_update_density",
    "pp_update_general", "pp_divergence",
    "pp_apply", "pp_solve", "pp_project", "pp_step", "pp_solve_adjoint", "pp_levels", "pp_level_dims",
    "pp_memory", "pp_destroy", "pp_strerror", "pp_last_error",
    "pp_k_smooth", "pp_k_smooth_fused", "pp_k_smooth2_fused_f32", "pp_k_smooth2_fused_dot_f32",
    "pp_k_smooth2_fused_dot_f32_noalloc", "pp_k_resid_restrict", "pp_k_prolong_add",
    "pp_k_prolong_weights", "pp_k_prolong_add_weighted", "pp_k_coarsen_beta", "pp_vcycle",
    "pp_k_copy", "pp_timing_enable", "pp_timing_reset", "pp_timing_get",
]

_lib = None


def load():
    """Load libpp.so and declare every signature; raises ImportError if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2012_11744_amd.build` "
                          "(hipcc, gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I32 = ctypes.c_int32
    D = ctypes.c_double
    GP = ctypes.POINTER(Grid)
    OP = ctypes.POINTER(Opts)
    SP = ctypes.POINTER(Stats)
    sig = {
        "pp_opts_default": (None, [OP]),
        "pp_face_coeffs": (I, [GP, P, P, P, P, P]),
        "pp_setup": (I, [GP, P, P, P, OP, P, ctypes.POINTER(P)]),
        "pp_setup_general": (I, [GP, P, P, P, P, OP, P, ctypes.POINTER(P)]),
        "pp_update_coeffs": (I, [P, P, P, P]),
        "pp_update_density": (I, [P, P]),
        "pp_update_general": (I, [P, P, P, P, P]),
        "pp_divergence": (I, [P, P, P, P, D, P]),
        "pp_apply": (I, [P, P, P]),
        "pp_solve": (I, [P, P, P, D, SP]),
        "pp_project": (I, [P, P, P, P, P, D, P, P, P]),
        "pp_step": (I, [P, P, P, P, P, D, D, P, P, P, P, P, SP]),
        "pp_solve_adjoint": (I, [P, P, P, D, P, P, P, P, SP]),
        "pp_levels": (I, [P, ctypes.POINTER(I32)]),
        "pp_level_dims": (I, [P, I32, ctypes.POINTER(I32)]),
        "pp_memory": (I, [P, ctypes.POINTER(ctypes.c_int64)]),
        "pp_destroy": (None, [P]),
        "pp_strerror": (ctypes.c_char_p, [I]),
        "pp_last_error": (ctypes.c_char_p, []),
        "pp_k_smooth": (I, [GP, P, P, P, P, P, I32, I32, D, P]),
        "pp_k_smooth_fused": (I, [GP, P, P, P, P, P, P, I32, I32, D, P]),
        "pp_k_smooth2_fused_f32": (I, [GP, P, P, P, P, P, P, I32, I32, D, P]),
        "pp_k_smooth2_fused_dot_f32": (I, [GP, P, P, P, P, P, P, I32, D, P, P]),
        "pp_k_smooth2_fused_dot_f32_noalloc": (I, [GP, P, P, P, P, P, P, I32, D, P, P]),
        "pp_k_resid_restrict": (I, [GP, P, P, P, P, P, P, P]),
        "pp_k_prolong_add": (I, [GP, P, P, P]),
        "pp_k_prolong_weights": (I, [GP, P, P, P, P, P]),
        "pp_k_prolong_add_weighted": (I, [GP, P, P, P, P]),
        "pp_k_coarsen_beta": (I, [GP, P, P, P, P, P, P, P]),
        "pp_vcycle": (I, [P, P, P]),
        "pp_k_copy": (I, [P, P, ctypes.c_int64, P]),
        "pp_timing_enable": (I, [P, I32]),
        "pp_timing_reset": (I, [P]),
        "pp_timing_get": (I, [P, I32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class PPError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load()
        self.code = code
        self.detail = lib.pp_last_error().decode(errors="replace")
        name = lib.pp_strerror(code).decode()
        super().__init__(f"{where}: {name} ({code}): {self.detail}")


def check(code: int, where: str) -> int:
    if code != PP_OK:
        raise PPError(code, where)
    return code
