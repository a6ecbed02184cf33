"""ctypes declarations of the C ABI in ``include/mg355.h`` (argument marshalling only).

The library is ``paper_2302_13903_amd/_build/libmg355.so`` (built by ``build.py``).  Loading
fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libmg355.so")
HEADER = os.path.join(HERE, "..", "include", "mg355.h")

MG_OK, MG_NOT_CONVERGED, MG_STALLED = 0, 1, 2
MG_ERR_INVALID_ARG, MG_ERR_UNSUPPORTED, MG_ERR_OOM, MG_ERR_DEVICE, MG_ERR_NONFINITE = -1, -2, -3, -4, -5
MG_BC_PERIODIC, MG_BC_ZERO_GRADIENT, MG_BC_FIXED, MG_BC_MULTIPOLE = 0, 1, 2, 3
MG_MODE_FMG, MG_MODE_MGI = 0, 1
MG_PREC_FP64, MG_PREC_MIXED = 0, 1
MG_LAYOUT_DENSE, MG_LAYOUT_BLOCKS = 0, 1
MG_SCHEME_CS, MG_SCHEME_FAS = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "STALLED", -1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "OOM",
                -4: "DEVICE", -5: "NONFINITE"}


class MgParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("dx", ctypes.c_double), ("four_pi_g", ctypes.c_double),
                ("mode", ctypes.c_int), ("npre", ctypes.c_int), ("npost", ctypes.c_int),
                ("omega", ctypes.c_double), ("tol", ctypes.c_double), ("max_cycles", ctypes.c_int),
                ("fixed_cycles", ctypes.c_int), ("precision", ctypes.c_int), ("layout", ctypes.c_int),
                ("block_n", ctypes.c_int), ("scheme", ctypes.c_int)]


class MgBC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int * 6), ("fixed_b", ctypes.c_void_p * 6), ("lmax", ctypes.c_int),
                ("use_origin", ctypes.c_int), ("origin", ctypes.c_double * 3)]


MG_AMR_MAX_LEVELS = 8


class MgAmrMesh(ctypes.Structure):
    _fields_ = [("NB", ctypes.c_int), ("nb", ctypes.c_int), ("levels", ctypes.c_int),
                ("box_lo", (ctypes.c_int * 3) * MG_AMR_MAX_LEVELS), ("box_hi", (ctypes.c_int * 3) * MG_AMR_MAX_LEVELS)]


class MgLevelBC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int * 6), ("b", ctypes.c_void_p * 6)]


MG_SERVE_FIFO, MG_SERVE_SKIP = 0, 1


class MgServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("workers", ctypes.c_int), ("hbm_budget", ctypes.c_size_t),
                ("policy", ctypes.c_int), ("simulate", ctypes.c_int)]


class MgRequest(ctypes.Structure):
    _fields_ = [("params", MgParams), ("bc", MgBC), ("rho", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("arrival_ms", ctypes.c_double), ("sim_ms", ctypes.c_double), ("hist_cap", ctypes.c_int),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("status", ctypes.c_int), ("n_hist", ctypes.c_int),
                ("resid", ctypes.c_double), ("admit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("end_ms", ctypes.c_double), ("worker", ctypes.c_int), ("reused", ctypes.c_int)]


class MgServerStats(ctypes.Structure):
    _fields_ = [("created", ctypes.c_int), ("reused", ctypes.c_int), ("evicted", ctypes.c_int),
                ("rejected", ctypes.c_int), ("max_concurrent", ctypes.c_int), ("resident_bytes", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t)]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class MgError(RuntimeError):
    pass


def lib():
    """Load libmg355.so and declare every entry point; raises when the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MgError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    d = ctypes.c_double
    i = ctypes.c_int
    sig = {
        "mg_default_params": (None, [ctypes.POINTER(MgParams)]),
        "mg_ctx_create": (i, [ctypes.POINTER(_vp), i, ctypes.c_size_t]),
        "mg_ctx_destroy": (None, [_vp]),
        "mg_last_error": (ctypes.c_char_p, [_vp]),
        "mg_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(MgParams)]),
        "mg_ctx_reserve": (i, [_vp, ctypes.POINTER(MgParams)]),
        "mg_autotune": (i, [_vp, ctypes.POINTER(MgParams), i]),
        "mg_tuning_get": (i, [_vp, ctypes.c_char_p, i]),
        "mg_tuning_set": (i, [_vp, ctypes.c_char_p]),
        "mg_server_create": (i, [ctypes.POINTER(_vp), ctypes.POINTER(MgServerConfig)]),
        "mg_server_destroy": (None, [_vp]),
        "mg_server_last_error": (ctypes.c_char_p, [_vp]),
        "mg_server_reserve": (i, [_vp, ctypes.POINTER(MgParams), i]),
        "mg_server_run": (i, [_vp, ctypes.POINTER(MgRequest), i]),
        "mg_server_get_stats": (i, [_vp, ctypes.POINTER(MgServerStats)]),
        "mg_solve": (i, [_vp, ctypes.POINTER(MgParams), ctypes.POINTER(MgBC), _vp, _vp, _dp, _ip, _vp]),
        "mg_solve_noalloc": (i, [_vp, ctypes.POINTER(MgParams), ctypes.POINTER(MgBC), _vp, _vp, _dp, _ip, _vp]),
        "mg_solve_simple": (i, [_vp, i, _vp, i, d, d, _vp, _dp, _ip, _vp]),
        "mg_last_timing": (i, [_vp, _dp, _dp, _dp, i, _ip]),
        "mg_last_inner": (i, [_vp, _ip]),
        "mg_set_kernel_timing": (i, [_vp, i]),
        "mg_kernel_timing": (i, [_vp, i, _ip, _dp, _dp, ctypes.c_char_p, i]),
        "mg_multipole_moments": (i, [_vp, i, d, _vp, i, i, _dp, _dp, _dp, _vp]),
        "mg_gravity": (i, [_vp, ctypes.POINTER(MgParams), ctypes.POINTER(MgBC), _vp, _vp, _vp, _vp, _vp, _vp]),
        "mg_amr_patch_dims": (i, [ctypes.POINTER(MgAmrMesh), i, _ip]),
        "mg_amr_solve": (i, [_vp, ctypes.POINTER(MgParams), ctypes.POINTER(MgAmrMesh), ctypes.POINTER(MgBC),
                             ctypes.POINTER(_vp), ctypes.POINTER(_vp), _dp, _ip, _vp]),
        "mg_gravity_kernel_name": (i, [ctypes.POINTER(MgParams), i, i, i, ctypes.c_char_p, i]),
        "mg_op_half_sweep": (i, [_vp, i, d, d, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_smooth": (i, [_vp, i, d, d, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_fill": (i, [_vp, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_defect": (i, [_vp, i, d, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp, _vp]),
        "mg_op_restrict": (i, [_vp, i, _vp, _vp, _vp]),
        "mg_op_prolong_add": (i, [_vp, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_prolong_fmg": (i, [_vp, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_coarsest": (i, [_vp, d, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_down": (i, [_vp, i, d, d, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp, _vp, _vp]),
        "mg_op_smooth_f32": (i, [_vp, i, d, d, i, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp]),
        "mg_op_down_f32": (i, [_vp, i, d, d, i, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp, _vp, _vp]),
        "mg_op_up_f32": (i, [_vp, i, d, d, i, ctypes.POINTER(MgLevelBC), ctypes.POINTER(MgLevelBC), _vp, _vp, _vp,
                             _vp]),
        "mg_op_sweep_input_norm": (i, [_vp, i, d, d, ctypes.POINTER(MgLevelBC), _vp, _vp, _dp, _vp]),
        "mg_op_mixed_update": (i, [_vp, i, d, ctypes.POINTER(MgLevelBC), _vp, _vp, _vp, _vp, _dp, _vp]),
        "mg_op_up": (i, [_vp, i, d, d, i, ctypes.POINTER(MgLevelBC), ctypes.POINTER(MgLevelBC), _vp, _vp, _vp,
                         _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def declared_functions():
    """Names of the functions declared in include/mg355.h (for the export check)."""
    import re
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", src)))
