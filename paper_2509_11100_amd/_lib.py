"""ctypes declarations of librelsim.so (include/relsim.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librelsim.so")

RELSIM_OK = 0
RELSIM_EINVAL = -1
RELSIM_ENOTCONVERGED = -2
RELSIM_EHIP = -3
RELSIM_ENONFINITE = -4
RELSIM_ERANGE = -5
RELSIM_EINTERNAL = -6
RELSIM_FP64 = 0
RELSIM_MIXED = 1


class relsim_params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("dt", C.c_double), ("c", C.c_double), ("theta", C.c_double),
        ("precision", C.c_int32), ("nspecies", C.c_int32),
        ("q", C.c_double * 8), ("m", C.c_double * 8),
        ("max_particles", C.c_int64),
        ("gmres_rtol", C.c_double), ("gmres_restart", C.c_int32), ("gmres_maxit", C.c_int32),
        ("nonrelativistic", C.c_int32), ("group", C.c_int32), ("mass_fp32", C.c_int32),
    ]


class relsim_particles(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("bin_start", C.c_void_p), ("cell", C.c_void_p),
        ("xy", C.c_void_p), ("uw", C.c_void_p), ("z", C.c_void_p),
        ("bin_start_back", C.c_void_p), ("cell_back", C.c_void_p),
        ("xy_back", C.c_void_p), ("uw_back", C.c_void_p), ("z_back", C.c_void_p),
        ("species", C.c_void_p),
    ]


class RelsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("relsim error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load librelsim.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("librelsim.so is not built (run: python -m paper_2509_11100_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    pp = C.POINTER(relsim_params)
    pt = C.POINTER(relsim_particles)
    dp = C.POINTER(C.c_double)
    i32 = C.c_int32
    sig = {
        "relsim_workspace_bytes": (C.c_size_t, [pp]),
        "relsim_init": (C.c_int, [pp, vp, vp, C.c_size_t, C.POINTER(vp)]),
        "relsim_finalize": (None, [vp]),
        "relsim_sort": (C.c_int, [vp, pt]),
        "relsim_deposit_moments": (C.c_int, [vp, pt, vp, vp, vp]),
        "relsim_field_solve": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i32), dp]),
        "relsim_field_solve_guess": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i32), dp]),
        "relsim_push": (C.c_int, [vp, pt, vp, vp, i32, vp]),
        "relsim_deposit_moments_ec": (C.c_int, [vp, pt, vp, vp, vp, vp]),
        "relsim_gamma_mean": (C.c_int, [vp, pt, vp, vp, vp, vp, dp]),
        "relsim_gamma_secant": (C.c_int, [vp, C.c_int64, vp, vp, vp, vp, C.c_int]),
        "relsim_push_ec": (C.c_int, [vp, pt, vp, vp, vp, i32, vp]),
        "relsim_apply_AT": (C.c_int, [vp, vp, vp, vp]),
        "relsim_push_adjoint": (C.c_int, [vp, pt, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "relsim_field_solve_adjoint": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i32), dp]),
        "relsim_deposit_adjoint": (C.c_int, [vp, pt, vp, vp, vp, vp, vp, vp]),
        "relsim_energy": (C.c_int, [vp, pt, vp, vp, dp]),
        "relsim_fill_cells": (C.c_int, [vp, pt]),
        "relsim_placement_clamps": (C.c_int, [vp, C.POINTER(C.c_int64)]),
        "relsim_energy_noalloc": (C.c_int, [pp, vp, pt, vp, vp, vp]),
        "relsim_energy_pushed": (C.c_int, [vp, vp, vp, dp]),
        "relsim_curl_nc": (C.c_int, [vp, vp, vp]),
        "relsim_curl_cn": (C.c_int, [vp, vp, vp]),
        "relsim_apply_A": (C.c_int, [vp, vp, vp, vp]),
        "relsim_timing_enable": (C.c_int, [vp, i32]),
        "relsim_timing_reset": (C.c_int, [vp]),
        "relsim_timing_read": (C.c_int, [vp, i32, C.c_void_p, dp, C.POINTER(C.c_int64)]),
        "relsim_strerror": (C.c_char_p, [C.c_int]),
        "relsim_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C functions this binding expects the library to export."""
    return [
        "relsim_workspace_bytes", "relsim_init", "relsim_finalize", "relsim_sort", "relsim_deposit_moments",
        "relsim_field_solve", "relsim_field_solve_guess", "relsim_push", "relsim_fill_cells", "relsim_energy", "relsim_curl_nc", "relsim_curl_cn",
        "relsim_apply_A", "relsim_apply_AT", "relsim_push_adjoint", "relsim_field_solve_adjoint",
        "relsim_deposit_adjoint", "relsim_timing_enable", "relsim_timing_reset", "relsim_timing_read",
        "relsim_strerror", "relsim_last_error", "relsim_deposit_moments_ec", "relsim_gamma_mean", "relsim_gamma_secant", "relsim_push_ec",
        "relsim_placement_clamps", "relsim_energy_noalloc", "relsim_energy_pushed",
    ]
