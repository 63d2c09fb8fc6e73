"""ctypes declarations of libtrg's C-ABI (include/trg.h).  Loads the in-tree
library only; there is no fallback: a missing library is an error."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrg.so")

TRG_OK, TRG_EINVAL, TRG_ENOMEM, TRG_EHIP, TRG_ESTATE, TRG_ENUMERIC = 0, -1, -2, -3, -4, -5
TRG_FP64, TRG_FP32, TRG_BF16X3, TRG_BF16X6 = 0, 1, 2, 3
TRG_HOTRG, TRG_ATRG = 0, 1
TRG_IMPURE_E, TRG_IMPURE_M = 1, 2

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TrgConfig(C.Structure):
    _fields_ = [
        ("precision", C.c_int),
        ("method", C.c_int),
        ("dcut", C.c_int),
        ("impure", C.c_uint),
        ("rsvd_p", C.c_int),
        ("rsvd_q", C.c_int),
        ("seed", C.c_uint64),
        ("stream", C.c_void_p),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_user", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
        ("fp64_steps", C.c_int),
        ("z2", C.c_int),
    ]


class TrgStepRec(C.Structure):
    _fields_ = [
        ("n", C.c_int),
        ("axis", C.c_int),
        ("dims", C.c_int * 4),
        ("side", C.c_int * 4),
        ("kept", C.c_int * 4),
        ("degenerate_cut", C.c_int * 4),
        ("sweeps", C.c_int * 4),
        ("join_precision", C.c_int),
        ("ln_c", C.c_double),
        ("eps", (C.c_double * 2) * 4),
        ("seconds", C.c_double),
    ]


# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "trg_init_ising": (C.c_int, [C.POINTER(C.c_void_p), C.c_double, C.c_double, C.c_int, C.POINTER(TrgConfig)]),
    "trg_init_tensor": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                  C.POINTER(TrgConfig)]),
    "trg_hotrg_step": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "trg_hotrg_step_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int]),
    "trg_atrg_step": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "trg_init_factors": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(TrgConfig)]),
    "trg_atrg_spectrum": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int)]),
    "trg_atrg_parities": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_size_t, C.POINTER(C.c_int), C.c_size_t,
                                    C.POINTER(C.c_int)]),
    "trg_get_factors": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t, C.POINTER(C.c_double), C.c_size_t,
                                  C.POINTER(C.c_int)]),
    "trg_run": (C.c_int, [C.c_void_p, C.c_longlong]),
    "trg_free_energy": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "trg_impure_energy": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "trg_impure_magnetization": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "trg_get_dims": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "trg_get_tensor": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_size_t]),
    "trg_get_isometry": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_size_t,
                                   C.POINTER(C.c_double), C.c_size_t]),
    "trg_step_log": (C.c_int, [C.c_void_p, C.POINTER(TrgStepRec), C.c_int, C.POINTER(C.c_int)]),
    "trg_accumulator": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "trg_export_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "trg_import_state": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.POINTER(TrgConfig)]),
    "trg_indicator_x": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double)]),
    "trg_indicator_x_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double)]),
    "trg_footprint_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint]),
    "trg_resident_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint]),
    "trg_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint]),
    "trg_share_workspace": (C.c_int, [C.c_void_p, C.c_void_p]),
    "trg_sync": (C.c_int, [C.c_void_p]),
    "trg_free": (None, [C.c_void_p]),
    "trg_last_error": (C.c_char_p, [C.c_void_p]),
    "trg_gemm": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong, C.c_longlong,
                           C.c_longlong, C.c_longlong, C.c_longlong, C.c_longlong, C.c_int, C.c_void_p]),
    "trg_gemm_tile": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "trg_eigh": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "trg_eigh_top": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int,
                               C.c_double, C.c_void_p, C.c_void_p]),
    "trg_eigh_top_work_bytes": (C.c_size_t, [C.c_int, C.c_int]),
    "trg_set_profiling": (C.c_int, [C.c_void_p, C.c_int]),
    "trg_join_profile": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_longlong),
                                   C.POINTER(C.c_double)]),
    "trg_set_force_side": (C.c_int, [C.c_void_p, C.c_int]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libtrg.so and declare every entry point.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1911_12954_amd.build` "
            "(the HIP library has no fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
