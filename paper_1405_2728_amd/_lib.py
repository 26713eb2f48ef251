"""ctypes declarations of the C ABI in include/mm.h."""

import ctypes as C
import os

from ._build import lib_path

MM_FP64, MM_MIXED = 0, 1
STATUS = {
    0: "MM_OK", 1: "MM_NOT_CONVERGED", 2: "MM_STALLED", -1: "MM_EINVAL", -2: "MM_ENOMEM",
    -3: "MM_EHIP", -4: "MM_ENONFINITE", -5: "MM_ESTATE", -6: "MM_EUNSUPPORTED",
}


class StepInfo(C.Structure):
    _fields_ = [("tau", C.c_double), ("torque", C.c_double), ("energy", C.c_double),
                ("k", C.c_int64)]


class MinResult(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int64), ("heff_evals", C.c_int64),
                ("torque", C.c_double), ("energy", C.c_double)]


# name -> (restype, argtypes)
SIGNATURES = {
    "mm_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_void_p]),
    "mm_destroy": (None, [C.c_void_p]),
    "mm_set_geometry": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                  C.c_double, C.c_double]),
    "mm_set_material": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_double), C.c_void_p]),
    "mm_set_field": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double)]),
    "mm_reset": (C.c_int, [C.c_void_p, C.c_int]),
    "mm_heff": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "mm_heff_static": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "mm_field_terms": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "mm_energy": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_double),
                            C.POINTER(C.c_double)]),
    "mm_minimize_step": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(StepInfo)]),
    "mm_minimize_to_tol": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_int64,
                                     C.POINTER(MinResult)]),
    "mm_hysteresis_sweep": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_double),
                                      C.c_int, C.c_double, C.c_int64, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]),
    "mm_mean": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    "mm_hessvec": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mm_adjoint_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_double, C.c_int64, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]),
    "mm_param_grads": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_void_p]),
    "mm_energy_grads": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(C.c_double)]),
    "mm_set_option": (C.c_int, [C.c_void_p, C.c_char_p, C.c_double]),
    "mm_minimize_continue": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_int64,
                                       C.POINTER(MinResult)]),
    "mm_state_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]),
    "mm_state_save": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "mm_state_load": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "mm_last_step": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(StepInfo)]),
    "mm_counters": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mm_rows_per_block": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "mm_yz_variant": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "mm_supported": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "mm_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "mm_profile_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_int64)]),
    "mm_kernel_name": (C.c_char_p, [C.c_int]),
    "mm_kernel_bytes": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "mm_strerror": (C.c_char_p, [C.c_int]),
    "mm_last_error": (C.c_char_p, [C.c_void_p]),
}

_LIB = None


def load():
    """Load libmmbb.so (built in-tree).  Raises if it is missing: there is no
    fallback path."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError("HIP library %s is not built; run __graft_entry__.build() or "
                          "python -m paper_1405_2728_amd._build" % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
