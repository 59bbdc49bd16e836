"""ctypes loader and signatures of libdgw.so (the C ABI of include/dgw.h)."""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

DGW_OK = 0
STATUS = {0: "DGW_OK", -1: "DGW_EINVAL", -2: "DGW_ENOMEM", -3: "DGW_EMESH",
          -4: "DGW_EHIP", -5: "DGW_ESTATE", -6: "DGW_ERANGE",
          -7: "DGW_ENONFINITE", -8: "DGW_EGROWTH"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64 = C.c_int64
_PI64 = C.POINTER(C.c_int64)

# name -> (restype, argtypes); the exported symbol list of include/dgw.h
SIGNATURES = {
    "dgw_create": (C.c_int, [C.c_int, C.c_int, C.c_int, _P, C.POINTER(_P)]),
    "dgw_destroy": (None, [_P]),
    "dgw_last_error": (C.c_char_p, [_P]),
    "dgw_set_allocator": (C.c_int, [_P, ALLOC_FN, FREE_FN, _P]),
    "dgw_set_mesh": (C.c_int, [_P, _I64, _D, _I64, C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32), C.POINTER(C.c_int8)]),
    "dgw_set_material": (C.c_int, [_P, _D, _D, _D]),
    "dgw_suggest_dt": (C.c_int, [_P, C.c_double, _D]),
    "dgw_set_dt": (C.c_int, [_P, C.c_double]),
    "dgw_set_source": (C.c_int, [_P, C.c_int, _D, _D, C.c_double, C.c_double,
                                 C.c_double, _I64]),
    "dgw_set_receivers": (C.c_int, [_P, C.c_int, C.c_int, _D, _I64]),
    "dgw_set_fields": (C.c_int, [_P, C.c_int, _D]),
    "dgw_get_fields": (C.c_int, [_P, C.c_int, _D]),
    "dgw_set_shot_step": (C.c_int, [_P, C.c_int, _I64]),
    "dgw_step": (C.c_int, [_P, _I64]),
    "dgw_read_traces": (C.c_int, [_P, C.c_int, _D, _I64, _PI64]),
    "dgw_shot_steps": (C.c_int, [_P, C.c_int, _PI64]),
    "dgw_energy": (C.c_int, [_P, C.c_int, _D]),
    "dgw_energy_noalloc": (C.c_int, [_P, C.c_int, _D]),
    "dgw_check_finite": (C.c_int, [_P]),
    "dgw_set_watchdog": (C.c_int, [_P, _I64, C.c_double]),
    "dgw_ref_nodes": (C.c_int, [C.c_int, _D]),
    "dgw_ref_operators": (C.c_int, [C.c_int, _D, _D, _D, _D, _D]),
    "dgw_order_elements": (C.c_int, [_I64, _D, _I64, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.c_int, _PI64]),
    "dgw_forward_checkpointed": (C.c_int, [_P, _I64, _I64, _D, _D]),
    "dgw_adjoint": (C.c_int, [_P, _D, _D, _D]),
    "dgw_state_generation": (C.c_int, [_P, C.POINTER(C.c_uint64)]),
    "dgw_autotune": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "dgw_set_launch": (C.c_int, [_P, C.c_int, C.c_int, C.c_int]),
    "dgw_set_flux": (C.c_int, [_P, C.c_double]),
    "dgw_set_damping": (C.c_int, [_P, _D]),
    "dgw_set_pml": (C.c_int, [_P, _I64, C.POINTER(C.c_int32), _D]),
    "dgw_get_pml_memory": (C.c_int, [_P, C.c_int, _D]),
    "dgw_set_pml_memory": (C.c_int, [_P, C.c_int, _D]),
    "dgw_pml_kernel_ms": (C.c_int, [_P, _D, _PI64]),
    "dgw_set_stiffness": (C.c_int, [_P, _D]),
    "dgw_set_adjoint_memory": (C.c_int, [_P, _I64]),
    "dgw_enable_timing": (C.c_int, [_P, C.c_int]),
    "dgw_stage_kernel_ms": (C.c_int, [_P, _D, _PI64]),
    "dgw_adjoint_stage_ms": (C.c_int, [_P, _D, _PI64]),
    "dgw_sizes": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), _PI64]),
}


class LibraryMissingError(RuntimeError):
    pass


def library_path():
    return os.environ.get("DGW_LIBRARY", os.path.join(_HERE, "libdgw.so"))


def load():
    """Load libdgw.so (built by paper_2205_11052_amd/build.py).  There is no
    fallback: a missing library is an error."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise LibraryMissingError(
            "libdgw.so not found at %s; build it with "
            "`python -m paper_2205_11052_amd.build`" % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
