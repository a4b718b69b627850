"""ctypes declarations of the C ABI in include/hamsim.h.

Loading fails loudly when ``libhamsim.so`` has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhamsim.so")

HS_C64, HS_C128 = 0, 1
HS_MERGE_DIAG, HS_RENORM, HS_NO_FUSE, HS_ORDER2, HS_ORDER4 = 1, 2, 4, 8, 16
STATUS = {0: "HS_OK", 1: "HS_EINVAL", 2: "HS_ENONHERMITIAN", 3: "HS_EBUDGET",
          4: "HS_ENOMEM", 5: "HS_EDEVICE", 6: "HS_ETOOLARGE"}

# every symbol the header declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_LL = ctypes.c_longlong
_SIG = {
    "hs_plan": (_I, [_I, _I, _P, _P, _D, _I, _I, ctypes.c_uint, ctypes.POINTER(_P)]),
    "hs_build_factors": (_I, [_I, _I, _P, _P, _D, _I, _I, _I, ctypes.c_uint, _P, ctypes.POINTER(_P)]),
    "hs_evolve": (_I, [_P, _P, _I, _I, _P, ctypes.c_uint]),
    "hs_factors_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                             ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_D),
                             ctypes.POINTER(_I)]),
    "hs_diag_terms": (_I, [_P, _P, _I]),
    "hs_factor_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                            ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_size_t)]),
    "hs_factor_terms": (_I, [_P, _I, _P, _I]),
    "hs_step_sequence": (_I, [_P, _P, _I, ctypes.POINTER(_I)]),
    "hs_factor_step": (_I, [_P, _I, ctypes.POINTER(_D)]),
    "hs_factor_offsets": (_I, [_P, _I, _P, _I]),
    "hs_factor_copy_diagonal": (_I, [_P, _I, _I, _LL, _LL, _P, _P]),
    "hs_factor_storage": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "hs_step_launches": (_I, [_P, _I, ctypes.c_uint, _I, ctypes.POINTER(_I), _P, _P, _I]),
    "hs_step_joint": (_I, [_P, ctypes.POINTER(_I)]),
    "hs_footprint": (_I, [_P, _I, ctypes.POINTER(ctypes.c_size_t)]),
    "hs_footprint_dtype": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_size_t)]),
    "hs_check": (_I, [_P, _P, ctypes.POINTER(_I)]),
    "hs_free_factors": (_I, [_P]),
    "hs_dia_spmv": (_I, [_I, _P, _P, _P, _P, _I, _LL, _I, _P]),
    "hs_norm2": (_I, [_P, _I, _LL, _I, _P, _P]),
    "hs_fidelity": (_I, [_P, _I, _P, _I, _I, _LL, _P, _P]),
    "hs_fidelity_noalloc": (_I, [_P, _I, _P, _I, _I, _LL, _P, _P]),
    "hs_dia_from_pauli": (_I, [_I, _I, _P, _P, _P, ctypes.POINTER(_P)]),
    "hs_dia_from_host": (_I, [_LL, _I, _P, _P, _P, ctypes.POINTER(_P)]),
    "hs_dia_info": (_I, [_P, ctypes.POINTER(_LL), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "hs_dia_offsets": (_I, [_P, _P, _I]),
    "hs_dia_copy_diagonal": (_I, [_P, _I, _LL, _LL, _P, _P]),
    "hs_dia_spgemm": (_I, [_P, _P, _P, ctypes.POINTER(_P)]),
    "hs_dia_maxabs": (_I, [_P, _P, ctypes.POINTER(_D)]),
    "hs_spme": (_I, [_P, _D, _D, _I, _I, _P, ctypes.POINTER(_P), ctypes.POINTER(_I)]),
    "hs_dia_norm_bound": (_I, [_P, _P, ctypes.POINTER(_D)]),
    "hs_taylor_terms": (_I, [_P, _D, _D, _I, _P, ctypes.POINTER(_I)]),
    "hs_taylor_steps": (_I, [_P, _D, _D, _P, ctypes.POINTER(_I)]),
    "hs_taylor_evolve": (_I, [_P, _P, _I, _D, _I, _I, _P]),
    "hs_estimate_timesteps": (_I, [_P, _D, _I, _D, _I, _P, ctypes.POINTER(_I)]),
    "hs_dia_to_c64": (_I, [_P, _P, ctypes.POINTER(_P)]),
    "hs_dia_evolve": (_I, [_P, _P, _I, _I, _P]),
    "hs_dia_free": (_I, [_P]),
    "hs_last_error": (ctypes.c_char_p, []),
    "hs_abi_version": (_I, []),
}

_lib = None


class HamsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2606_16959_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int):
    if status != 0:
        raise HamsimError(status, load().hs_last_error().decode())
