"""ctypes binding of liblbrr.so: the C ABI of include/lbrr.h, same names.

Argument marshalling only.  The library must have been built in-tree
(``python -m paper_1505_06900_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbrr.so")

LB_D2Q9, LB_D3Q19, LB_D3Q27 = 0, 1, 2
LB_STORE_FP64, LB_STORE_FP32, LB_STORE_FP16 = 0, 1, 2
LB_STORE_MOM_FP64, LB_STORE_MOM_FP32 = 3, 4  # moment storage: rho - rho0, rho u, a1^(2) per node
LB_F64, LB_F32 = 0, 1
LB_OK = 0
LB_ERR_INVALID_ARG = -1
LB_ERR_UNSUPPORTED = -2
LB_ERR_OOM = -3
LB_ERR_HIP = -4
LB_ERR_UNSTABLE = -5
LB_ERR_STATE = -6
LB_MLP_NPARAM, LB_MLP_NNORM, LB_MLP_NIN = 6723, 78, 36
LB_REDUCE_STATIC_MAX_BLOCKS = 2048

# name -> (restype, argtypes), exactly the declarations of include/lbrr.h
_VP, _I, _D, _LL, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
SIGNATURES = {
    "lb_create": (_VP, [_I, _I, _I, _I, _D, _I]),
    "lb_config": (_I, [_VP, _I, _D]),
    "lb_set_stream": (_I, [_VP, _VP]),
    "lb_init_fields": (_I, [_VP, _VP, _VP, _VP, _I, _I]),
    "lb_step": (_I, [_VP, _LL]),
    "lb_set_check_interval": (_I, [_VP, _LL]),
    "lb_set_walls": (_I, [_VP, _I]),
    "lb_moments": (_I, [_VP, _VP, _VP, _VP, _I, _I]),
    "lb_reduce": (_I, [_VP, ctypes.POINTER(_D)]),
    "lb_reduce_static": (_I, [_I, _I, _I, _I, _I, _D, _VP, _VP, _VP]),
    "lb_enstrophy": (_I, [_VP, ctypes.POINTER(_D)]),
    "lb_get_populations": (_I, [_VP, _VP, _I]),
    "lb_set_populations": (_I, [_VP, _VP, _I]),
    "lb_step_count": (_LL, [_VP]),
    "lb_bytes_per_update": (_D, [_VP]),
    "lb_destroy": (None, [_VP]),
    "lb_last_error": (ctypes.c_char_p, []),
    "lb_probe_copy": (_I, [_VP, _VP, _SZ, _VP]),
    "lb_probe_bandwidth": (_I, [_I, _I, _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "lb_set_closure": (_I, [_VP, _VP, _VP, _I]),
    "lb_closure_features": (_I, [_VP, _VP, _D, _VP, _VP]),
    "lb_closure_coarsen": (_I, [_VP, _VP, _VP, _I, _I, _I, _I, _D, _D, _VP, _VP, _VP, _VP]),
    "lb_mlp_forward": (_I, [_VP, _VP, _VP, _LL, _VP, _VP]),
    "lb_mlp_gradient": (_I, [_VP, _VP, _VP, _VP, _LL, _VP, _I, _VP, _VP, _VP]),
    "lb_column_stats": (_I, [_VP, _LL, _I, _VP, _VP, _VP]),
    "lb_mlp_adam": (_I, [_VP, _VP, _VP, _VP, _LL, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                         _VP]),
}

_lib = None


class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def load():
    """Load liblbrr.so (raises if it has not been built).

    torch is imported first so that its HIP runtime is the one already in the
    process: the library's libamdhip64.so.7 dependency then binds to it, and
    device pointers and streams from torch are valid in the library.
    """
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (must precede the CDLL below)

        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1505_06900_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def last_error():
    return load().lb_last_error().decode()


def check(code):
    if code != LB_OK:
        raise LBError(code, last_error())
    return code
