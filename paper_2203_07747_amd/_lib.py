"""ctypes declarations of librtn.so (the C ABI in include/rtn.h)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtn.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_float = ctypes.c_float
c_void_p = ctypes.c_void_p
P = ctypes.POINTER

RTN_OK, RTN_EINVAL, RTN_ENOMEM, RTN_EHIP, RTN_ENOTSUP = 0, -1, -2, -3, -4
PREC = {"fp32": 0, "bf16": 1, "fp8": 2}
INPUT = {"full": 0, "vb": 1, "vb_u": 2}
ACT = {"silu": 0, "identity": 1}


class MlpDesc(ctypes.Structure):
    _fields_ = [("d_in", c_int32), ("d_out", c_int32), ("n_hidden", c_int32), ("width", c_int32),
                ("activation", c_int32), ("input", c_int32)]


class Quad(ctypes.Structure):
    _fields_ = [("mass", c_float), ("Jx", c_float), ("Jy", c_float), ("Jz", c_float), ("arm", c_float),
                ("c_tau", c_float), ("g", c_float)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("calls", c_int32), ("total_ms", ctypes.c_double)]


# name -> (restype, argtypes); every function returns rtn_status unless stated
SIGNATURES = {
    "rtn_version": (ctypes.c_char_p, []),
    "rtn_last_error": (ctypes.c_char_p, []),
    "rtn_param_count": (c_int32, [P(MlpDesc), P(c_int64)]),
    "rtn_model_create": (c_int32, [P(MlpDesc), c_void_p, P(c_void_p)]),
    "rtn_model_destroy": (c_int32, [c_void_p]),
    "rtn_model_set_params": (c_int32, [c_void_p, c_void_p]),
    "rtn_model_get_params": (c_int32, [c_void_p, c_void_p]),
    "rtn_model_calibrate": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "rtn_model_get_scales": (c_int32, [c_void_p, c_void_p, P(c_int32)]),
    "rtn_linearize": (c_int32, [c_void_p, c_int32, P(Quad), c_float, c_int32, c_void_p, c_int32,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p]),
    "rtn_linearize_exact": (c_int32, [c_void_p, c_int32, P(Quad), c_float, c_int32, c_void_p, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rtn_riccati": (c_int32, [c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p]),
    "rtn_riccati_noalloc": (c_int32, [c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p]),
    "rtn_linearize_second": (c_int32, [c_void_p, c_int32, c_void_p, c_float, c_int32, c_void_p, c_int32, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p]),
    "rtn_riccati_box": (c_int32, [c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  ctypes.c_double, c_int32, ctypes.c_double, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "rtn_lq_rollout": (c_int32, [c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rtn_di_param_count": (c_int32, [c_int32, c_int32, P(c_int64)]),
    "rtn_di_model_create": (c_int32, [c_int32, c_int32, c_int32, c_void_p, P(c_void_p)]),
    "rtn_di_model_destroy": (c_int32, [c_void_p]),
    "rtn_di_linearize": (c_int32, [c_void_p, c_float, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p]),
    "rtn_di_rti": (c_int32, [c_void_p, c_float, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_void_p]),
    "rtn_tune_mode": (c_int32, [c_int32]),
    "rtn_tune_get": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "rtn_tune_set": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p]),
    "rtn_tune_save": (c_int32, [ctypes.c_char_p]),
    "rtn_tune_load": (c_int32, [ctypes.c_char_p]),
    "rtn_mlp_forward": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "rtn_mlp_backward": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "rtn_model_zero_grad": (c_int32, [c_void_p, c_void_p]),
    "rtn_model_get_grad": (c_int32, [c_void_p, c_void_p]),
    "rtn_adam_step": (c_int32, [c_void_p, c_float, c_float, c_float, c_float, c_void_p]),
    "rtn_train_step": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_float, c_float,
                                 c_float, c_float, c_void_p, c_void_p]),
    "rtn_model_get_adam": (c_int32, [c_void_p, c_void_p, c_void_p, P(c_int64)]),
    "rtn_model_set_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64]),
    "rtn_profile_enable": (c_int32, [c_int32]),
    "rtn_profile_read": (c_int32, [c_void_p, c_int32, P(c_int32)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load librtn.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_07747_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class RtnError(RuntimeError):
    def __init__(self, code: int, fn: str):
        msg = load().rtn_last_error().decode(errors="replace")
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


def check(code: int, fn: str) -> None:
    if code != RTN_OK:
        raise RtnError(code, fn)
