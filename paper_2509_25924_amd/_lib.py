"""ctypes declarations of libofv.so (include/ofv.h and include/ofv_stages.h)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libofv.so")

OFV_OK = 0
OFV_ERR_INVALID_ARG = -1
OFV_ERR_UNSUPPORTED = -2
OFV_ERR_CAPACITY = -3
OFV_ERR_OUT_OF_MEMORY = -4
OFV_ERR_DEVICE = -5

PIX_U8, PIX_U16, PIX_F32 = 0, 1, 2
STORE = {"f32": 0, "f16": 1, "bf16": 2}
FLOW_IN_ZERO, FLOW_IN_DIRECT, FLOW_IN_UPSAMPLE = 0, 1, 2
MAX_LEVELS = 16
FLAG_FORWARD_ADDITIVE = 1
FLAG_INCREMENT_UPDATE = 2
FLAG_NO_FP64_FALLBACK = 4
FLAG_STORE_ALL = 8
FLAG_SAVE_ITERATES = 16
FLAG_SAVED_FORWARD = 32
BACKWARD_STORE_ALL = 1
MAX_KERNEL_RADIUS = 12
MAX_NORM_RADIUS = 16
GN_VARIANTS = {"auto": -1, "march": 0, "tile64x32": 1, "tile64x16": 2, "tile32x16": 3, "tile16x16": 4,
               "tile64x32w": 5, "tile64x16w": 6, "tile64x64": 7, "tile16x16w": 8, "tile32x16w": 9,
               "tile32x32w": 10, "band": 11}


class OfvImage(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("width", c_int32), ("height", c_int32), ("pitch", c_int64),
                ("type", c_int32), ("bit_depth", c_int32)]


class OfvParams(ctypes.Structure):
    _fields_ = [("num_levels", c_int32), ("kernel_radius", c_int32), ("iterations", c_int32),
                ("norm_radius", c_int32), ("norm_eps", c_float), ("reg_rel", c_float), ("reg_abs", c_float),
                ("storage", c_int32), ("flags", c_uint32)]


class OfvDerivedParams(ctypes.Structure):
    _fields_ = [("dx", c_float), ("dz", c_float), ("dt", c_float), ("streamwise_sign", c_int32)]


EXPORTS = {
    # name: (restype, argtypes)
    "ofv_default_params": (None, [POINTER(OfvParams)]),
    "ofv_create": (c_int, [POINTER(c_void_p), c_int, c_int, c_int, c_int, c_void_p]),
    "ofv_set_stream": (c_int, [c_void_p, c_void_p]),
    "ofv_workspace_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
    "ofv_compute_flow": (c_int, [c_void_p, POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams), c_void_p]),
    "ofv_compute_flow_ex": (c_int, [c_void_p, POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams),
                                    c_void_p, c_void_p]),
    "ofv_compute_flow_batch": (c_int, [c_void_p, c_int, POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams),
                                       POINTER(c_void_p), POINTER(c_void_p)]),
    "ofv_compute_flow_static": (c_int, [POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams), c_void_p,
                                        c_void_p]),
    "ofv_autotune_batch": (c_int, [c_void_p, c_int, POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams),
                                   POINTER(c_void_p), c_int]),
    "ofv_destroy": (c_int, [c_void_p]),
    "ofv_reserve_backward": (c_int, [c_void_p, c_int, c_int]),
    "ofv_reserve_backward_ex": (c_int, [c_void_p, c_int, c_int, c_int, c_uint32]),
    "ofv_backward_workspace_bytes": (c_int, [c_void_p, c_int, c_int, c_int, c_uint32, POINTER(c_size_t)]),
    "ofv_compute_flow_backward_batch": (c_int, [c_void_p, c_int, POINTER(OfvImage), POINTER(OfvImage),
                                                POINTER(OfvParams), POINTER(c_void_p), POINTER(c_void_p),
                                                POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p)]),
    "ofv_compute_flow_backward": (c_int, [c_void_p, POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams),
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ofv_set_gn_variant": (c_int, [c_void_p, c_int, c_int]),
    "ofv_default_derived_params": (None, [POINTER(OfvDerivedParams)]),
    "ofv_stream_push": (c_int, [c_void_p, POINTER(OfvImage), POINTER(OfvParams), c_void_p, c_void_p,
                                POINTER(c_int)]),
    "ofv_stream_reset": (c_int, [c_void_p]),
    "ofv_derived": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int64, c_void_p, c_int64, POINTER(OfvDerivedParams),
                            c_void_p, c_int64, c_void_p, c_int, c_void_p, c_void_p]),
    "ofv_stage_pyramid": (c_int, [c_void_p, c_int, c_void_p, c_int, c_int, c_int64, c_int, POINTER(c_void_p),
                                  POINTER(c_int64)]),
    "ofv_autotune": (c_int, [c_void_p, POINTER(OfvImage), POINTER(OfvImage), POINTER(OfvParams), c_void_p, c_int]),
    "ofv_tuning_export": (c_int, [c_void_p, c_char_p, c_size_t, POINTER(c_size_t)]),
    "ofv_tuning_import": (c_int, [c_void_p, c_char_p]),
    "ofv_status_string": (c_char_p, [c_int]),
    "ofv_last_error": (c_char_p, [c_void_p]),
    "ofv_stage_normalize": (c_int, [c_void_p, POINTER(OfvImage), c_int, c_float, c_int, c_void_p, c_int64]),
    "ofv_stage_reduce": (c_int, [c_void_p, c_int, c_void_p, c_int, c_int, c_int64, c_void_p, c_int64]),
    "ofv_stage_restrict_flow": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int64, c_void_p, c_int64]),
    "ofv_stage_upsample": (c_int, [c_void_p, c_void_p, c_int, c_int, c_int64, c_void_p, c_int, c_int, c_int64]),
    "ofv_stage_gn_iteration": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int, c_int, c_int64, c_int,
                                       c_void_p, c_int, c_int, c_int64, c_void_p, c_int64, c_int, c_float,
                                       c_float]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libofv.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_2509_25924_amd._build); "
                           "the OFV estimator has no non-HIP implementation")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class OfvError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def check(status: int, handle=None) -> None:
    if status == OFV_OK:
        return
    lib = load()
    msg = lib.ofv_last_error(handle)
    text = (msg.decode() if msg else "") or lib.ofv_status_string(status).decode()
    raise OfvError(status, text)
