"""ctypes declarations of libartemis.so (the C ABI in include/artemis.h).

Argument marshalling only: every step of the renderer runs in the library's
HIP kernels.  Importing this module fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# ARTEMIS_LIB selects another build of the library (e.g. a tuning variant)
LIB_PATH = os.environ.get("ARTEMIS_LIB") or os.path.join(HERE, "libartemis.so")

ART_OK, ART_EINVAL, ART_ENOMEM, ART_EDEVICE, ART_ESTATE, ART_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ART_F32, ART_BF16 = 0, 1
ART_GEOM_FP32 = 1
ART_TIMING = 2
ART_PROPOSAL_MARGIN_H = 2.0
ART_PROPOSAL_NEAR_ONLY = 4
ART_REUSE_BUILD = 8
ART_NUM_STATS = 15
ART_ASYNC = 16
ART_SHADING_NOALLOC_BYTES = 100663296

STATUS_NAMES = {0: "ART_OK", -1: "ART_EINVAL", -2: "ART_ENOMEM", -3: "ART_EDEVICE",
                -4: "ART_ESTATE", -5: "ART_EUNSUPPORTED"}

# (name, restype, argtypes) of every exported function
_P = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint
_F = ctypes.c_float
_L = ctypes.c_int64
SIGNATURES = [
    ("art_version", _I, []),
    ("art_create", _I, [_I, _P, ctypes.POINTER(_P)]),
    ("art_destroy", None, [_P]),
    ("art_last_error", ctypes.c_char_p, [_P]),
    ("art_state_version", ctypes.c_uint64, [_P]),
    ("art_set_memory_limit", _I, [_P, _L]),
    ("art_get_memory", _I, [_P, _P, _P]),
    ("art_load_octree", _I, [_P, _I, _L, _P]),
    ("art_set_skin", _I, [_P, _P, _P]),
    ("art_set_skeleton", _I, [_P, _I, _P, _P]),
    ("art_set_poses", _I, [_P, _I, _P, _P, _P]),
    ("art_set_cameras", _I, [_P, _I, _I, _I, _P, _P]),
    ("art_render", _I, [_P, _I, _I, _P, _P, _F, _U, _P, _P, _P]),
    ("art_backward", _I, [_P, _I, _I, _P, _P, _F, _U, _P, _P, _P, _P, _P, _P]),
    ("art_render_ckpt", _I, [_P, _I, _I, _P, _P, _F, _U, _P, _P, _P, _I, _I, _P, _P]),
    ("art_backward_ckpt", _I, [_P, _I, _I, _P, _P, _F, _U, _P, _P, _P, _P, _P, _P, _I, _I, _P, _P]),
    ("art_proposal_labels", _I, [_P, _I, _I, _P, _P, _F, _U, _P]),
    ("art_render_proposal", _I, [_P, _I, _I, _P, _P, _F, _U, _P, _F, _F, _P, _P, _P]),
    ("art_render_depth", _I, [_P, _I, _I, _P, _P, _F, _U, _F, _P, _P, _P, _P]),
    ("art_render_sh", _I, [_P, _I, _I, _I, _P, _P, _F, _U, _P, _P, _P]),
    ("art_shading_param_count", _L, [_I]),
    ("art_shading_set_weights", _I, [_P, _I, _L, _P]),
    ("art_shading_forward", _I, [_P, _I, _I, _I, _I, _P, _P]),
    ("art_shading_forward_noalloc", _I, [_P, _I, _I, _I, _I, _P, _P]),
    ("art_vrt", _I, [_P, _I, _I, _P, _F, _U, _P, ctypes.POINTER(ctypes.c_double)]),
    ("art_query", _I, [_P, _I, _U, _L, _P, _P]),
    ("art_flut_adam", _I, [_P, _L, _P, _P, _P, _P, _I, _F, _F, _F, _F, _F]),
    ("art_proposal_param_count", _L, [_I]),
    ("art_proposal_set_weights", _I, [_P, _L, _P]),
    ("art_proposal_get_weights", _I, [_P, _L, _P]),
    ("art_proposal_init", _I, [_P, ctypes.c_uint64]),
    ("art_proposal_gather", _I, [_P, _L, _P, _P, _P, _P, _P]),
    ("art_proposal_set_loss", _I, [_P, _I, _F, _F]),
    ("art_proposal_calibrate", _I, [_P, _L, _P, _P, _P, _F, _F, ctypes.POINTER(_F)]),
    ("art_proposal_io", _I, [_P, _I, ctypes.c_char_p]),
    ("art_map_loss", _I, [_P, _L, _L, _P, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    ("art_proposal_forward", _I, [_P, _L, _P, _P, _P]),
    ("art_proposal_grad", _I, [_P, _L, _P, _P, _P, _P, _P]),
    ("art_proposal_train", _I, [_P, _L, _P, _P, _P, _L, _I, _F, _F, _F, _F, _P]),
    ("art_get_bones", _I, [_P, _P]),
    ("art_get_posed_keys", _I, [_P, _I, _U, _P]),
    ("art_get_octree", _I, [_P, _I, _U, _P, _P, _P, _P, _P, _P]),
    ("art_get_hits", _I, [_P, _I, _I, _I, _I, _P, _P, _F, _U, _I, _P, _P, _P]),
    ("art_get_stats", _I, [_P, _P]),
    ("art_render_status", _I, [_P, _P, _P]),
    ("art_get_timing", _I, [_P, _P, _P]),
]

_lib = None


def load() -> ctypes.CDLL:
    """Load libartemis.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_05628_amd.build` "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ArtemisError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
