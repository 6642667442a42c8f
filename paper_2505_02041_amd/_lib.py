"""ctypes declarations of the C ABI in ``include/hrc.h`` (argument marshalling only).

Loading never falls back to anything: if ``libhrc.so`` is missing the import of
the library raises, and every computation runs in its HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhrc.so")

HRC_OK = 0
HRC_ERR_INVALID_ARG = -1
HRC_ERR_SHAPE = -2
HRC_ERR_WORKSPACE = -3
HRC_ERR_HIP = -4
HRC_ERR_UNSUPPORTED = -5
HRC_ERR_INPUT = -6
HRC_ERR_TIMEOUT = -7
HRC_ERR_TOO_LARGE = -8
HRC_MIN_LOG2 = 3
HRC_MAX_LOG2 = 12
HRC_FLAG_VALIDATE = 0x1
HRC_FLAG_BLUR = 0x2
HRC_FLAG_HALF_INTERVALS = 0x4
HRC_FLAG_KEEP_PYRAMID = 0x8
HRC_FLAG_REUSE_PYRAMID = 0x40
HRC_FLAG_QUADRANTS_1 = 0x10
HRC_FLAG_QUADRANTS_2 = 0x20
HRC_FLAG_QUADRANTS_4 = 0x30
HRC_FLAG_QUADRANTS_MASK = 0x30
HRC_FLAG_BATCH_FULL = 0x100
HRC_FLAG_BATCH_DENSE = 0x200
HRC_FLAG_BATCH_PERSISTENT = 0x400
PASS_NAMES = ["seed", "merge_up", "merge_down", "tail", "gather_adj",
              "merge_down_adj", "interval_adj", "seed_adj", "blur", "blur_adj",
              "seed_rgb", "merge_up_rgb", "merge_down_rgb", "tail_rgb",
              "merge_down_adj_rgb", "interval_adj_rgb", "seed_adj_rgb"]
# Kernel symbol of each pass kind (what a profiler shows).
PASS_KERNELS = ["hrc_seed", "hrc_merge_up", "hrc_merge_down", "hrc_tail",
                "hrc_gather_adj", "hrc_merge_down_adj", "hrc_interval_adj", "hrc_seed_adj",
                "hrc_blur", "hrc_blur_adj", "hrc_seed_rgb", "hrc_merge_up_rgb",
                "hrc_merge_down_rgb", "hrc_tail_rgb", "hrc_merge_down_adj_rgb",
                "hrc_interval_adj_rgb", "hrc_seed_adj_rgb"]

# Every function the header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


class hrc_scene(ctypes.Structure):
    _fields_ = [
        ("log2_size", ctypes.c_int),
        ("emission", _vp),
        ("sigma_t", _vp),
        ("fluence", _vp),
        ("grad_fluence", _vp),
        ("grad_emission", _vp),
        ("grad_sigma_t", _vp),
    ]


SIGNATURES = {
    "hrc_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "hrc_destroy": (None, [_vp]),
    "hrc_set_environment": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "hrc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "hrc_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint,
                                           ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "hrc_forward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp,
                                   ctypes.c_uint]),
    "hrc_forward_static": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                                          ctypes.c_uint]),
    "hrc_backward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                    _vp, ctypes.c_uint]),
    "hrc_workspace_bytes_rgb": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint,
                                               ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
    "hrc_forward_rgb": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp,
                                       ctypes.c_uint]),
    "hrc_backward_rgb": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                        _vp, ctypes.c_uint]),
    "hrc_multibounce_workspace_bytes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                                       ctypes.POINTER(_sz),
                                                       ctypes.POINTER(_sz)]),
    "hrc_multibounce_forward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_int,
                                               _vp, _vp, _sz, _vp, ctypes.c_uint]),
    "hrc_multibounce_backward": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, ctypes.c_int,
                                                _vp, _vp, _vp, _vp, _vp, _sz, _vp,
                                                ctypes.c_uint]),
    "hrc_profile_solve": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _sz, _vp, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]),
    "hrc_batch_plan": (ctypes.c_int, [_vp, ctypes.POINTER(hrc_scene), ctypes.c_int,
                                      ctypes.c_uint, _vp, ctypes.POINTER(_vp)]),
    "hrc_batch_launch": (ctypes.c_int, [_vp, _vp]),
    "hrc_batch_workspace_bytes": (_sz, [_vp]),
    "hrc_batch_describe": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int)]),
    "hrc_batch_status": (ctypes.c_int, [_vp, _vp]),
    "hrc_batch_debug_waits": (ctypes.c_int, [_vp, ctypes.c_uint]),
    "hrc_batch_queues": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int)]),
    "hrc_batch_candidates": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_float)]),
    "hrc_batch_destroy": (None, [_vp]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load ``libhrc.so`` (built in-tree by ``paper_2505_02041_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2505_02041_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class HRCError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().hrc_status_string(status).decode()
        super().__init__(f"{where}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != HRC_OK:
        raise HRCError(status, where)
