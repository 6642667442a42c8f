"""ctypes front end of ``bruteforce.c`` (test infrastructure only).

``build()`` compiles the C file with gcc and OpenMP into ``_bruteforce.so`` next
to it; ``fluence(eps, sigma, M, crop)`` returns the FP64 brute-force fluence of
Eq. 1-3 at the pixel centres of ``crop = (r0, r1, c0, c1)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bruteforce.c")
_LIB = os.path.join(_HERE, "_bruteforce.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.bf_fluence.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        lib.bf_fluence.restype = ctypes.c_int
        lib.bf_fluence_env.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                       ctypes.c_int, dp]
        lib.bf_fluence_env.restype = ctypes.c_int
        lib.bf_radiance.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double]
        lib.bf_radiance.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fluence(eps, sigma, M: int = 4096, crop=None, environment=None) -> np.ndarray:
    """Brute-force F at pixel centres of the crop (rows r0:r1, cols c0:c1);
    ``environment``: K radiance samples at world angles 2 pi k / K (nearest
    sample) lighting the grid from outside, or None."""
    lib = _load()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    S = eps.shape[0]
    r0, r1, c0, c1 = crop if crop is not None else (0, S, 0, S)
    out = np.zeros((r1 - r0, c1 - c0))
    env = (np.zeros(1) if environment is None
           else np.ascontiguousarray(environment, dtype=np.float64))
    K = 0 if environment is None else len(env)
    rc = lib.bf_fluence_env(S, _ptr(eps), _ptr(sigma), int(M), r0, r1, c0, c1, _ptr(env), K,
                            _ptr(out))
    if rc != 0:
        raise ValueError("bad brute-force arguments")
    return out


def radiance(eps, sigma, px, py, dx, dy) -> float:
    lib = _load()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    return lib.bf_radiance(eps.shape[0], _ptr(eps), _ptr(sigma), px, py, dx, dy)
