"""ctypes wrapper and build step for the plain C oracle (oracle/lu_blk.c).

TEST INFRASTRUCTURE ONLY.  Built with gcc (no GPU toolchain); see build().
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lu_blk.c")
_LIB = os.path.join(_HERE, "liblu_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile lu_blk.c into liblu_oracle.so with gcc -O2 -fopenmp."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_dgetrf_rl.restype = ctypes.c_int
        lib.oracle_dgetrf_rl.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def dgetrf_rl(A: np.ndarray, nb: int = 64):
    """Factor a C-ordered float64 matrix in place; returns (ipiv 1-based int32, info)."""
    if A.dtype != np.float64 or not A.flags.c_contiguous:
        raise ValueError("A must be a C-contiguous float64 array")
    m, n = A.shape
    ipiv = np.zeros(min(m, n), dtype=np.int32)
    info = _load().oracle_dgetrf_rl(m, n, A.ctypes.data, n, nb, ipiv.ctypes.data)
    return ipiv, int(info)
