"""Exact direct kernel sum s_m = sum_n w_n F(||x_n - y_m||) (problem statement, Sec. 1 / Sec. 3).

FP64, computed by the plain loops of oracle/csrc/direct_sum.c (OpenMP over
targets).  The shared object is built next to the source by ``build_clib`` (also
called by the package build step); it is part of the oracle, i.e. test
infrastructure only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "direct_sum.c")
_LIB = os.path.join(_HERE, "csrc", "liboracle_direct.so")
_KERNEL_ID = {"gaussian": 1, "laplacian": 2, "negdist": 3, "matern": 4}
_lib = None


def build_clib(force: bool = False) -> str:
    """Compile the oracle's C loops with gcc (FP64, -O2 without fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_clib()
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_direct_sum_f64", "oracle_direct_sum_f32"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                           ctypes.c_void_p]
        _lib = lib
    return _lib


def direct_sum(kernel: str, x, y, w, sigma: float = 1.0) -> np.ndarray:
    """s_m for every row of y (pass a subset of targets to bound the O(MN d) cost)."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    w = np.ascontiguousarray(w)
    if x.dtype == np.float32 and y.dtype == np.float32 and w.dtype == np.float32:
        fn = _load().oracle_direct_sum_f32
    else:
        x = x.astype(np.float64)
        y = y.astype(np.float64)
        w = w.astype(np.float64)
        fn = _load().oracle_direct_sum_f64
    N, d = x.shape
    M = y.shape[0]
    s = np.empty(M, dtype=np.float64)
    fn(x.ctypes.data, N, y.ctypes.data, M, d, w.ctypes.data, _KERNEL_ID[kernel], float(sigma),
       s.ctypes.data)
    return s
