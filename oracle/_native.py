"""Build and load the oracle's C helper (test infrastructure only).

``build()`` compiles ``line_min.c`` with gcc and OpenMP into ``_line_min.so``
next to it; ``lib()`` loads it, building first if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "line_min.c")
_SO = os.path.join(_HERE, "_line_min.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_SO)
        L.oracle_line_min.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_double]
        L.oracle_line_min.restype = None
        L.oracle_line_min_p.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_double, ctypes.c_double]
        L.oracle_line_min_p.restype = None
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib
