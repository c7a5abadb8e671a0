"""Build and load the oracle's C routines (``oracle.c``) with gcc.

Test infrastructure only: the GPU library never loads this.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            i64 = ctypes.c_int64
            u32 = ctypes.c_uint32
            L.orc_polymul.argtypes = [u32p, i64, u32p, i64, u32, u32p]
            L.orc_polymul.restype = None
            L.orc_polymul_sample.argtypes = [u32p, i64, u32p, i64, u32, i64p, i64, u32p]
            L.orc_polymul_sample.restype = None
            L.orc_cyclic.argtypes = [u32p, u32p, i64, u32, u32p]
            L.orc_cyclic.restype = None
            L.orc_negacyclic.argtypes = [u32p, u32p, i64, u32, u32p]
            L.orc_negacyclic.restype = None
            L.orc_eval.argtypes = [u32p, i64, u32, u32]
            L.orc_eval.restype = u32
            L.orc_ntt.argtypes = [u32p, i64, u32, u32, ctypes.c_int]
            L.orc_ntt.restype = ctypes.c_int
            L.orc_polymul_ntt.argtypes = [u32p, i64, u32p, i64, u32, u32, u32p]
            L.orc_polymul_ntt.restype = ctypes.c_int
            _lib = L
    return _lib
