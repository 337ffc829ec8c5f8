"""rocRAND's Philox4x32-10 engine as an external reference for raw words."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "philox_ref.cpp")
_LIB = os.path.join(_HERE, "libphilox_ref.so")


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["hipcc", "-O1", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def philox4x32_10(seed: int, ctr) -> np.ndarray:
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _lib.ref_philox4x32_10.argtypes = [ctypes.c_ulonglong,
                                           ctypes.POINTER(ctypes.c_uint32),
                                           ctypes.POINTER(ctypes.c_uint32)]
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    _lib.ref_philox4x32_10(seed, c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out
