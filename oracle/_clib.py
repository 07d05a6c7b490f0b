"""Loader for the oracle's plain-C loops (oracle/o1.c, oracle/mapped.c); test infrastructure only.

The shared object is built with gcc next to the source on first use (or by the repository's
build step) and rebuilt when the source is newer.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "o1.c"), os.path.join(_HERE, "mapped.c")]
_LIB = os.path.join(_HERE, "libo1.so")
_lib = None


def build(force=False):
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp] + _SRCS + ["-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        vp = ctypes.c_void_p  # the Gauss order array and its tables (NULL for the 2x2x2 rule)
        _lib.o1_entries.argtypes = [ctypes.c_int64, i64p, i64p, i64p, i64p, f64p, f64p, f64p, vp, vp, vp, f64p]
        _lib.o1_entries.restype = ctypes.c_int
        _lib.o1_apply.argtypes = [ctypes.c_int64, i64p, i64p, f64p, f64p, f64p, vp, vp, vp, f64p, ctypes.c_int64,
                                  i64p, f64p]
        _lib.o1_apply.restype = ctypes.c_int
        _lib.o1_gauss_rule.argtypes = [f64p, ctypes.c_double, ctypes.c_int, f64p, ctypes.c_double, ctypes.c_int, f64p,
                                       f64p]
        _lib.o1_gauss_rule.restype = ctypes.c_double
        _lib.o1_point_potential.argtypes = [ctypes.c_int64, f64p, ctypes.c_int64, f64p, f64p, f64p]
        _lib.o1_point_potential.restype = None
        i32 = ctypes.c_int
        _lib.om_map.argtypes = [i32, ctypes.c_int64, f64p, f64p, f64p]
        _lib.om_map.restype = None
        _lib.om_touch_entries.argtypes = [i32, ctypes.c_int64, f64p, f64p, f64p, f64p, i32, i32, i32, i32, i32, f64p,
                                          f64p, f64p]
        _lib.om_touch_entries.restype = None
        _lib.om_regular_entries.argtypes = [i32, ctypes.c_int64, f64p, f64p, f64p, f64p, i32, f64p, f64p, f64p]
        _lib.om_regular_entries.restype = None
    return _lib
