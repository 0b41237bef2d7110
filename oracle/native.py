"""ctypes access to the plain C oracle (ldp_oracle.c).

TEST INFRASTRUCTURE ONLY: the product path never imports this module.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_ldp.so")
_lib = None


def build(force=True):
    """Compile ldp_oracle.c into liboracle_ldp.so with gcc -O2 (no SIMD
    intrinsics, no threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.ldp_oracle_codes.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
        lib.ldp_oracle_codes.restype = ctypes.c_int
        lib.ldp_oracle_codes_ex.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_void_p]
        lib.ldp_oracle_codes_ex.restype = ctypes.c_int
        lib.ldp_oracle_histograms.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
        lib.ldp_oracle_histograms.restype = ctypes.c_int
        _lib = lib
    return _lib


def ldp_codes(img, k=3, magnitude=False):
    """Interior code map of a 2-D uint8 image (rows may be strided); with
    ``magnitude`` the responses are ranked by absolute value."""
    a = np.asarray(img)
    if a.ndim != 2 or a.dtype != np.uint8:
        raise ValueError("image must be a 2-D uint8 array")
    if a.strides[1] != 1:
        a = np.ascontiguousarray(a)
    H, W = a.shape
    out = np.empty((max(H - 2, 0), max(W - 2, 0)), dtype=np.uint8)
    rc = _load().ldp_oracle_codes_ex(a.ctypes.data, H, W, a.strides[0], k, 1 if magnitude else 0,
                                     out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid arguments to ldp_oracle_codes")
    return out


def ldp_histograms(codes, cells_y, cells_x):
    """Per-cell 256-bin histograms, uint32 array (cells_y, cells_x, 256)."""
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    if c.ndim != 2:
        raise ValueError("codes must be 2-D")
    hist = np.empty((cells_y, cells_x, 256), dtype=np.uint32)
    rc = _load().ldp_oracle_histograms(c.ctypes.data, c.shape[0] + 2, c.shape[1] + 2,
                                       cells_y, cells_x, hist.ctypes.data)
    if rc != 0:
        raise ValueError("invalid arguments to ldp_oracle_histograms")
    return hist


def ldp_extract(img, k, cells_y, cells_x, magnitude=False):
    codes = ldp_codes(img, k, magnitude)
    return codes, ldp_histograms(codes, cells_y, cells_x)
