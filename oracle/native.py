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
    intrinsics; OpenMP only to run several images at once in the batch
    call)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
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
        p = ctypes.c_void_p
        lib.ldp_oracle_extract_batch.argtypes = [p, p, p, p, p, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 p, p, p, ctypes.c_int32]
        lib.ldp_oracle_extract_batch.restype = ctypes.c_int
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


def default_threads():
    """Host threads for the batch call: OMP_NUM_THREADS if set, else the CPUs
    this process may run on, at most 16."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(16, len(os.sched_getaffinity(0))))


def ldp_extract_batch(buf, offsets, Hs, Ws, strides, k, cells_y, cells_x, magnitude=False,
                      threads=None):
    """Codes and histograms of every image of a packed batch (image j: Hs[j]
    rows of Ws[j] bytes, pitch strides[j], at byte offsets[j] of ``buf``).

    Returns (codes, code_offsets, hist): the code maps back to back (image j's
    at codes[code_offsets[j]:code_offsets[j+1]]) and hist of shape
    (n, cells_y, cells_x, 256).  Images run on ``threads`` host threads
    (default: default_threads())."""
    b = np.ascontiguousarray(buf, dtype=np.uint8).reshape(-1)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    H = np.ascontiguousarray(Hs, dtype=np.int32)
    W = np.ascontiguousarray(Ws, dtype=np.int32)
    st = np.ascontiguousarray(strides, dtype=np.int64)
    n = len(off)
    if not (len(H) == len(W) == len(st) == n):
        raise ValueError("size arrays differ in length")
    if n and np.any(off + (H.astype(np.int64) - 1) * st + W > b.size):
        raise ValueError("an image does not fit in the buffer")
    coff = np.zeros(n + 1, dtype=np.int64)
    coff[1:] = np.cumsum(np.maximum(H.astype(np.int64) - 2, 0) * np.maximum(W.astype(np.int64) - 2, 0))
    codes = np.empty(int(coff[-1]), dtype=np.uint8)
    hist = np.empty((n, cells_y, cells_x, 256), dtype=np.uint32)
    rc = _load().ldp_oracle_extract_batch(b.ctypes.data, off.ctypes.data, H.ctypes.data,
                                          W.ctypes.data, st.ctypes.data, n, k,
                                          1 if magnitude else 0, cells_y, cells_x,
                                          codes.ctypes.data, coff.ctypes.data, hist.ctypes.data,
                                          default_threads() if threads is None else int(threads))
    if rc != 0:
        raise ValueError("invalid arguments to ldp_oracle_extract_batch")
    return codes, coff, hist
