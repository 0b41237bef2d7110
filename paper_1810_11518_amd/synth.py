"""Seeded synthetic inputs shaped like the paper's workloads.

Input generation only: this module holds none of the LDP arithmetic, and both
the HIP path's tests and the CPU oracle's tests take their images from it.
The generator itself is ``csrc/synth.c`` (integer arithmetic and a
counter-based random stream, so every machine produces the same bytes and any
image of a batch can be regenerated alone).

The paper extracts features from CK+ face frames of 640x490 pixels, face crops
resized to 260x260 (Section 3.1).  The dataset is not available here; the
recipes below stand in for it with the same frame shape and with content that
has the edges, smooth regions and exact ties that real frames have.

Workloads (the benchmark and the parity tests use these names):

``single``   one 490x640 image of iid uniform bytes, k=3, 7x6 cells.
``batch``    4096 images of 490x640, blurred noise plus 8 rectangles, k=3, 7x6.
``uneven``   10,000 images with H and W each uniform in [48, 1024], blurred
             noise plus rectangles, k=3, 7x6.
``large``    64 images of 8192x8192, blurred noise, 5% salt-and-pepper and 32
             flat patches (exact ties), k in {2, 3, 4}, 16x16 cells.
``serve``    a Poisson request stream of single images with sides
             log-uniform in [64, 2048], k=3, 7x6.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "synth.c")
_LIB = os.path.join(_HERE, "libldp_synth.so")
_lib = None

KIND_UNIFORM = 0
KIND_BLUR_RECTS = 1
KIND_BLUR_SP_FLAT = 2

# Base seeds per workload (arbitrary fixed constants).
SEEDS = {"single": 18101151800, "batch": 18101151801, "uneven": 18101151802,
         "large": 18101151803, "serve": 18101151804}

WORKLOADS = {
    "single": dict(n=1, H=490, W=640, kind=KIND_UNIFORM, k=3, cells=(7, 6)),
    "batch": dict(n=4096, H=490, W=640, kind=KIND_BLUR_RECTS, k=3, cells=(7, 6)),
    "uneven": dict(n=10000, side=(48, 1024), kind=KIND_BLUR_RECTS, k=3, cells=(7, 6)),
    "large": dict(n=64, H=8192, W=8192, kind=KIND_BLUR_SP_FLAT, k=(2, 3, 4), cells=(16, 16)),
    "serve": dict(side=(64, 2048), kind=KIND_BLUR_RECTS, k=3, cells=(7, 6),
                  rates=(1000, 2000, 5000, 10000, 20000, 50000)),
}


def build(force=True):
    """Compile csrc/synth.c into libldp_synth.so (gcc -O2 -fopenmp)."""
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
        p = ctypes.c_void_p
        lib.synth_images.argtypes = [p, p, p, p, p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_images.restype = ctypes.c_int
        lib.synth_uniform_ints.argtypes = [p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_uint64]
        lib.synth_uniform_ints.restype = None
        lib.synth_u64.argtypes = [p, ctypes.c_int32, ctypes.c_uint64]
        lib.synth_u64.restype = None
        _lib = lib
    return _lib


def fill(buf, offsets, Hs, Ws, strides, kind, seed, first_index=0):
    """Write images into ``buf`` (a writable contiguous uint8 numpy array).

    Image j has Hs[j] rows, Ws[j] columns and row pitch strides[j] bytes, starts
    at byte offsets[j], and is image number first_index + j of the stream.
    """
    buf = np.asarray(buf)
    if buf.dtype != np.uint8 or not buf.flags["C_CONTIGUOUS"] or not buf.flags["WRITEABLE"]:
        raise ValueError("buf must be a writable contiguous uint8 array")
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    Hs = np.ascontiguousarray(Hs, dtype=np.int32)
    Ws = np.ascontiguousarray(Ws, dtype=np.int32)
    strides = np.ascontiguousarray(strides, dtype=np.int64)
    n = len(offsets)
    if not (len(Hs) == len(Ws) == len(strides) == n):
        raise ValueError("size arrays differ in length")
    if n and np.any(offsets + (Hs.astype(np.int64) - 1) * strides + Ws > buf.size):
        raise ValueError("an image does not fit in the buffer")
    rc = _load().synth_images(buf.ctypes.data, offsets.ctypes.data, Hs.ctypes.data,
                              Ws.ctypes.data, strides.ctypes.data, n, kind, seed, first_index)
    if rc != 0:
        raise ValueError("invalid image sizes or kind")
    return buf


def image(kind, seed, index, H, W, stride=None):
    """One image as a (H, W) uint8 array (a view with row pitch ``stride``)."""
    stride = W if stride is None else stride
    buf = np.zeros(H * stride, dtype=np.uint8)
    fill(buf, [0], [H], [W], [stride], kind, seed, index)
    return buf.reshape(H, stride)[:, :W]


def uniform_ints(n, lo, hi, seed):
    out = np.empty(n, dtype=np.int32)
    _load().synth_uniform_ints(out.ctypes.data, n, lo, hi, seed)
    return out


def uniform01(n, seed):
    """n doubles in [0, 1) from the top 53 bits of the stream."""
    raw = np.empty(n, dtype=np.uint64)
    _load().synth_u64(raw.ctypes.data, n, seed)
    return (raw >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def layout(Hs, Ws, row_align=1, image_align=256):
    """Pack images back to back: returns (offsets, strides, total_bytes).

    Rows have pitch W rounded up to ``row_align``; every image starts on an
    ``image_align`` boundary (as separate device allocations would).
    """
    Hs = np.asarray(Hs, dtype=np.int64)
    Ws = np.asarray(Ws, dtype=np.int64)
    strides = (Ws + row_align - 1) // row_align * row_align
    sizes = Hs * strides
    sizes_al = (sizes + image_align - 1) // image_align * image_align
    offsets = np.zeros(len(Hs), dtype=np.int64)
    if len(Hs) > 1:
        offsets[1:] = np.cumsum(sizes_al)[:-1]
    total = int(sizes_al.sum()) if len(Hs) else 0
    return offsets, strides, total


def workload_sizes(name, n=None):
    """(Hs, Ws) of a workload, optionally only its first n images."""
    w = WORKLOADS[name]
    count = w["n"] if n is None else n
    if "H" in w:
        return (np.full(count, w["H"], dtype=np.int32), np.full(count, w["W"], dtype=np.int32))
    lo, hi = w["side"]
    seed = SEEDS[name]
    Hs = uniform_ints(w["n"], lo, hi, seed * 2 + 0)[:count]
    Ws = uniform_ints(w["n"], lo, hi, seed * 2 + 1)[:count]
    return Hs, Ws


def workload_image(name, index):
    """Image ``index`` of a workload, regenerated alone."""
    Hs, Ws = workload_sizes(name, index + 1)
    w = WORKLOADS[name]
    return image(w["kind"], SEEDS[name], index, int(Hs[index]), int(Ws[index]))


def serve_stream(rate, n, seed=None):
    """Open-loop Poisson arrivals at ``rate`` images/s and log-uniform sides.

    Returns (arrival_s, Hs, Ws): arrival times in seconds from the start,
    increasing, and image sizes with sides round(exp(U(ln 64, ln 2048))).
    """
    seed = SEEDS["serve"] if seed is None else seed
    u = uniform01(3 * n, seed + int(rate))
    gaps = -np.log1p(-u[:n]) / float(rate)
    arrival = np.cumsum(gaps)
    lo, hi = WORKLOADS["serve"]["side"]
    a, b = math.log(lo), math.log(hi)
    Hs = np.rint(np.exp(a + (b - a) * u[n:2 * n])).astype(np.int32)
    Ws = np.rint(np.exp(a + (b - a) * u[2 * n:])).astype(np.int32)
    return arrival, Hs, Ws
