"""Thin ctypes binding of libldp.so (include/ldp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libldp.so.  Tensors are torch CUDA (ROCm) tensors; torch supplies
device memory and the current stream.  If the library is not built this
module raises -- there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldp.so")

LDP_OK = 0
LDP_ERR_INVALID_ARG = -1
LDP_ERR_HIP = -2
LDP_ERR_NO_MEMORY = -3
LDP_ERR_UNSUPPORTED = -4
LDP_ERR_BUSY = -5

# flags of the _ex calls (at most one)
LDP_RANK_MAGNITUDE = 1
LDP_DIRECT_MASKS = 2
LDP_CODE_LBP = 4

# every symbol include/ldp.h declares
EXPORTED = [
    "ldp_status_string", "ldp_version", "ldp_codes", "ldp_histograms", "ldp_extract",
    "ldp_codes_ex", "ldp_extract_ex", "ldp_compact_bins", "ldp_compact_histograms",
    "ldp_window_grid", "ldp_histograms_windows", "ldp_extract_windows",
    "ldp_batch_plan_create", "ldp_batch_plan_create_ex", "ldp_batch_plan_create_windows",
    "ldp_batch_plan_set", "ldp_batch_run", "ldp_batch_launch", "ldp_batch_run_per_image",
    "ldp_batch_plan_info", "ldp_batch_plan_layout", "ldp_batch_plan_destroy",
    "ldp_now", "ldp_server_create", "ldp_server_submit", "ldp_server_poll",
    "ldp_server_stats_get", "ldp_server_destroy", "ldp_stream_copy", "ldp_batch_launch_noalloc",
]


class LdpError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, status_string(status), status))


class ImageDesc(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("codes", ctypes.c_void_p), ("hist", ctypes.c_void_p),
                ("stride", ctypes.c_int64), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


MAX_SIZE_CLASSES = 4


class SizeClass(ctypes.Structure):
    _fields_ = [("max_pixels", ctypes.c_int64), ("cell_rows_per_item", ctypes.c_int32),
                ("rows_per_task", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("classes", SizeClass * MAX_SIZE_CLASSES)]


def make_tune(tune):
    """ldp_tune from a dict {block_threads, grid_blocks, classes: [{max_pixels,
    cell_rows_per_item, rows_per_task}, ...]} (missing fields take defaults)."""
    t = Tune()
    t.block_threads = int(tune.get("block_threads", 0))
    t.grid_blocks = int(tune.get("grid_blocks", 0))
    classes = tune.get("classes", [])
    if len(classes) > MAX_SIZE_CLASSES:
        raise ValueError("at most %d size classes" % MAX_SIZE_CLASSES)
    t.n_classes = len(classes)
    for i, c in enumerate(classes):
        t.classes[i].max_pixels = int(c.get("max_pixels", 2 ** 62))
        t.classes[i].cell_rows_per_item = int(c.get("cell_rows_per_item", 0))
        t.classes[i].rows_per_task = int(c.get("rows_per_task", 0))
    return t


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("depth", ctypes.c_int32), ("k", ctypes.c_int32),
                ("cells_y", ctypes.c_int32), ("cells_x", ctypes.c_int32),
                ("dry_run", ctypes.c_int32), ("dry_run_us", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


LDP_SERVER_NO_MIRROR = 1


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int32),
                ("batch_size", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("memory_waits", ctypes.c_int64), ("peak_pool_bytes", ctypes.c_int64), ("peak_inflight", ctypes.c_int32),
                ("peak_batches", ctypes.c_int32), ("max_batch_seen", ctypes.c_int32),
                ("waiting", ctypes.c_int32)]


_lib = None


def load():
    """Load libldp.so (raises if it has not been built).

    torch is imported first: a PyTorch ROCm build can carry its own HIP
    runtime library, and libldp.so must bind to that one (the library's HIP
    dependency resolves to the runtime already in the process).  Loaded
    before torch, the library would bring in a second HIP runtime, whose
    context does not know torch's device memory."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libldp.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_1810_11518_amd.build" % LIB_PATH)
    import torch  # noqa: F401  (see above)
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "ldp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "ldp_version": (ctypes.c_int, []),
        "ldp_codes": (ctypes.c_int, [p, i32, i32, i64, i32, p, p]),
        "ldp_histograms": (ctypes.c_int, [p, i32, i32, i32, i32, p, p]),
        "ldp_extract": (ctypes.c_int, [p, i32, i32, i64, i32, i32, i32, p, p, p]),
        "ldp_codes_ex": (ctypes.c_int, [p, i32, i32, i64, i32, i32, p, p]),
        "ldp_extract_ex": (ctypes.c_int, [p, i32, i32, i64, i32, i32, i32, i32, p, p, p]),
        "ldp_compact_bins": (i32, [i32]),
        "ldp_compact_histograms": (ctypes.c_int, [p, i64, i32, p, p]),
        "ldp_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(p), i32, i64, i32, i32, i32,
                                                 ctypes.POINTER(Tune)]),
        "ldp_batch_plan_create_ex": (ctypes.c_int, [ctypes.POINTER(p), i32, i64, i32, i32, i32,
                                                    i32, ctypes.POINTER(Tune)]),
        "ldp_batch_plan_create_windows": (ctypes.c_int, [ctypes.POINTER(p), i32, i64, i32, i32,
                                                         i32, i32, i32, ctypes.POINTER(Tune)]),
        "ldp_window_grid": (ctypes.c_int, [i32, i32, i32, i32, ctypes.POINTER(i32),
                                           ctypes.POINTER(i32)]),
        "ldp_histograms_windows": (ctypes.c_int, [p, i32, i32, i32, i32, p, p]),
        "ldp_extract_windows": (ctypes.c_int, [p, i32, i32, i64, i32, i32, i32, i32, p, p, p]),
        "ldp_batch_plan_set": (ctypes.c_int, [p, ctypes.POINTER(ImageDesc), i32, p]),
        "ldp_batch_run": (ctypes.c_int, [p, p]),
        "ldp_batch_launch": (ctypes.c_int, [p, ctypes.POINTER(ImageDesc), i32, p]),
        "ldp_batch_run_per_image": (ctypes.c_int, [p, p]),
        "ldp_batch_plan_info": (ctypes.c_int, [p, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "ldp_batch_plan_layout": (ctypes.c_int, [p, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                                 ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "ldp_batch_plan_destroy": (ctypes.c_int, [p]),
        "ldp_now": (ctypes.c_double, []),
        "ldp_server_create": (ctypes.c_int, [ctypes.POINTER(p), ctypes.POINTER(ServerConfig)]),
        "ldp_server_submit": (ctypes.c_int, [p, p, i32, i32, i64, p, p, ctypes.POINTER(i64)]),
        "ldp_server_poll": (ctypes.c_int, [p, ctypes.POINTER(Completion), i32,
                                           ctypes.POINTER(i32), i32]),
        "ldp_server_stats_get": (ctypes.c_int, [p, ctypes.POINTER(ServerStats)]),
        "ldp_server_destroy": (ctypes.c_int, [p]),
        "ldp_stream_copy": (ctypes.c_int, [p, p, i64, p]),
        "ldp_batch_launch_noalloc": (ctypes.c_int, [ctypes.POINTER(ImageDesc), i32, i32, i32, i32,
                                                    p]),
    }
    for name, (res, args) in sig.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(status):
    try:
        return load().ldp_status_string(status).decode()
    except RuntimeError:
        return "status %d" % status


def _check(status, what):
    if status != LDP_OK:
        raise LdpError(status, what)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _image_args(img):
    import torch
    if not isinstance(img, torch.Tensor) or img.dtype != torch.uint8 or img.dim() != 2:
        raise ValueError("image must be a 2-D torch.uint8 tensor")
    if not img.is_cuda:
        raise ValueError("image must be a device tensor")
    if img.stride(1) != 1:
        raise ValueError("image columns must be contiguous (stride(1) == 1)")
    H, W = img.shape
    return img.data_ptr(), int(H), int(W), int(img.stride(0))


def codes(img, k=3, out=None, stream=None, flags=0):
    """LDP codes of every interior pixel: uint8 tensor (H-2, W-2).  ``flags``:
    LDP_RANK_MAGNITUDE ranks |m_i|."""
    import torch
    ptr, H, W, stride = _image_args(img)
    if out is None:
        out = torch.empty((max(H - 2, 0), max(W - 2, 0)), dtype=torch.uint8, device=img.device)
    _check(load().ldp_codes_ex(ptr, H, W, stride, k, flags, out.data_ptr(), _stream(stream)),
           "ldp_codes_ex")
    return out


def histograms(code_map, cells_y, cells_x, out=None, stream=None):
    """Per-cell 256-bin histograms of a dense code map: int32 tensor
    (cells_y, cells_x, 256) holding the uint32 counts."""
    import torch
    if code_map.dtype != torch.uint8 or code_map.dim() != 2 or not code_map.is_contiguous():
        raise ValueError("code map must be a contiguous 2-D torch.uint8 tensor")
    Hc, Wc = code_map.shape
    if out is None:
        out = torch.empty((cells_y, cells_x, 256), dtype=torch.int32, device=code_map.device)
    _check(load().ldp_histograms(code_map.data_ptr(), Hc + 2, Wc + 2, cells_y, cells_x,
                                 out.data_ptr(), _stream(stream)), "ldp_histograms")
    return out


def extract(img, k, cells_y, cells_x, want_codes=True, codes_out=None, hist_out=None,
            stream=None, flags=0):
    """Codes and per-cell histograms in one launch: (codes or None, hist)."""
    import torch
    ptr, H, W, stride = _image_args(img)
    if want_codes and codes_out is None:
        codes_out = torch.empty((H - 2, W - 2), dtype=torch.uint8, device=img.device)
    if hist_out is None:
        hist_out = torch.empty((cells_y, cells_x, 256), dtype=torch.int32, device=img.device)
    cptr = codes_out.data_ptr() if want_codes else None
    _check(load().ldp_extract_ex(ptr, H, W, stride, k, flags, cells_y, cells_x, cptr,
                                 hist_out.data_ptr(), _stream(stream)), "ldp_extract_ex")
    return (codes_out if want_codes else None), hist_out


def window_grid(H, W, win_y, win_x):
    """(ny, nx): windows over the (H-2) x (W-2) code map."""
    ny, nx = ctypes.c_int32(), ctypes.c_int32()
    _check(load().ldp_window_grid(H, W, win_y, win_x, ctypes.byref(ny), ctypes.byref(nx)),
           "ldp_window_grid")
    return int(ny.value), int(nx.value)


def extract_windows(img, k, win_y, win_x, want_codes=True, codes_out=None, hist_out=None,
                    stream=None, flags=0):
    """Codes and per-window histograms: (codes or None, hist (ny, nx, 256))."""
    import torch
    ptr, H, W, stride = _image_args(img)
    ny, nx = window_grid(H, W, win_y, win_x)
    if want_codes and codes_out is None:
        codes_out = torch.empty((H - 2, W - 2), dtype=torch.uint8, device=img.device)
    if hist_out is None:
        hist_out = torch.empty((ny, nx, 256), dtype=torch.int32, device=img.device)
    cptr = codes_out.data_ptr() if want_codes else None
    _check(load().ldp_extract_windows(ptr, H, W, stride, k, flags, win_y, win_x, cptr,
                                      hist_out.data_ptr(), _stream(stream)),
           "ldp_extract_windows")
    return (codes_out if want_codes else None), hist_out


def histograms_windows(code_map, win_y, win_x, out=None, stream=None):
    """Per-window histograms of a dense code map: int32 (ny, nx, 256)."""
    import torch
    if code_map.dtype != torch.uint8 or code_map.dim() != 2 or not code_map.is_contiguous():
        raise ValueError("code map must be a contiguous 2-D torch.uint8 tensor")
    Hc, Wc = code_map.shape
    ny, nx = window_grid(Hc + 2, Wc + 2, win_y, win_x)
    if out is None:
        out = torch.empty((ny, nx, 256), dtype=torch.int32, device=code_map.device)
    _check(load().ldp_histograms_windows(code_map.data_ptr(), Hc + 2, Wc + 2, win_y, win_x,
                                         out.data_ptr(), _stream(stream)),
           "ldp_histograms_windows")
    return out


def compact_bins(k):
    """C(8, k) + 1: bins of Eq. 6's compact vector plus the tie bin."""
    n = load().ldp_compact_bins(k)
    if n < 0:
        raise LdpError(n, "ldp_compact_bins")
    return int(n)


def compact_histograms(hist, k, out=None, stream=None):
    """Compact vectors of raw-code histograms (last axis 256, contiguous
    int32/uint32 device tensor): same leading shape, last axis
    compact_bins(k)."""
    import torch
    if hist.dtype != torch.int32 or hist.shape[-1] != 256 or not hist.is_contiguous():
        raise ValueError("histograms must be a contiguous int32 tensor with 256 bins last")
    n_cells = hist.numel() // 256
    nb = compact_bins(k)
    if out is None:
        out = torch.empty(tuple(hist.shape[:-1]) + (nb,), dtype=torch.int32, device=hist.device)
    _check(load().ldp_compact_histograms(hist.data_ptr(), n_cells, k, out.data_ptr(),
                                         _stream(stream)), "ldp_compact_histograms")
    return out


def batch_launch_noalloc(descs, k, cells_y, cells_x, stream=None):
    """ldp_batch_launch_noalloc: a small batch (ctypes ImageDesc array, see
    BatchPlan.descs) with no plan and no allocation."""
    _check(load().ldp_batch_launch_noalloc(descs, len(descs), k, cells_y, cells_x,
                                           _stream(stream)), "ldp_batch_launch_noalloc")


def stream_copy(src, dst, stream=None):
    """Copy device tensor ``src`` into ``dst`` (same byte size, 16-byte
    aligned) with the library's streaming copy kernel (ldp_stream_copy)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst differ in size")
    _check(load().ldp_stream_copy(src.data_ptr(), dst.data_ptr(), nb, _stream(stream)),
           "ldp_stream_copy")
    return dst


class BatchPlan:
    """A persistent, graph-captured launch over many images (ldp_batch_*)."""

    def __init__(self, max_images, max_pixels, k, cells_y, cells_x, tune=None, flags=0,
                 windows=False, max_width=None):
        """cells_y x cells_x cells, or with ``windows`` windows of cells_y x
        cells_x code pixels over images at most ``max_width`` wide."""
        self._lib = load()
        self._plan = ctypes.c_void_p()
        t = make_tune(tune) if tune is not None else None
        tp = ctypes.byref(t) if t is not None else None
        if windows:
            _check(self._lib.ldp_batch_plan_create_windows(ctypes.byref(self._plan), max_images,
                                                           max_pixels, max_width, k, flags,
                                                           cells_y, cells_x, tp),
                   "ldp_batch_plan_create_windows")
        else:
            _check(self._lib.ldp_batch_plan_create_ex(ctypes.byref(self._plan), max_images,
                                                      max_pixels, k, flags, cells_y, cells_x, tp),
                   "ldp_batch_plan_create_ex")
        self.k, self.cells, self.flags, self.windows = k, (cells_y, cells_x), flags, windows

    @staticmethod
    def descs(imgs, codes, hists, strides=None, Hs=None, Ws=None):
        """Descriptor array from lists of pointers (ints) and sizes."""
        n = len(imgs)
        arr = (ImageDesc * n)()
        for j in range(n):
            arr[j].img = imgs[j]
            arr[j].codes = codes[j] if codes is not None else None
            arr[j].hist = hists[j]
            arr[j].stride = strides[j]
            arr[j].H = Hs[j]
            arr[j].W = Ws[j]
        return arr

    def set(self, descs, stream=None):
        _check(self._lib.ldp_batch_plan_set(self._plan, descs, len(descs), _stream(stream)),
               "ldp_batch_plan_set")

    def run(self, stream=None):
        _check(self._lib.ldp_batch_run(self._plan, _stream(stream)), "ldp_batch_run")

    def launch(self, descs, stream=None):
        """Load and run `descs` in one call (ldp_batch_launch): small batches
        travel in the launch's arguments and leave the loaded batch as it was."""
        _check(self._lib.ldp_batch_launch(self._plan, descs, len(descs), _stream(stream)),
               "ldp_batch_launch")

    def run_per_image(self, stream=None):
        _check(self._lib.ldp_batch_run_per_image(self._plan, _stream(stream)),
               "ldp_batch_run_per_image")

    def info(self):
        items, grid = ctypes.c_int64(), ctypes.c_int32()
        _check(self._lib.ldp_batch_plan_info(self._plan, ctypes.byref(items), ctypes.byref(grid)),
               "ldp_batch_plan_info")
        return int(items.value), int(grid.value)

    def layout(self):
        """(threads per workgroup, LDS bytes per workgroup, histogram copies,
        non-temporal stores as 0 or 1)."""
        th, lds, cp, nt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.ldp_batch_plan_layout(self._plan, ctypes.byref(th), ctypes.byref(lds),
                                               ctypes.byref(cp), ctypes.byref(nt)),
               "ldp_batch_plan_layout")
        return int(th.value), int(lds.value), int(cp.value), int(nt.value)

    def close(self):
        if self._plan:
            self._lib.ldp_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now():
    """The server clock (seconds, monotonic)."""
    return load().ldp_now()


class Server:
    """Continuous-batching request server (ldp_server_*).

    submit() takes HOST numpy buffers; they are kept alive here until the
    request completes.  Page-locked ones (e.g. views of torch.empty(...,
    pin_memory=True)) are read and written by the kernel in place; pageable
    ones go through the server's page-locked mirror of its memory pool
    (copied in before the batch's launch and out once it has run).  While
    requests keep arriving the dispatcher thread polls rather than sleeps
    (up to 200 us after its last piece of work): a busy server keeps one
    host core busy.
    """

    def __init__(self, pool_bytes, max_inflight, max_batch, depth, k, cells_y, cells_x,
                 dry_run=False, dry_run_us=0, no_mirror=False):
        self._lib = load()
        self._srv = ctypes.c_void_p()
        cfg = ServerConfig(int(pool_bytes), int(max_inflight), int(max_batch), int(depth), int(k),
                           int(cells_y), int(cells_x), 1 if dry_run else 0, int(dry_run_us),
                           LDP_SERVER_NO_MIRROR if no_mirror else 0)
        _check(self._lib.ldp_server_create(ctypes.byref(self._srv), ctypes.byref(cfg)),
               "ldp_server_create")
        self.cells = (cells_y, cells_x)
        self._live = {}

    def submit(self, img, hist_out, codes_out=None):
        a = img
        if a.ndim != 2 or a.dtype != np.uint8 or a.strides[1] != 1:
            raise ValueError("image must be a 2-D uint8 array with contiguous columns")
        if hist_out.dtype not in (np.uint32, np.int32) or not hist_out.flags["C_CONTIGUOUS"]:
            raise ValueError("hist_out must be a contiguous 32-bit array")
        if hist_out.size != self.cells[0] * self.cells[1] * 256:
            raise ValueError("hist_out has the wrong size")
        H, W = a.shape
        if codes_out is not None and (codes_out.dtype != np.uint8 or codes_out.size != (H - 2) * (W - 2)
                                      or not codes_out.flags["C_CONTIGUOUS"]):
            raise ValueError("codes_out must be a contiguous uint8 array of (H-2)*(W-2)")
        rid = ctypes.c_int64()
        _check(self._lib.ldp_server_submit(self._srv, a.ctypes.data, H, W, a.strides[0],
                                           codes_out.ctypes.data if codes_out is not None else None,
                                           hist_out.ctypes.data, ctypes.byref(rid)),
               "ldp_server_submit")
        self._live[rid.value] = (img, hist_out, codes_out)
        return rid.value

    def poll(self, max_n=4096, wait_us=0):
        buf = (Completion * max_n)()
        n = ctypes.c_int32()
        _check(self._lib.ldp_server_poll(self._srv, buf, max_n, ctypes.byref(n), int(wait_us)),
               "ldp_server_poll")
        out = []
        for i in range(n.value):
            c = buf[i]
            self._live.pop(c.id, None)
            out.append(dict(id=c.id, t_submit=c.t_submit, t_admit=c.t_admit, t_done=c.t_done,
                            status=c.status, batch_size=c.batch_size))
        return out

    def stats(self):
        st = ServerStats()
        _check(self._lib.ldp_server_stats_get(self._srv, ctypes.byref(st)), "ldp_server_stats_get")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._srv:
            self._lib.ldp_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
