"""The C ABI library: loads, exports every symbol include/ldp.h declares,
and rejects invalid arguments on the host before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1810_11518_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "ldp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ldp_\w+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_t")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1810_11518_amd import build
        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(binding.EXPORTED) | {"ldp_stream_t"}


def test_status_strings_and_version(lib):
    assert lib.ldp_version() == 1
    assert lib.ldp_status_string(0) == b"ok"
    assert b"invalid" in lib.ldp_status_string(-1)


def test_invalid_arguments_return_before_any_launch(lib):
    p = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    E = binding.LDP_ERR_INVALID_ARG
    assert lib.ldp_codes(None, 10, 10, 10, 3, p, None) == E
    assert lib.ldp_codes(p, 2, 10, 10, 3, p, None) == E
    assert lib.ldp_codes(p, 10, 2, 10, 3, p, None) == E
    assert lib.ldp_codes(p, 10, 10, 9, 3, p, None) == E
    assert lib.ldp_codes(p, 10, 10, 10, 0, p, None) == E
    assert lib.ldp_codes(p, 10, 10, 10, 9, p, None) == E
    assert lib.ldp_codes(p, 10, 70000, 70000, 3, p, None) == E
    assert lib.ldp_histograms(p, 10, 10, 9, 1, p, None) == E
    assert lib.ldp_histograms(p, 10, 10, 1, 0, p, None) == E
    assert lib.ldp_extract(p, 10, 10, 10, 3, 1, 1, None, None, None) == E
    assert lib.ldp_extract(p, 10, 10, 10, 3, 0, 1, p, p, None) == E
    assert lib.ldp_codes(p, 40000, 60000, 60000, 3, p, None) == binding.LDP_ERR_UNSUPPORTED
    # sides above 65536, and the first extents past (H - 1) * stride + W + 8 <= 2^31 - 64
    # (32767 x 65536 at pitch 65536, the largest image the GPU tests run, is inside)
    assert lib.ldp_codes(p, 10, 65537, 65537, 3, p, None) == E
    assert lib.ldp_codes(p, 65537, 10, 10, 3, p, None) == E
    assert lib.ldp_codes(p, 32768, 65536, 65536, 3, p, None) == binding.LDP_ERR_UNSUPPORTED
    assert lib.ldp_codes(p, 32767, 65536, 65538, 3, p, None) == binding.LDP_ERR_UNSUPPORTED
    assert lib.ldp_extract(p, 32768, 65536, 65536, 3, 16, 16, p, p, None) == binding.LDP_ERR_UNSUPPORTED
    plan = ctypes.c_void_p()
    assert lib.ldp_batch_plan_create(ctypes.byref(plan), 0, 100, 3, 7, 6, None) == E
    assert lib.ldp_batch_plan_create(ctypes.byref(plan), 10, 100, 9, 7, 6, None) == E
    assert lib.ldp_batch_plan_create(ctypes.byref(plan), 10, 100, 3, 7, 70000, None) == E
    assert lib.ldp_batch_plan_create(ctypes.byref(plan), 1 << 30, 100, 3, 7, 6, None) == E
    for th in (300, 32, 1088):  # not a whole number of waves, or above 1024
        t = binding.make_tune(dict(block_threads=th))
        assert lib.ldp_batch_plan_create(ctypes.byref(plan), 10, 100, 3, 7, 6, ctypes.byref(t)) == E
    assert lib.ldp_batch_run(None, None) == E
    assert lib.ldp_batch_launch(None, None, 0, None) == E
    assert lib.ldp_batch_launch(None, None, -1, None) == E
    # variants: unknown flag bits, and the same checks as the plain calls
    for bad_flags in (3, 5, 6, 7, 8, -1):  # one flag at most, and only known ones
        assert lib.ldp_codes_ex(p, 10, 10, 10, 3, bad_flags, p, None) == E
    assert lib.ldp_codes_ex(p, 10, 10, 10, 0, binding.LDP_CODE_LBP, p, None) == E  # k still checked
    assert lib.ldp_codes_ex(p, 10, 10, 9, 3, binding.LDP_RANK_MAGNITUDE, p, None) == E
    assert lib.ldp_extract_ex(p, 10, 10, 10, 3, 8, 1, 1, p, p, None) == E
    assert lib.ldp_extract_ex(p, 10, 10, 10, 9, 1, 1, 1, p, p, None) == E
    assert lib.ldp_batch_plan_create_ex(ctypes.byref(plan), 10, 100, 3, 8, 7, 6, None) == E
    assert lib.ldp_compact_histograms(p, 5, 0, p, None) == E
    assert lib.ldp_compact_histograms(p, -1, 3, p, None) == E
    assert lib.ldp_compact_histograms(None, 5, 3, p, None) == E
    assert lib.ldp_compact_histograms(None, 0, 3, None, None) == binding.LDP_OK  # nothing to do
    assert lib.ldp_extract_windows(p, 10, 10, 10, 3, 0, 0, 2, p, p, None) == E
    assert lib.ldp_extract_windows(p, 10, 10, 10, 3, 0, 2, 0, p, p, None) == E
    assert lib.ldp_extract_windows(p, 10, 10, 10, 3, 8, 2, 2, p, p, None) == E
    assert lib.ldp_histograms_windows(p, 10, 10, 0, 1, p, None) == E
    assert lib.ldp_batch_plan_create_windows(ctypes.byref(plan), 10, 100, 2, 3, 0, 5, 5, None) == E
    assert lib.ldp_batch_plan_create_windows(ctypes.byref(plan), 10, 10 ** 6, 70000, 3, 0, 5, 5,
                                             None) == E
    descs = (binding.ImageDesc * 29)()
    for d in descs:
        d.img, d.hist, d.stride, d.H, d.W = 0x1000, 0x2000, 40, 40, 40
    assert lib.ldp_batch_launch_noalloc(descs, -1, 3, 7, 6, None) == E
    assert lib.ldp_batch_launch_noalloc(None, 3, 3, 7, 6, None) == E
    assert lib.ldp_batch_launch_noalloc(descs, 3, 0, 7, 6, None) == E
    assert lib.ldp_batch_launch_noalloc(descs, 3, 3, 0, 6, None) == E
    assert lib.ldp_batch_launch_noalloc(descs, 3, 3, 7, 39, None) == E       # W - 2 < cells_x
    assert lib.ldp_batch_launch_noalloc(descs, 29, 3, 7, 6, None) == binding.LDP_ERR_UNSUPPORTED
    assert lib.ldp_batch_launch_noalloc(descs, 28, 3, 8, 6, None) == binding.LDP_ERR_UNSUPPORTED
    assert lib.ldp_batch_launch_noalloc(descs, 0, 3, 7, 6, None) == binding.LDP_OK  # nothing to do
    assert lib.ldp_stream_copy(p, p, -1, None) == E
    assert lib.ldp_stream_copy(None, p, 16, None) == E
    assert lib.ldp_stream_copy(p, None, 16, None) == E
    assert lib.ldp_stream_copy(ctypes.c_void_p(0x1004), p, 16, None) == E   # not 16-byte aligned
    assert lib.ldp_stream_copy(None, None, 0, None) == binding.LDP_OK      # nothing to do
    srv = ctypes.c_void_p()
    bad = binding.ServerConfig(0, 1, 1, 1, 3, 7, 6, 1, 0)
    assert lib.ldp_server_create(ctypes.byref(srv), ctypes.byref(bad)) == E
    bad = binding.ServerConfig(1 << 20, 1, 1, 9, 3, 7, 6, 1, 0)
    assert lib.ldp_server_create(ctypes.byref(srv), ctypes.byref(bad)) == E
    bad = binding.ServerConfig(1 << 20, 1, 1, 1, 3, 7, 6, 1, 0, 2)   # unknown flag
    assert lib.ldp_server_create(ctypes.byref(srv), ctypes.byref(bad)) == E
    ok = binding.ServerConfig(1 << 20, 1, 1, 1, 3, 7, 6, 1, 0, binding.LDP_SERVER_NO_MIRROR)
    assert lib.ldp_server_create(ctypes.byref(srv), ctypes.byref(ok)) == binding.LDP_OK
    assert lib.ldp_server_destroy(srv) == binding.LDP_OK


def test_compact_bin_counts(lib):
    import math
    assert lib.ldp_compact_bins(3) == 57  # Eq. 6: 56 pattern values, plus the tie bin
    for k in range(1, 9):
        assert lib.ldp_compact_bins(k) == math.comb(8, k) + 1
    assert lib.ldp_compact_bins(0) == binding.LDP_ERR_INVALID_ARG
    assert lib.ldp_compact_bins(9) == binding.LDP_ERR_INVALID_ARG


def test_window_grid_counts_of_table3(lib):
    """Table 3: 784, 196, 144, 36 and 9 windows for a 280x280 image."""
    for w, n in ((10, 784), (20, 196), (25, 144), (50, 36), (100, 9)):
        ny, nx = binding.window_grid(280, 280, w, w)
        assert ny * nx == n
    assert binding.window_grid(3, 3, 5, 5) == (1, 1)
    assert lib.ldp_window_grid(2, 9, 1, 1, None, None) == binding.LDP_ERR_INVALID_ARG


def test_tune_struct_layout():
    t = binding.make_tune(dict(block_threads=512, classes=[dict(max_pixels=10, cell_rows_per_item=2,
                                                                 rows_per_task=4), {}]))
    assert ctypes.sizeof(binding.Tune) == 16 + 4 * 16
    assert t.n_classes == 2 and t.classes[0].max_pixels == 10 and t.classes[1].cell_rows_per_item == 0
    assert ctypes.sizeof(binding.ImageDesc) == 40
