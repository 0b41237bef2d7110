"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact equality is required everywhere: the path is integer-only.
"""
import numpy as np
import pytest

from _golden import closed_forms
from conftest import gpu_available
from oracle import ldp as oracle_np
from oracle import native as oracle_c
from paper_1810_11518_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1810_11518_amd import binding
    binding.load()
    return binding


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _strided(img, pad, shift):
    """Device view of img with row pitch W+pad starting `shift` bytes into a
    buffer (so the base address is misaligned when shift % 4 != 0)."""
    H, W = img.shape
    pitch = W + pad
    buf = torch.zeros(shift + H * pitch + 16, dtype=torch.uint8, device="cuda")
    host = np.zeros((H, pitch), np.uint8)
    host[:, :W] = img
    buf[shift:shift + H * pitch] = torch.from_numpy(host.ravel()).cuda()
    return buf[shift:shift + H * pitch].view(H, pitch)[:, :W]


def _imgs():
    r = np.random.default_rng(21)
    out = []
    for H, W in [(3, 3), (3, 11), (4, 3), (5, 9), (9, 10), (17, 23), (64, 64), (33, 130),
                 (100, 257), (48, 1024), (1024, 48)]:
        out.append(r.integers(0, 256, (H, W), dtype=np.uint8))
    out.append(synth.workload_image("single", 0))                         # 490x640 noise
    out.append(synth.image(synth.KIND_BLUR_RECTS, 5, 0, 203, 317))
    out.append(synth.image(synth.KIND_BLUR_SP_FLAT, 6, 0, 300, 411))      # many ties
    out.append((r.integers(0, 3, (77, 91)) * 100).astype(np.uint8))         # tiny alphabet
    return out


@pytest.mark.parametrize("k", range(1, 9))
def test_codes_match_oracle(lib, k):
    for img in _imgs():
        got = lib.codes(_dev(img), k).cpu().numpy()
        want = oracle_c.ldp_codes(img, k)
        assert got.shape == want.shape
        assert (got == want).all(), (img.shape, k, np.argwhere(got != want)[:5])


@pytest.mark.parametrize("pad,shift", [(0, 1), (1, 0), (3, 2), (5, 3), (4, 0), (13, 1), (64, 3)])
def test_codes_strided_and_misaligned(lib, pad, shift):
    for H, W in [(5, 7), (31, 45), (70, 333), (257, 130)]:
        img = synth.image(synth.KIND_BLUR_RECTS, 100 + pad, shift, H, W)
        dimg = _strided(img, pad, shift)
        for k in (2, 3, 4):
            got = lib.codes(dimg, k).cpu().numpy()
            assert (got == oracle_c.ldp_codes(img, k)).all(), (H, W, pad, shift, k)


def test_closed_forms_on_gpu(lib):
    for case in closed_forms():
        got = lib.codes(_dev(case["image"]), case["k"]).cpu().numpy()
        assert (got == case["codes"]).all(), case["name"]


def test_quarter_turn_rotates_codes(lib):
    img = synth.image(synth.KIND_BLUR_RECTS, 9, 0, 123, 207)
    c = lib.codes(_dev(img), 3).cpu().numpy().astype(np.int64)
    c2 = lib.codes(_dev(np.rot90(img)), 3).cpu().numpy().astype(np.int64)
    rot = (((c << 2) | (c >> 6)) & 255)
    assert (c2 == np.rot90(rot)).all()


@pytest.mark.parametrize("cells", [(1, 1), (7, 6), (3, 5), (16, 16), (2, 64), (1, 100)])
def test_histograms_match_oracle(lib, cells):
    cy, cx = cells
    for H, W in [(490, 640), (67, 129), (20, 500), (130, 66)]:
        if cy > H - 2 or cx > W - 2:
            continue
        img = synth.image(synth.KIND_BLUR_RECTS, 3, H * W, H, W)
        codes = oracle_c.ldp_codes(img, 3)          # oracle codes as the input
        got = lib.histograms(_dev(codes), cy, cx).cpu().numpy().view(np.uint32)
        assert (got == oracle_c.ldp_histograms(codes, cy, cx)).all(), (H, W, cells)


@pytest.mark.parametrize("shift", [0, 1, 3])
def test_histograms_kernel_layouts(lib, shift):
    """The histogram kernel's layouts: code maps narrower than one 16-column
    chunk, widths with and without 4-aligned rows, a code map starting at any
    byte, cells narrower than 16 columns, more than 63 cells in a row (several
    items per cell row), tall maps whose cell rows are split over workgroups
    (atomic flush), and flat regions (one add of 16)."""
    r = np.random.default_rng(40 + shift)
    cases = [(5, 9, (1, 1)), (9, 14, (2, 3)), (20, 18, (3, 2)), (34, 66, (4, 4)),
             (70, 130, (5, 9)), (300, 260, (16, 16)), (40, 1002, (2, 100)),
             (1500, 42, (3, 1)), (2000, 2000, (1, 1)), (515, 1030, (7, 64))]
    for H, W, (cy, cx) in cases:
        img = synth.image(synth.KIND_BLUR_RECTS, 5, H * 7 + W, H, W)
        codes = oracle_c.ldp_codes(img, int(r.integers(1, 9)))
        if H * W % 3 == 0:
            codes[: codes.shape[0] // 2] = 255          # a flat half: equal codes
        n = codes.size
        buf = torch.zeros(shift + n + 16, dtype=torch.uint8, device="cuda")
        buf[shift:shift + n] = torch.from_numpy(codes.ravel()).cuda()
        dev = buf[shift:shift + n].view(codes.shape)
        got = lib.histograms(dev, cy, cx).cpu().numpy().view(np.uint32)
        assert (got == oracle_c.ldp_histograms(codes, cy, cx)).all(), (H, W, cy, cx, shift)
        for w in (3, 16, 25):
            if (codes.shape[0] // w + 1) * (codes.shape[1] // w + 1) > 20000:
                continue                                  # the oracle loops over windows
            got = lib.histograms_windows(dev, w, w).cpu().numpy().view(np.uint32)
            want = oracle_np.window_histograms(codes, w, w)
            assert (got == want).all(), (H, W, w, shift)


def test_histograms_one_pixel_cells(lib):
    img = np.random.default_rng(4).integers(0, 256, (12, 14), dtype=np.uint8)
    codes = oracle_c.ldp_codes(img, 3)
    got = lib.histograms(_dev(codes), 10, 12).cpu().numpy().view(np.uint32)
    assert (got == oracle_np.ldp_histograms(codes, 10, 12)).all()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8])
def test_extract_matches_oracle(lib, k):
    cases = [((490, 640), (7, 6)), ((203, 317), (7, 6)), ((48, 48), (7, 6)), ((1024, 48), (16, 1)),
             ((600, 2050), (16, 16)), ((9, 9), (7, 7)), ((130, 1000), (3, 64)), ((40, 300), (2, 70))]
    for (H, W), (cy, cx) in cases:
        img = synth.image(synth.KIND_BLUR_SP_FLAT if H > 500 else synth.KIND_BLUR_RECTS, 11, k, H, W)
        codes, hist = lib.extract(_dev(img), k, cy, cx)
        want_c, want_h = oracle_c.ldp_extract(img, k, cy, cx)
        assert (codes.cpu().numpy() == want_c).all(), ((H, W), k)
        assert (hist.cpu().numpy().view(np.uint32) == want_h).all(), ((H, W), (cy, cx), k)


def test_extract_histograms_only(lib):
    img = synth.image(synth.KIND_BLUR_RECTS, 12, 0, 300, 500)
    none, hist = lib.extract(_dev(img), 3, 7, 6, want_codes=False)
    assert none is None
    assert (hist.cpu().numpy().view(np.uint32) == oracle_c.ldp_extract(img, 3, 7, 6)[1]).all()


def test_extract_misaligned_strided(lib):
    img = synth.image(synth.KIND_BLUR_RECTS, 13, 0, 211, 333)
    dimg = _strided(img, 7, 3)
    codes, hist = lib.extract(dimg, 3, 7, 6)
    want_c, want_h = oracle_c.ldp_extract(img, 3, 7, 6)
    assert (codes.cpu().numpy() == want_c).all()
    assert (hist.cpu().numpy().view(np.uint32) == want_h).all()


def test_argument_errors_do_not_launch(lib):
    x = torch.zeros((2, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.LdpError):
        lib.codes(x, 3)
    y = torch.zeros((10, 10), dtype=torch.uint8, device="cuda")
    with pytest.raises(lib.LdpError):
        lib.codes(y, 9)
    with pytest.raises(lib.LdpError):
        lib.extract(y, 3, 9, 1)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_large_image_full_size(lib, k):
    """One 8192x8192 image of the bandwidth workload (flat patches: exact
    ties), 16x16 cells: codes and histograms bit-exact against the oracle."""
    img = synth.workload_image("large", 0)
    codes, hist = lib.extract(_dev(img), k, 16, 16)
    want_c = oracle_c.ldp_codes(img, k)
    assert (codes.cpu().numpy() == want_c).all()
    assert (hist.cpu().numpy().view(np.uint32) == oracle_c.ldp_histograms(want_c, 16, 16)).all()
