"""The largest inputs the C ABI accepts, through the C ABI against the oracle:
images LDP_MAX_SIDE (65536) pixels long in one direction and a few pixels in
the other (every code checked), and one image at the largest byte extent the
path takes (32767 x 65536, 2.1 G pixels, just under 2^31 bytes: every row
and code offset near the top of its 32-bit range), checked on sampled code
rows and through histograms that must equal the oracle's histograms of the
returned codes."""
import numpy as np
import pytest

from conftest import gpu_available
from oracle import lbp as oracle_lbp
from oracle import ldp as oracle_np
from oracle import native as oracle_c
from paper_1810_11518_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAX_SIDE = 65536
SKINNY = [(MAX_SIDE, 3), (MAX_SIDE, 5), (MAX_SIDE, 13), (3, MAX_SIDE), (4, MAX_SIDE),
          (7, MAX_SIDE)]


@pytest.fixture(scope="module")
def lib():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1810_11518_amd import binding
    binding.load()
    return binding


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _skinny(j, H, W):
    return synth.image(synth.KIND_BLUR_SP_FLAT if j % 2 else synth.KIND_UNIFORM, 120, j, H, W)


def _oracle_codes(lib, img, k, flags):
    if flags == lib.LDP_CODE_LBP:
        return oracle_lbp.lbp_codes(img)
    return oracle_c.ldp_codes(img, k, magnitude=(flags == lib.LDP_RANK_MAGNITUDE))


@pytest.mark.parametrize("k", [1, 3, 5, 8])
def test_max_side_codes_and_histograms(lib, k):
    for j, (H, W) in enumerate(SKINNY):
        img = _skinny(j, H, W)
        want = oracle_c.ldp_codes(img, k)
        assert (lib.codes(_dev(img), k).cpu().numpy() == want).all(), (H, W, k)
        # one run of cells per row, and for the long rows also rows cut into runs
        # (more than 63 cell columns)
        grids = [(min(7, H - 2), min(6, W - 2))]
        if W == MAX_SIDE:
            grids += [(1, 63), (H - 2, 64)]
        for cy, cx in grids:
            c, h = lib.extract(_dev(img), k, cy, cx)
            assert (c.cpu().numpy() == want).all(), (H, W, k, cy, cx)
            wh = oracle_c.ldp_histograms(want, cy, cx)
            assert (h.cpu().numpy().view(np.uint32) == wh).all(), (H, W, k, cy, cx)


@pytest.mark.parametrize("mode", ["magnitude", "direct", "lbp"])
def test_max_side_variants(lib, mode):
    flags = {"magnitude": lib.LDP_RANK_MAGNITUDE, "direct": lib.LDP_DIRECT_MASKS,
             "lbp": lib.LDP_CODE_LBP}[mode]
    for j, (H, W) in enumerate(SKINNY):
        img = _skinny(j + 10, H, W)
        want = _oracle_codes(lib, img, 3, flags)
        assert (lib.codes(_dev(img), 3, flags=flags).cpu().numpy() == want).all(), (H, W)
        cy, cx = min(5, H - 2), min(3, W - 2)
        c, h = lib.extract(_dev(img), 3, cy, cx, flags=flags)
        assert (c.cpu().numpy() == want).all(), (H, W)
        assert (h.cpu().numpy().view(np.uint32) == oracle_c.ldp_histograms(want, cy, cx)).all()


def test_max_side_windows(lib):
    """Windows over 65536-long maps: a window grid of 63 columns (one run),
    66 columns (two runs of 33) and 656 window rows."""
    cases = [((4, MAX_SIDE), (2, 1041)), ((4, MAX_SIDE), (2, 1000)), ((MAX_SIDE, 7), (100, 100)),
             ((MAX_SIDE, 13), (1000, 4))]
    for j, ((H, W), win) in enumerate(cases):
        img = _skinny(j + 20, H, W)
        want = oracle_c.ldp_codes(img, 3)
        c, h = lib.extract_windows(_dev(img), 3, *win)
        assert (c.cpu().numpy() == want).all(), (H, W, win)
        assert (h.cpu().numpy().view(np.uint32) == oracle_np.window_histograms(want, *win)).all()


def _plan_outputs(lib, imgs, k, grid, flags=0, windows=False, max_width=None):
    """Run one batch plan over device copies of imgs; returns (codes, hists)
    as host arrays."""
    dev = [_dev(i) for i in imgs]
    codes = [torch.full(((i.shape[0] - 2), (i.shape[1] - 2)), 0xAB, dtype=torch.uint8,
                        device="cuda") for i in imgs]
    if windows:
        shapes = [(-(-(i.shape[0] - 2) // grid[0]), -(-(i.shape[1] - 2) // grid[1])) for i in imgs]
    else:
        shapes = [grid] * len(imgs)
    hists = [torch.full(s + (256,), 7, dtype=torch.int32, device="cuda") for s in shapes]
    pixels = sum(i.size for i in imgs)
    plan = lib.BatchPlan(len(imgs), pixels, k, *grid, flags=flags, windows=windows,
                         max_width=max_width)
    plan.set(lib.BatchPlan.descs([d.data_ptr() for d in dev], [c.data_ptr() for c in codes],
                                 [h.data_ptr() for h in hists], [d.stride(0) for d in dev],
                                 [d.shape[0] for d in dev], [d.shape[1] for d in dev]))
    plan.run()
    torch.cuda.synchronize()
    out = [c.cpu().numpy() for c in codes], [h.cpu().numpy().view(np.uint32) for h in hists]
    plan.close()
    return out


@pytest.mark.parametrize("mode", ["signed", "magnitude", "lbp"])
def test_max_side_batch_plans(lib, mode):
    flags = {"signed": 0, "magnitude": lib.LDP_RANK_MAGNITUDE, "lbp": lib.LDP_CODE_LBP}[mode]
    imgs = [_skinny(j + 30, H, W) for j, (H, W) in enumerate(SKINNY)]
    imgs.append(synth.workload_image("single", 1))
    grid = (1, 1)
    codes, hists = _plan_outputs(lib, imgs, 3, grid, flags=flags)
    for j, img in enumerate(imgs):
        want = _oracle_codes(lib, img, 3, flags)
        assert (codes[j] == want).all(), (mode, img.shape)
        assert (hists[j] == oracle_c.ldp_histograms(want, *grid)).all(), (mode, img.shape)


def test_max_side_window_batch_plan(lib):
    win = (5, 1100)  # 60 window columns over a 65534-column map
    imgs = [_skinny(40, 3, MAX_SIDE), _skinny(41, MAX_SIDE, 9), _skinny(42, 20, 30000),
            _skinny(43, 6, MAX_SIDE)]
    codes, hists = _plan_outputs(lib, imgs, 3, win, windows=True, max_width=MAX_SIDE)
    for j, img in enumerate(imgs):
        want = oracle_c.ldp_codes(img, 3)
        assert (codes[j] == want).all(), img.shape
        assert (hists[j] == oracle_np.window_histograms(want, *win)).all(), img.shape


# ------------------------------------------------------------ largest extent

BIG_H, BIG_W = 32767, MAX_SIDE   # (H - 1) * W + W + 8 = 2^31 - 65528 bytes


def _sample_rows(Hc):
    r = np.random.default_rng(121)
    rows = {0, 1, 2, Hc // 2, Hc - 3, Hc - 2, Hc - 1}
    rows.update(int(x) for x in r.integers(0, Hc, 40))
    return sorted(rows)


def _check_big(img, codes, hist, k, cells):
    """Sampled code rows against the oracle (a code row depends on three image
    rows only); every histogram against the oracle's histograms of the
    returned code map, which the sampled rows tie to the image."""
    c = codes.cpu().numpy()
    for r in _sample_rows(c.shape[0]):
        want = oracle_c.ldp_codes(img[r:r + 3], k)[0]
        assert (c[r] == want).all(), ("code row", r)
    got_h = hist.cpu().numpy().view(np.uint32)
    assert (got_h == oracle_c.ldp_histograms(c, *cells)).all()
    assert int(got_h.sum(dtype=np.int64)) == c.size


@pytest.fixture(scope="module")
def big_image(lib):
    img = synth.image(synth.KIND_UNIFORM, 122, 0, BIG_H, BIG_W)
    return img, _dev(img)


def test_largest_extent_single_image(lib, big_image):
    img, dev = big_image
    cells = (16, 16)
    codes, hist = lib.extract(dev, 3, *cells)
    torch.cuda.synchronize()
    _check_big(img, codes, hist, 3, cells)


def test_largest_extent_in_a_batch_plan(lib, big_image):
    img, dev = big_image
    small = synth.workload_image("single", 2)
    sdev = _dev(small)
    cells = (7, 6)
    codes = [torch.full((BIG_H - 2, BIG_W - 2), 0xAB, dtype=torch.uint8, device="cuda"),
             torch.full((small.shape[0] - 2, small.shape[1] - 2), 0xAB, dtype=torch.uint8,
                        device="cuda")]
    hists = [torch.full(cells + (256,), 7, dtype=torch.int32, device="cuda") for _ in range(2)]
    plan = lib.BatchPlan(2, img.size + small.size, 3, *cells)
    plan.set(lib.BatchPlan.descs([dev.data_ptr(), sdev.data_ptr()], [c.data_ptr() for c in codes],
                                 [h.data_ptr() for h in hists], [BIG_W, small.shape[1]],
                                 [BIG_H, small.shape[0]], [BIG_W, small.shape[1]]))
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    _check_big(img, codes[0], hists[0], 3, cells)
    wc, wh = oracle_c.ldp_extract(small, 3, *cells)
    assert (codes[1].cpu().numpy() == wc).all()
    assert (hists[1].cpu().numpy().view(np.uint32) == wh).all()
