"""Window histograms (non-overlapping w x w windows, Section 3.2) through the
C ABI against the oracle: single images (fused and two-pass paths) and batch
plans, bit-exact."""
import numpy as np
import pytest

from conftest import gpu_available
from oracle import lbp as oracle_lbp
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


@pytest.mark.parametrize("win", [(10, 10), (20, 20), (25, 25), (50, 50), (100, 100), (7, 13),
                                 (1, 1), (500, 3), (3, 700)])
def test_window_extract_matches_oracle(lib, win):
    """280x280 (Table 3's geometry), the 490x640 frame (10-px windows give 64
    columns: two runs of cells per cell row) and a small odd image."""
    for img in [synth.image(synth.KIND_BLUR_RECTS, 12, 0, 280, 280),
                synth.workload_image("single", 0),
                synth.image(synth.KIND_BLUR_SP_FLAT, 13, 1, 37, 51)]:
        wc = oracle_c.ldp_codes(img, 3)
        wh = oracle_np.window_histograms(wc, *win)
        c, h = lib.extract_windows(_dev(img), 3, *win)
        assert (c.cpu().numpy() == wc).all(), (img.shape, win)
        assert h.shape == wh.shape
        assert (h.cpu().numpy().view(np.uint32) == wh).all(), (img.shape, win)
        h2 = lib.histograms_windows(c, *win)
        assert (h2.cpu().numpy().view(np.uint32) == wh).all(), (img.shape, win)


def test_window_extract_without_codes(lib):
    img = synth.image(synth.KIND_BLUR_RECTS, 14, 0, 280, 280)
    _, h = lib.extract_windows(_dev(img), 3, 10, 10, want_codes=False)
    wh = oracle_np.window_histograms(oracle_c.ldp_codes(img, 3), 10, 10)
    assert (h.cpu().numpy().view(np.uint32) == wh).all()
    big = synth.workload_image("single", 0)  # 64 window columns: two runs of 32
    for win in ((10, 10), (1, 1), (3, 5)):
        _, h = lib.extract_windows(_dev(big), 3, *win, want_codes=False)
        wh = oracle_np.window_histograms(oracle_c.ldp_codes(big, 3), *win)
        assert (h.cpu().numpy().view(np.uint32) == wh).all(), win


class WinBatch:
    def __init__(self, Hs, Ws, kind, seed, win):
        self.Hs, self.Ws, self.win = np.asarray(Hs), np.asarray(Ws), win
        off, strides, total = synth.layout(self.Hs, self.Ws)
        host = np.zeros(total + 64, np.uint8)
        synth.fill(host, off, self.Hs, self.Ws, strides, kind, seed)
        self.host, self.off, self.strides = host, off, strides
        self.dev = torch.from_numpy(host).cuda()
        self.codes, self.hist = [], []
        for h, w in zip(self.Hs, self.Ws):
            ny, nx = -(-(int(h) - 2) // win[0]), -(-(int(w) - 2) // win[1])
            self.codes.append(torch.full(((h - 2) * (w - 2),), 0xAB, dtype=torch.uint8, device="cuda"))
            self.hist.append(torch.full((ny, nx, 256), 7, dtype=torch.int32, device="cuda"))
        base = self.dev.data_ptr()
        self.args = ([base + int(o) for o in off], [c.data_ptr() for c in self.codes],
                     [h.data_ptr() for h in self.hist], [int(s) for s in strides],
                     [int(h) for h in self.Hs], [int(w) for w in self.Ws])

    def image(self, j):
        H, W, s, o = int(self.Hs[j]), int(self.Ws[j]), int(self.strides[j]), int(self.off[j])
        return self.host[o:o + H * s].reshape(H, s)[:, :W]


@pytest.mark.parametrize("mode", ["signed", "magnitude", "lbp", "direct"])
def test_window_batch_plan_matches_oracle(lib, mode):
    r = np.random.default_rng(90)
    n = 40
    win = (10, 10)
    Hs, Ws = r.integers(3, 400, n), r.integers(3, 600, n)
    Hs[:3], Ws[:3] = [280, 3, 490], [280, 600, 3]
    b = WinBatch(Hs, Ws, synth.KIND_BLUR_SP_FLAT, 91, win)
    flags = {"signed": 0, "magnitude": lib.LDP_RANK_MAGNITUDE, "lbp": lib.LDP_CODE_LBP,
             "direct": lib.LDP_DIRECT_MASKS}[mode]
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, 3, *win, flags=flags, windows=True, max_width=600)
    plan.set(lib.BatchPlan.descs(*b.args))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        img = b.image(j)
        if mode == "lbp":
            wc = oracle_lbp.lbp_codes(img)
        else:
            wc = oracle_c.ldp_codes(img, 3, magnitude=(mode == "magnitude"))
        wh = oracle_np.window_histograms(wc, *win)
        assert (b.codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (b.hist[j].cpu().numpy().view(np.uint32) == wh).all(), j
    plan.close()


def test_window_plan_grows_its_item_table_and_rejects_wide_images(lib):
    """One-row windows give one work item per code row: far more than the
    initial table holds.  Images wider than max_width are refused."""
    r = np.random.default_rng(92)
    n = 12
    win = (1, 16)
    Hs, Ws = r.integers(100, 300, n), r.integers(20, 200, n)
    b = WinBatch(Hs, Ws, synth.KIND_BLUR_RECTS, 93, win)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, 2, *win, windows=True, max_width=200)
    plan.set(lib.BatchPlan.descs(*b.args))
    items, _ = plan.info()
    assert items > 8 * n
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        wc = oracle_c.ldp_codes(b.image(j), 2)
        assert (b.hist[j].cpu().numpy().view(np.uint32) == oracle_np.window_histograms(wc, *win)).all(), j
    wide = WinBatch([50], [300], synth.KIND_BLUR_RECTS, 94, win)
    with pytest.raises(lib.LdpError):
        plan.set(lib.BatchPlan.descs(*wide.args))
    plan.close()


@pytest.mark.parametrize("win", [(10, 10), (7, 3), (2, 1)])
def test_window_plan_rows_wider_than_63_windows(lib, win):
    """Table 3's 10x10 windows on 640-wide frames (64 window columns) and finer
    grids (up to 638 windows a row) in a batch plan: each cell row is cut into
    runs of at most 63 windows over several work items; images of other widths
    in the same batch take their own runs."""
    r = np.random.default_rng(95)
    n = 24
    Hs, Ws = r.integers(3, 500, n), r.integers(3, 641, n)
    Hs[:4], Ws[:4] = [490, 490, 100, 12], [640, 640, 639, 400]
    b = WinBatch(Hs, Ws, synth.KIND_BLUR_RECTS, 96, win)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, 3, *win, windows=True, max_width=640)
    plan.set(lib.BatchPlan.descs(*b.args))
    plan.run()
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        wc = oracle_c.ldp_codes(b.image(j), 3)
        assert (b.codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (b.hist[j].cpu().numpy().view(np.uint32) == oracle_np.window_histograms(wc, *win)).all(), j
    plan.close()


@pytest.mark.parametrize("cells_x", [64, 100, 130])
def test_cell_plan_more_than_63_cell_columns(lib, cells_x):
    """Cell grids wider than one workgroup's LDS row, in batch plans and in the
    single-image call without a code map."""
    r = np.random.default_rng(97 + cells_x)
    n = 10
    Hs, Ws = r.integers(20, 300, n), r.integers(cells_x + 2, 900, n)
    off, strides, total = synth.layout(Hs, Ws)
    host = np.zeros(total + 64, np.uint8)
    synth.fill(host, off, Hs, Ws, strides, synth.KIND_BLUR_SP_FLAT, 98)
    dev = torch.from_numpy(host).cuda()
    grid = (3, cells_x)
    codes = [torch.empty((int(h) - 2) * (int(w) - 2), dtype=torch.uint8, device="cuda")
             for h, w in zip(Hs, Ws)]
    hists = [torch.full(grid + (256,), 7, dtype=torch.int32, device="cuda") for _ in range(n)]
    plan = lib.BatchPlan(n, int((Hs.astype(np.int64) * Ws).sum()), 3, *grid)
    plan.set(lib.BatchPlan.descs([dev.data_ptr() + int(o) for o in off],
                                 [c.data_ptr() for c in codes], [h.data_ptr() for h in hists],
                                 [int(s) for s in strides], [int(h) for h in Hs],
                                 [int(w) for w in Ws]))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        H, W, s, o = int(Hs[j]), int(Ws[j]), int(strides[j]), int(off[j])
        img = host[o:o + H * s].reshape(H, s)[:, :W]
        wc = oracle_c.ldp_codes(img, 3)
        wh = oracle_c.ldp_histograms(wc, *grid)
        assert (codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (hists[j].cpu().numpy().view(np.uint32) == wh).all(), j
        _, h1 = lib.extract(_dev(img), 3, *grid, want_codes=False)
        assert (h1.cpu().numpy().view(np.uint32) == wh).all(), j
    plan.close()


@pytest.mark.parametrize("w", [10, 20, 25, 50, 100])
def test_window_plan_with_cached_tunes(lib, w):
    """The launch shapes the autotuner cached for window plans of the 490x640
    batch (smaller workgroups, two window rows per item, short lane tasks)
    give the oracle's codes and window histograms: 6 frames of that batch."""
    from paper_1810_11518_amd import autotune
    Hs, Ws = synth.workload_sizes("batch")
    tune = autotune.load_cache().get(
        "gfx950|k3|%dx%d|%dx%d|win" % (w, w, int(Hs[0]), int(Ws[0])), {}).get("tune")
    assert tune, "no cached window tune for %d px" % w
    n = 6
    b = WinBatch(Hs[:n], Ws[:n], synth.WORKLOADS["batch"]["kind"], synth.SEEDS["batch"], (w, w))
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, 3, w, w, tune, windows=True, max_width=int(Ws[0]))
    plan.set(lib.BatchPlan.descs(*b.args))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        wc = oracle_c.ldp_codes(b.image(j), 3)
        assert (b.codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (b.hist[j].cpu().numpy().view(np.uint32) == oracle_np.window_histograms(wc, w, w)).all(), j
    plan.close()
