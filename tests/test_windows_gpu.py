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
    columns: the two-pass path) and a small odd image."""
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
    big = synth.workload_image("single", 0)  # 64 window columns need the code map
    with pytest.raises(lib.LdpError):
        lib.extract_windows(_dev(big), 3, 10, 10, want_codes=False)


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
