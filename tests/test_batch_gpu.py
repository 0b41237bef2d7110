"""The persistent, graph-captured batch launch against the oracle."""
import numpy as np
import pytest

from conftest import gpu_available
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


class Batch:
    """Images packed back to back in one device buffer, with outputs."""

    def __init__(self, Hs, Ws, kind, seed, cells, row_align=1, shift=0, with_codes=True):
        self.Hs, self.Ws = np.asarray(Hs), np.asarray(Ws)
        off, strides, total = synth.layout(self.Hs, self.Ws, row_align=row_align)
        off = off + shift
        host = np.zeros(total + shift + 64, np.uint8)
        synth.fill(host, off, self.Hs, self.Ws, strides, kind, seed)
        self.host, self.off, self.strides = host, off, strides
        self.dev = torch.from_numpy(host).cuda()
        n = len(Hs)
        self.codes = [torch.full(((h - 2) * (w - 2),), 0xAB, dtype=torch.uint8, device="cuda")
                      if with_codes else None for h, w in zip(Hs, Ws)]
        cy, cx = cells
        self.hist = [torch.full((cy * cx * 256,), 7, dtype=torch.int32, device="cuda")
                     for _ in range(n)]
        base = self.dev.data_ptr()
        self.descs_args = ([base + int(o) for o in off],
                           [c.data_ptr() if c is not None else None for c in self.codes],
                           [h.data_ptr() for h in self.hist], [int(s) for s in strides],
                           [int(h) for h in Hs], [int(w) for w in Ws])

    def image(self, j):
        H, W, s, o = int(self.Hs[j]), int(self.Ws[j]), int(self.strides[j]), int(self.off[j])
        return self.host[o:o + H * s].reshape(H, s)[:, :W]

    def check(self, j, k, cells, codes=True):
        img = self.image(j)
        want_c, want_h = oracle_c.ldp_extract(img, k, *cells)
        if codes:
            got_c = self.codes[j].cpu().numpy().reshape(want_c.shape)
            assert (got_c == want_c).all(), ("codes", j, img.shape)
        got_h = self.hist[j].cpu().numpy().view(np.uint32).reshape(want_h.shape)
        assert (got_h == want_h).all(), ("hist", j, img.shape)


def _plan(lib, b, k, cells, tune=None):
    n = len(b.Hs)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(max(n, 1), max(pixels, 9), k, cells[0], cells[1], tune)
    plan.set(lib.BatchPlan.descs(*b.descs_args))
    return plan


@pytest.mark.parametrize("k", [2, 3, 4])
def test_uneven_batch_matches_oracle(lib, k):
    r = np.random.default_rng(k)
    n = 60
    Hs = r.integers(9, 400, n)
    Ws = r.integers(9, 700, n)
    Hs[:3], Ws[:3] = [490, 9, 1024], [640, 1024, 9]
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 31 + k, (7, 6))
    plan = _plan(lib, b, k, (7, 6))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        b.check(j, k, (7, 6))


def test_histograms_in_buffers_not_16_byte_aligned(lib):
    """Each image's histograms 4 bytes past a 16-byte boundary: the flush
    goes word by word instead of 16 bytes at a time; same results (batch
    plan, and single-image extract with and without split cell rows)."""
    r = np.random.default_rng(61)
    n = 12
    cells = (7, 6)
    Hs, Ws = r.integers(20, 400, n), r.integers(20, 500, n)
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 62, cells)
    per = cells[0] * cells[1] * 256
    big = torch.full((n * per + 4,), 7, dtype=torch.int32, device="cuda")
    hists = [big[1 + j * per:1 + (j + 1) * per] for j in range(n)]
    assert all(h.data_ptr() % 16 == 4 for h in hists)
    args = list(b.descs_args)
    args[2] = [h.data_ptr() for h in hists]
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, 3, cells[0], cells[1])
    plan.set(lib.BatchPlan.descs(*args))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        _, want = oracle_c.ldp_extract(b.image(j), 3, *cells)
        assert (hists[j].cpu().numpy().view(np.uint32).reshape(want.shape) == want).all(), j
    plan.close()
    for img in (b.image(0), synth.workload_image("single", 0)):
        hv = torch.full((per + 4,), 7, dtype=torch.int32, device="cuda")[1:1 + per].view(7, 6, 256)
        _, h = lib.extract(torch.from_numpy(np.ascontiguousarray(img)).cuda(), 3, *cells,
                           hist_out=hv)
        _, want = oracle_c.ldp_extract(img, 3, *cells)
        assert (h.cpu().numpy().view(np.uint32) == want).all()


@pytest.mark.parametrize("tune", [
    dict(block_threads=256), dict(block_threads=1024, classes=[dict(rows_per_task=16)]),
    dict(block_threads=512, classes=[dict(cell_rows_per_item=3)]),
    dict(grid_blocks=5, classes=[dict(cell_rows_per_item=7)]),
    dict(block_threads=64, classes=[dict(rows_per_task=3)]),
    dict(block_threads=320, classes=[dict(cell_rows_per_item=2)]),
    dict(block_threads=448, grid_blocks=37, classes=[dict(cell_rows_per_item=4, rows_per_task=5)]),
    dict(block_threads=512, classes=[dict(max_pixels=20000, cell_rows_per_item=7, rows_per_task=2),
                                     dict(max_pixels=60000, cell_rows_per_item=2, rows_per_task=4),
                                     dict(cell_rows_per_item=1, rows_per_task=32)])])
def test_tunings_give_identical_results(lib, tune):
    r = np.random.default_rng(7)
    n = 24
    Hs, Ws = r.integers(20, 300, n), r.integers(20, 300, n)
    b = Batch(Hs, Ws, synth.KIND_BLUR_SP_FLAT, 5, (7, 6), row_align=4)
    plan = _plan(lib, b, 3, (7, 6), tune)
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        b.check(j, 3, (7, 6))


def test_graph_replay_with_new_batch_and_determinism(lib):
    r = np.random.default_rng(11)
    b1 = Batch(r.integers(30, 200, 20), r.integers(30, 200, 20), synth.KIND_BLUR_RECTS, 1, (4, 4))
    b2 = Batch(r.integers(30, 200, 35), r.integers(30, 200, 35), synth.KIND_BLUR_RECTS, 2, (4, 4),
               shift=1)
    plan = lib.BatchPlan(64, 10 ** 7, 3, 4, 4)
    plan.set(lib.BatchPlan.descs(*b1.descs_args))
    plan.run()
    torch.cuda.synchronize()
    first = [h.clone() for h in b1.hist]
    for j in range(20):
        b1.check(j, 3, (4, 4))
    plan.set(lib.BatchPlan.descs(*b2.descs_args))
    plan.run()
    torch.cuda.synchronize()
    for j in range(35):
        b2.check(j, 3, (4, 4))
    plan.set(lib.BatchPlan.descs(*b1.descs_args))
    # replays without a new set(): the kernel leaves its work queue reset, so
    # every replay recomputes every image (outputs poisoned in between)
    for rep in range(3):
        for h in b1.hist:
            h.fill_(7)
        for c in b1.codes:
            c.fill_(0xAB)
        plan.run()
        torch.cuda.synchronize()
        for j in range(20):
            assert torch.equal(first[j], b1.hist[j]), (rep, j)
        b1.check(0, 3, (4, 4))
        b1.check(19, 3, (4, 4))


def test_histograms_only_batch(lib):
    r = np.random.default_rng(12)
    b = Batch(r.integers(10, 150, 16), r.integers(10, 150, 16), synth.KIND_BLUR_RECTS, 3, (7, 6),
              with_codes=False)
    plan = _plan(lib, b, 3, (7, 6))
    plan.run()
    torch.cuda.synchronize()
    for j in range(16):
        b.check(j, 3, (7, 6), codes=False)


def test_per_image_path_matches_batched(lib):
    r = np.random.default_rng(13)
    Hs, Ws = r.integers(10, 500, 12), r.integers(10, 500, 12)
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 4, (7, 6))
    plan = _plan(lib, b, 3, (7, 6))
    plan.run_per_image()
    torch.cuda.synchronize()
    for j in range(12):
        b.check(j, 3, (7, 6))


def test_plan_rejects_bad_batches(lib):
    b = Batch([50, 2 + 5], [50, 60], synth.KIND_UNIFORM, 1, (7, 6))
    plan = lib.BatchPlan(4, 10 ** 6, 3, 7, 6)
    with pytest.raises(lib.LdpError):           # second image has fewer code rows than cells
        plan.set(lib.BatchPlan.descs(*b.descs_args))
    big = Batch([100] * 5, [100] * 5, synth.KIND_UNIFORM, 1, (7, 6))
    with pytest.raises(lib.LdpError):           # more images than the plan holds
        plan.set(lib.BatchPlan.descs(*big.descs_args))


# ------------------------------------------------------------ ldp_batch_launch

def _subset(lib, b, idx):
    return lib.BatchPlan.descs(*[[x[j] for j in idx] for x in b.descs_args])


def _poison(b):
    for c in b.codes:
        c.fill_(0xAB)
    for h in b.hist:
        h.fill_(7)


def test_launch_small_batches_in_arguments_and_larger_ones_loaded(lib):
    """One cell row per work item, 7 cell rows: 28 images are exactly the 196
    items the launch arguments hold; 29 images and more are loaded into the
    plan.  Launches interleave with runs of the loaded batch on one stream
    (the two share the plan's work queue); the loaded batch changes only when
    a launch loads one."""
    r = np.random.default_rng(70)
    n = 64
    cells = (7, 6)
    Hs, Ws = r.integers(9, 300, n), r.integers(8, 400, n)
    Hs[:2], Ws[:2] = [490, 9], [640, 500]
    b = Batch(Hs, Ws, synth.KIND_BLUR_SP_FLAT, 71, cells)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, 3, *cells,
                         tune=dict(block_threads=512, classes=[dict(cell_rows_per_item=1)]))
    loaded = list(range(40, 64))
    plan.set(_subset(lib, b, loaded))
    for idx in ([0], list(range(1, 6)), list(range(6, 34)), list(range(0, 29)), [7, 3],
                list(range(0, 40)), list(range(30, 58))):
        _poison(b)
        plan.launch(_subset(lib, b, idx))
        if len(idx) > 28:
            loaded = idx
        plan.run()
        torch.cuda.synchronize()
        for j in sorted(set(idx) | set(loaded)):
            b.check(j, 3, cells)
        assert plan.info()[0] == 7 * len(loaded), idx
    plan.launch(_subset(lib, b, []))  # nothing to do
    plan.close()


def test_launch_loads_batches_past_the_item_limit(lib):
    """16 cell rows, one per item: 12 images (192 items) go in the arguments,
    13 (208) are loaded."""
    r = np.random.default_rng(72)
    cells = (16, 6)
    Hs, Ws = r.integers(18, 260, 13), r.integers(8, 300, 13)
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 73, cells)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(13, pixels, 3, *cells, tune=dict(classes=[dict(cell_rows_per_item=1)]))
    plan.set(_subset(lib, b, [0]))
    _poison(b)
    plan.launch(_subset(lib, b, list(range(12))))
    torch.cuda.synchronize()
    for j in range(12):
        b.check(j, 3, cells)
    assert plan.info()[0] == 16
    _poison(b)
    plan.launch(_subset(lib, b, list(range(13))))
    torch.cuda.synchronize()
    for j in range(13):
        b.check(j, 3, cells)
    assert plan.info()[0] == 16 * 13
    plan.close()


def test_launch_on_flagged_and_window_plans_loads_the_batch(lib):
    from oracle import ldp as oracle_np
    r = np.random.default_rng(74)
    Hs, Ws = r.integers(12, 200, 5), r.integers(12, 300, 5)
    b = Batch(Hs, Ws, synth.KIND_BLUR_SP_FLAT, 75, (7, 6))
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(5, pixels, 3, 7, 6, flags=lib.LDP_RANK_MAGNITUDE)
    plan.launch(lib.BatchPlan.descs(*b.descs_args))
    torch.cuda.synchronize()
    assert plan.info()[0] == 5 * 7  # loaded: one cell row per item by default
    for j in range(5):
        wc, wh = oracle_c.ldp_extract(b.image(j), 3, 7, 6, magnitude=True)
        assert (b.codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (b.hist[j].cpu().numpy().view(np.uint32).reshape(wh.shape) == wh).all(), j
    plan.close()
    win = (40, 50)
    hists = [torch.full((-(-(int(h) - 2) // win[0]) * -(-(int(w) - 2) // win[1]) * 256,), 7,
                        dtype=torch.int32, device="cuda") for h, w in zip(Hs, Ws)]
    args = list(b.descs_args)
    args[2] = [h.data_ptr() for h in hists]
    plan = lib.BatchPlan(5, pixels, 3, *win, windows=True, max_width=300)
    plan.launch(lib.BatchPlan.descs(*args))
    torch.cuda.synchronize()
    assert plan.info()[0] > 0
    for j in range(5):
        wc = oracle_c.ldp_codes(b.image(j), 3)
        wh = oracle_np.window_histograms(wc, *win)
        assert (hists[j].cpu().numpy().view(np.uint32) == wh.ravel()).all(), j
    plan.close()


def test_launch_rejects_a_bad_image_and_launches_nothing(lib):
    r = np.random.default_rng(76)
    Hs, Ws = r.integers(20, 100, 4), r.integers(20, 100, 4)
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 77, (7, 6))
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(4, pixels, 3, 7, 6)
    args = [list(x) for x in b.descs_args]
    args[4][2] = 8  # 6 code rows: fewer than the 7 cell rows
    with pytest.raises(lib.LdpError):
        plan.launch(lib.BatchPlan.descs(*args))
    torch.cuda.synchronize()
    assert all((h == 7).all() for h in b.hist)
    assert plan.info()[0] == 0
    plan.close()


def test_plan_layout_histogram_copies(lib):
    """Plans take two LDS copies of the histograms only when the kernel keeps
    as many workgroups per CU with them: the 490x640 frames with 7x6 cells on
    256 threads and 2 cell rows per item (2 x 14 KB) do; 4 cell rows per item
    (2 x 28 KB would halve the workgroups) and window plans do not.  Only
    window plans of small windows store non-temporally."""
    Hs, Ws = [490] * 4, [640] * 4
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 11, (7, 6), row_align=4)
    row = (6 + 1) * 1024   # one cell row: 6 cells and the discard cell
    for cpi, copies in ((2, 2), (4, 1)):
        plan = _plan(lib, b, 3, (7, 6), dict(block_threads=256,
                                              classes=[dict(cell_rows_per_item=cpi)]))
        th, lds, cp, nt = plan.layout()
        # two copies: the second starts 64 bytes (16 banks) past the first's end
        slot = cpi * row + (64 if copies == 2 else 0)
        assert (th, cp, nt) == (256, copies, 0) and lds == copies * slot + 16, (cpi, th, lds, cp)
        plan.run()
        torch.cuda.synchronize()
        for j in range(len(Hs)):
            b.check(j, 3, (7, 6))
        plan.close()
    # window plans: one copy; non-temporal stores for windows of at most
    # 1024 pixels
    for (wy, wx), nt in (((20, 20), 1), ((32, 32), 1), ((33, 32), 0), ((50, 50), 0)):
        win = lib.BatchPlan(4, 4 * 490 * 640, 3, wy, wx, dict(block_threads=256), windows=True,
                            max_width=640)
        assert win.layout()[2:] == (1, nt), (wy, wx, win.layout())
        win.close()


def _stripes(H, W, period, seed):
    """Vertical stripes (columns cycling through `period` levels) with a few
    noisy rows: every lane of a wave sees the same short cycle of codes, so
    a wave's LDS adds land on the same few bins (the worst case for the
    histogram updates, and not the equal-codes fast path)."""
    r = np.random.default_rng(seed)
    levels = r.integers(0, 256, period).astype(np.uint8)
    img = np.broadcast_to(levels[np.arange(W) % period], (H, W)).copy()
    rows = r.integers(0, H, max(1, H // 50))
    img[rows] = r.integers(0, 256, (len(rows), W), dtype=np.uint8)
    return img


@pytest.mark.parametrize("k", [2, 3, 4])
def test_histogram_copies_under_same_bin_contention(lib, k):
    """One and two LDS copies of the histograms give the oracle's codes and
    histograms on images where every lane adds into the same few bins."""
    Hs, Ws = [490, 490, 333, 490], [640, 640, 517, 640]
    b = Batch(Hs, Ws, synth.KIND_BLUR_RECTS, 90 + k, (7, 6), row_align=4)
    for j, period in enumerate((2, 3, 2, 5)):
        b.image(j)[:, :] = _stripes(Hs[j], Ws[j], period, 100 * k + j)
    b.dev.copy_(torch.from_numpy(b.host))
    for cpi, copies in ((2, 2), (4, 1)):
        for h in b.hist:
            h.fill_(7)
        plan = _plan(lib, b, k, (7, 6), dict(block_threads=256,
                                              classes=[dict(cell_rows_per_item=cpi)]))
        assert plan.layout()[2] == copies
        plan.run()
        torch.cuda.synchronize()
        for j in range(len(Hs)):
            b.check(j, k, (7, 6))
        plan.close()
