"""Parity of the variant paths through the C ABI with the CPU oracle,
bit-exact: ranking by response magnitude, Eq. 6 compact histograms, the
unaccelerated direct-mask route (same codes as Eq. 2) and LBP labels."""
import math

import numpy as np
import pytest

from conftest import gpu_available
from oracle import ldp as oracle_np
from oracle import native as oracle_c
from paper_1810_11518_amd import synth
from test_batch_gpu import Batch

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


def _imgs():
    r = np.random.default_rng(41)
    out = [r.integers(0, 256, (H, W), dtype=np.uint8)
           for H, W in [(3, 3), (3, 12), (5, 9), (9, 10), (17, 23), (64, 64), (100, 257), (48, 1024)]]
    out.append(synth.image(synth.KIND_BLUR_RECTS, 5, 1, 203, 317))
    out.append(synth.image(synth.KIND_BLUR_SP_FLAT, 6, 1, 300, 411))      # flat patches: ties
    out.append((r.integers(0, 3, (77, 91)) * 100).astype(np.uint8))
    inv = out[-2].copy()
    out.append(255 - inv)                                                   # negated responses
    return out


@pytest.mark.parametrize("k", range(1, 9))
def test_magnitude_codes_match_oracle(lib, k):
    for img in _imgs():
        got = lib.codes(_dev(img), k, flags=lib.LDP_RANK_MAGNITUDE).cpu().numpy()
        want = (oracle_np.ldp_codes(img, k, magnitude=True) if img.size < 20000
                else oracle_c.ldp_codes(img, k, magnitude=True))
        assert (got == want).all(), (img.shape, k)


def test_flags_zero_is_the_signed_path(lib):
    img = synth.image(synth.KIND_BLUR_RECTS, 7, 0, 130, 170)
    a = lib.codes(_dev(img), 3, flags=0).cpu().numpy()
    assert (a == oracle_c.ldp_codes(img, 3)).all()
    b = lib.codes(_dev(img), 3, flags=lib.LDP_RANK_MAGNITUDE).cpu().numpy()
    assert (a != b).any()  # the two rankings differ on real content


@pytest.mark.parametrize("cells", [(7, 6), (1, 1), (3, 63), (2, 80)])
def test_magnitude_extract_matches_oracle(lib, cells):
    """Fused path (cells_x <= 63, split cell rows) and the two-pass path."""
    for img in [synth.workload_image("single", 0), synth.image(synth.KIND_BLUR_SP_FLAT, 9, 2, 257, 333)]:
        c, h = lib.extract(_dev(img), 3, *cells, flags=lib.LDP_RANK_MAGNITUDE)
        wc, wh = oracle_c.ldp_extract(img, 3, *cells, magnitude=True)
        assert (c.cpu().numpy() == wc).all()
        assert (h.cpu().numpy().view(np.uint32) == wh).all()


@pytest.mark.parametrize("k", [1, 3, 6])
def test_magnitude_batch_plan_matches_oracle(lib, k):
    r = np.random.default_rng(50 + k)
    n = 40
    Hs, Ws = r.integers(9, 300, n), r.integers(3, 500, n)
    Hs[:2], Ws[:2] = [490, 12], [640, 700]
    cells = (7, 6)
    Ws = np.maximum(Ws, cells[1] + 2)
    b = Batch(Hs, Ws, synth.KIND_BLUR_SP_FLAT, 60 + k, cells)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    plan = lib.BatchPlan(n, pixels, k, cells[0], cells[1], flags=lib.LDP_RANK_MAGNITUDE)
    plan.set(lib.BatchPlan.descs(*b.descs_args))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        img = b.image(j)
        wc, wh = oracle_c.ldp_extract(img, k, *cells, magnitude=True)
        assert (b.codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (b.hist[j].cpu().numpy().view(np.uint32).reshape(wh.shape) == wh).all(), j
    # the per-image comparison path takes the same flags
    for h in b.hist:
        h.fill_(7)
    plan.run_per_image()
    torch.cuda.synchronize()
    for j in (0, 1, n - 1):
        _, wh = oracle_c.ldp_extract(b.image(j), k, *cells, magnitude=True)
        assert (b.hist[j].cpu().numpy().view(np.uint32).reshape(wh.shape) == wh).all(), j
    plan.close()


@pytest.mark.parametrize("k", range(1, 9))
def test_compact_histograms_match_oracle(lib, k):
    img = synth.image(synth.KIND_BLUR_SP_FLAT, 11, k, 301, 409)
    _, h = lib.extract(_dev(img), k, 9, 13, want_codes=False)
    got = lib.compact_histograms(h, k).cpu().numpy().view(np.uint32)
    want = oracle_np.compact_histograms(h.cpu().numpy().view(np.uint32), k)
    assert got.shape == (9, 13, math.comb(8, k) + 1)
    assert (got == want).all()
    assert (got.sum(-1) == h.cpu().numpy().view(np.uint32).sum(-1)).all()


def test_compact_histograms_many_cells_and_odd_counts(lib):
    """Random bins (not from codes), cell counts that are not a multiple of
    the four cells per workgroup, and more cells than the grid holds."""
    r = np.random.default_rng(77)
    for n in (1, 3, 5, 4099, 40001):
        h = r.integers(0, 1 << 20, (n, 256)).astype(np.int32)
        got = lib.compact_histograms(_dev(h), 3).cpu().numpy().view(np.uint32)
        assert (got == oracle_np.compact_histograms(h.view(np.uint32), 3)).all(), n


# ------------------------------------------------------------ direct masks, LBP

@pytest.mark.parametrize("k", range(1, 9))
def test_direct_masks_give_the_signed_codes(lib, k):
    """The unaccelerated route (each response its own 8-tap correlation) must
    give exactly the codes of Eq. 2 as the oracle computes them."""
    for img in _imgs():
        got = lib.codes(_dev(img), k, flags=lib.LDP_DIRECT_MASKS).cpu().numpy()
        want = oracle_np.ldp_codes(img, k) if img.size < 20000 else oracle_c.ldp_codes(img, k)
        assert (got == want).all(), (img.shape, k)


def test_lbp_codes_match_oracle(lib):
    from oracle import lbp as oracle_lbp
    imgs = _imgs() + [np.full((40, 37), 77, np.uint8)]
    for img in imgs:
        for k in (1, 3, 8):  # k is ignored for LBP
            got = lib.codes(_dev(img), k, flags=lib.LDP_CODE_LBP).cpu().numpy()
            assert (got == oracle_lbp.lbp_codes(img)).all(), (img.shape, k)


@pytest.mark.parametrize("cells", [(7, 6), (4, 70)])
@pytest.mark.parametrize("mode", ["lbp", "direct"])
def test_lbp_and_direct_extract_match_oracle(lib, cells, mode):
    from oracle import lbp as oracle_lbp
    for img in [synth.workload_image("single", 0), synth.image(synth.KIND_BLUR_SP_FLAT, 3, 4, 211, 290)]:
        if mode == "lbp":
            wc = oracle_lbp.lbp_codes(img)
            flags = lib.LDP_CODE_LBP
        else:
            wc = oracle_c.ldp_codes(img, 3)
            flags = lib.LDP_DIRECT_MASKS
        wh = oracle_np.ldp_histograms(wc, *cells)
        c, h = lib.extract(_dev(img), 3, *cells, flags=flags)
        assert (c.cpu().numpy() == wc).all()
        assert (h.cpu().numpy().view(np.uint32) == wh).all()


@pytest.mark.parametrize("mode", ["lbp", "direct"])
def test_lbp_and_direct_batch_plans_match_oracle(lib, mode):
    from oracle import lbp as oracle_lbp
    r = np.random.default_rng(88)
    n = 30
    cells = (7, 6)
    Hs, Ws = r.integers(9, 260, n), r.integers(8, 420, n)
    Ws[:2] = [640, 9]
    b = Batch(Hs, Ws, synth.KIND_BLUR_SP_FLAT, 89, cells)
    pixels = int((b.Hs.astype(np.int64) * b.Ws).sum())
    flags = lib.LDP_CODE_LBP if mode == "lbp" else lib.LDP_DIRECT_MASKS
    plan = lib.BatchPlan(n, pixels, 3, cells[0], cells[1], flags=flags)
    plan.set(lib.BatchPlan.descs(*b.descs_args))
    plan.run()
    torch.cuda.synchronize()
    for j in range(n):
        img = b.image(j)
        wc = oracle_lbp.lbp_codes(img) if mode == "lbp" else oracle_c.ldp_codes(img, 3)
        wh = oracle_np.ldp_histograms(wc, *cells)
        assert (b.codes[j].cpu().numpy().reshape(wc.shape) == wc).all(), j
        assert (b.hist[j].cpu().numpy().view(np.uint32).reshape(wh.shape) == wh).all(), j
    plan.close()
