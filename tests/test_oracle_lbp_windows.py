"""Pins of the LBP oracle and of window histograms (no GPU).

LBP: closed forms, a brute-force loop, invariance under strictly increasing
grey-level maps, the complement law, quarter turns.  Windows: the window
counts the paper prints in Table 3, per-window areas, and agreement with the
cell partition where the two coincide."""
import itertools

import numpy as np
import pytest

from oracle import lbp, ldp


def _rotl8(c, s):
    c = np.asarray(c).astype(np.int64)
    return (((c << s) | (c >> (8 - s))) & 255).astype(np.uint8)


# ------------------------------------------------------------------ LBP

def test_lbp_closed_forms():
    flat = np.full((4, 5), 9, np.uint8)
    assert (lbp.lbp_codes(flat) == 255).all()          # every neighbour ties with the centre
    peak = np.full((3, 3), 10, np.uint8)
    peak[1, 1] = 11
    assert lbp.lbp_codes(peak)[0, 0] == 0              # a strict maximum sets no bit
    for j, (dx, dy) in enumerate(lbp.RING):
        img = np.full((3, 3), 10, np.uint8)
        img[1, 1] = 50
        img[1 + dx, 1 + dy] = 50                        # only neighbour j reaches the centre
        assert lbp.lbp_codes(img)[0, 0] == 1 << j


def test_lbp_ring_directions_are_the_kirsch_order():
    """Direction i of the LBP ring is the neighbour that Kirsch mask i centres
    its three +5 weights on (E, NE, N, ... SE)."""
    for i, (dx, dy) in enumerate(lbp.RING):
        m = ldp.KIRSCH[i]
        assert m[1 + dx, 1 + dy] == 5
        assert m[1 - dx, 1 - dy] == -3


def test_lbp_bruteforce_tiny_images():
    r = np.random.default_rng(31)
    for _ in range(10):
        H, W = int(r.integers(3, 8)), int(r.integers(3, 8))
        img = r.integers(0, 4, (H, W), dtype=np.uint8)
        codes = lbp.lbp_codes(img)
        for x, y in itertools.product(range(1, H - 1), range(1, W - 1)):
            want = 0
            for i, (dx, dy) in enumerate(lbp.RING):
                if int(img[x + dx, y + dy]) >= int(img[x, y]):
                    want |= 1 << i
            assert codes[x - 1, y - 1] == want


def test_lbp_invariant_under_increasing_grey_maps():
    r = np.random.default_rng(32)
    img = r.integers(0, 127, (21, 26), dtype=np.uint8)
    mapped = (2 * img.astype(np.int64) + img % 2 + 1).astype(np.uint8)  # strictly increasing, <= 253
    assert (lbp.lbp_codes(mapped) == lbp.lbp_codes(img)).all()


def test_lbp_complement_law():
    """In 255 - I every comparison reverses, ties stay ties: the two codes
    together cover every bit, and they share exactly the tied bits."""
    r = np.random.default_rng(33)
    img = r.integers(0, 6, (19, 23), dtype=np.uint8)
    a, b = lbp.lbp_codes(img), lbp.lbp_codes(255 - img)
    assert ((a | b) == 255).all()
    ties = np.zeros(a.shape, np.int64)
    H, W = img.shape
    for i, (dx, dy) in enumerate(lbp.RING):
        ties |= (img[1 + dx:H - 1 + dx, 1 + dy:W - 1 + dy] == img[1:H - 1, 1:W - 1]).astype(np.int64) << i
    assert ((a & b) == ties).all()


def test_lbp_quarter_turn():
    r = np.random.default_rng(34)
    img = r.integers(0, 256, (13, 18), dtype=np.uint8)
    assert (lbp.lbp_codes(np.rot90(img)) == np.rot90(_rotl8(lbp.lbp_codes(img), 2))).all()


# ------------------------------------------------------------------ windows

def test_window_counts_of_table3():
    """Table 3: a 280x280 image (a 278x278 code map) gives 784, 196, 144, 36
    and 9 windows for windows of 10, 20, 25, 50 and 100 pixels."""
    codes = np.zeros((278, 278), np.uint8)
    for w, n in ((10, 784), (20, 196), (25, 144), (50, 36), (100, 9)):
        h = ldp.window_histograms(codes, w, w)
        assert h.shape[0] * h.shape[1] == n


def test_window_areas_and_mass():
    r = np.random.default_rng(35)
    codes = r.integers(0, 256, (47, 61), dtype=np.uint8)
    h = ldp.window_histograms(codes, 10, 25)
    assert h.shape == (5, 3, 256)
    rows = [10, 10, 10, 10, 7]
    cols = [25, 25, 11]
    for a, b in itertools.product(range(5), range(3)):
        assert h[a, b].sum() == rows[a] * cols[b]


def test_windows_equal_cells_when_the_side_divides():
    """w | n: floor(r / w) = floor(r * (n / w) / n), so windows are the cells
    of an (n / w)-cell partition."""
    r = np.random.default_rng(36)
    codes = r.integers(0, 256, (40, 60), dtype=np.uint8)
    assert (ldp.window_histograms(codes, 10, 20) == ldp.ldp_histograms(codes, 4, 3)).all()


def test_window_extremes():
    r = np.random.default_rng(37)
    codes = r.integers(0, 256, (9, 11), dtype=np.uint8)
    whole = ldp.window_histograms(codes, 100, 100)
    assert whole.shape == (1, 1, 256)
    assert (whole[0, 0] == np.bincount(codes.ravel(), minlength=256)).all()
    one = ldp.window_histograms(codes, 1, 1)
    assert one.shape == (9, 11, 256)
    assert (one.sum(-1) == 1).all()
    assert (one.argmax(-1) == codes).all()
    with pytest.raises(ValueError):
        ldp.window_histograms(codes, 0, 3)
