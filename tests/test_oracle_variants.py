"""Pins of the oracle's variants (no GPU): ranking by response magnitude, and
Eq. 6's compact histogram of the C(8, k) pattern values plus a tie bin.

Each check rests on something other than the oracle's own code: closed forms
worked out by hand from the masks, a sort-free rank count, the symmetry that
inverting the image negates every response, counting identities, and the bin
count Eq. 6 prints for k = 3."""
import itertools
import math

import numpy as np
import pytest

from oracle import ldp

RING = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]  # E, NE, N, ... SE


def _rng(seed):
    return np.random.default_rng(seed)


def _rotl8(c, s):
    return ((c << s) | (c >> (8 - s))) & 255


def _code_by_rank(m, k):
    """Bit i set when fewer than k values are strictly larger than m_i."""
    return sum(1 << i for i in range(8) if sum(1 for j in range(8) if m[j] > m[i]) < k)


# ------------------------------------------------------------ magnitude ranking

def test_magnitude_codes_ignore_inverting_the_image():
    """255 - I negates every response (the masks sum to zero), so ranking by
    |m_i| gives the same codes, for every k."""
    r = _rng(21)
    img = r.integers(0, 256, (23, 29), dtype=np.uint8)
    for k in range(1, 9):
        assert (ldp.ldp_codes(255 - img, k, magnitude=True) ==
                ldp.ldp_codes(img, k, magnitude=True)).all()


@pytest.mark.parametrize("j", range(8))
def test_magnitude_closed_form_one_dark_neighbour(j):
    """Centre pixel whose eight neighbours are v except neighbour j, which is
    0.  Mask i weighs its three ring neighbours around direction i with +5 and
    the other five with -3, so m_i = 5*(sum of its three) - 3*(the other five).
    For the three masks i with j among their +5 neighbours: 5*2v - 3*5v = -5v;
    for the other five: 5*3v - 3*4v = +3v.  By magnitude the top three are
    directions j-1, j, j+1: code rotl8(131, j) for k = 3.  By signed value the
    five +3v responses tie for the top: code 255 - rotl8(131, j)."""
    v = 40
    img = np.full((3, 3), v, np.uint8)
    img[1, 1] = 200  # the centre does not enter any mask
    dx, dy = RING[j]
    img[1 + dx, 1 + dy] = 0
    assert ldp.ldp_codes(img, 3, magnitude=True)[0, 0] == _rotl8(131, j)
    assert ldp.ldp_codes(img, 3)[0, 0] == 255 - _rotl8(131, j)
    # k = 4: by magnitude the 4th largest is 3v, tied five ways: all bits set
    assert ldp.ldp_codes(img, 4, magnitude=True)[0, 0] == 255


def test_magnitude_rank_bruteforce_tiny_images():
    """Bit i of the magnitude code is set exactly when fewer than k of the
    |m_j| (from hand-written mask sums) are strictly larger than |m_i|."""
    r = _rng(22)
    imgs = [r.integers(0, 256, (int(r.integers(3, 8)), int(r.integers(3, 8))), dtype=np.uint8)
            for _ in range(10)]
    imgs.append(r.integers(0, 3, (6, 7), dtype=np.uint8))  # many ties
    for img in imgs:
        H, W = img.shape
        for k in range(1, 9):
            codes = ldp.ldp_codes(img, k, magnitude=True)
            for x, y in itertools.product(range(1, H - 1), range(1, W - 1)):
                m = []
                for i in range(8):
                    acc = 0
                    for a in range(3):
                        for b in range(3):
                            acc += int(ldp.KIRSCH[i, a, b]) * int(img[x + a - 1, y + b - 1])
                    m.append(abs(acc))
                assert codes[x - 1, y - 1] == _code_by_rank(m, k)


def test_magnitude_popcount_law():
    r = _rng(23)
    img = r.integers(0, 256, (31, 30), dtype=np.uint8)
    mag = np.abs(ldp.responses_direct(img))
    desc = -np.sort(-mag, axis=0)
    for k in range(1, 8):
        pc = np.unpackbits(ldp.ldp_codes(img, k, magnitude=True)[..., None], axis=-1).sum(-1)
        assert (pc >= k).all()
        assert ((pc == k) == (desc[k - 1] > desc[k])).all()


def test_magnitude_quarter_turn_rotates_bits():
    r = _rng(24)
    img = r.integers(0, 256, (14, 19), dtype=np.uint8)
    c = ldp.ldp_codes(img, 3, magnitude=True).astype(np.int64)
    turned = ldp.ldp_codes(np.rot90(img), 3, magnitude=True)
    assert (turned == np.rot90(_rotl8(c, 2))).all()


def test_magnitude_c_oracle_equals_numpy(oracle_c):
    r = _rng(25)
    for _ in range(12):
        H, W = int(r.integers(3, 40)), int(r.integers(3, 40))
        img = r.integers(0, 256, (H, W + 3), dtype=np.uint8)[:, :W]
        k = int(r.integers(1, 9))
        assert (oracle_c.ldp_codes(img, k, magnitude=True) ==
                ldp.ldp_codes(np.ascontiguousarray(img), k, magnitude=True)).all()


# ------------------------------------------------------------ compact histograms

def test_eq6_has_56_bins_for_k3_and_binomial_counts():
    assert len(ldp.pattern_values(3)) == 56  # Eq. 6 lists H_1 .. H_56
    for k in range(1, 9):
        pv = ldp.pattern_values(k)
        assert len(pv) == math.comb(8, k)
        assert (np.diff(pv) > 0).all()


def test_compact_bin_positions_closed_forms():
    """Positions counted by hand for k = 3: 7 = 0b111 is the smallest 3-bit
    code (bin 0); 224 = 0b11100000 the largest (bin 55); 131 = 0b10000011 has
    C(7,3) = 35 three-bit codes below it (all below 128) and none between 128
    and 131 (bin 35); 255 (a tie code) goes to the last bin, 56."""
    h = np.zeros(256, np.uint32)
    h[7], h[224], h[131], h[255], h[0] = 1, 2, 3, 4, 5
    c = ldp.compact_histograms(h, 3)
    assert c.shape == (57,)
    assert c[0] == 1 and c[55] == 2 and c[35] == 3 and c[56] == 4 + 5
    assert c.sum() == h.sum()


def test_compact_histograms_keep_mass_and_the_k_bit_counts():
    r = _rng(26)
    img = r.integers(0, 4, (40, 37), dtype=np.uint8)  # small range: many ties
    for k in (1, 2, 3, 5):
        codes = ldp.ldp_codes(img, k)
        hist = ldp.ldp_histograms(codes, 3, 4)
        comp = ldp.compact_histograms(hist, k)
        assert comp.shape == (3, 4, math.comb(8, k) + 1)
        assert (comp.sum(-1) == hist.sum(-1)).all()
        pc = np.unpackbits(np.arange(256, dtype=np.uint8)[:, None], axis=1).sum(1)
        # pixels with exactly k bits land in the pattern bins, the rest in the last
        assert (comp[..., :-1].sum(-1) == hist[..., pc == k].sum(-1)).all()
        assert comp[..., -1].sum() == (np.unpackbits(codes[..., None], -1).sum(-1) != k).sum()
