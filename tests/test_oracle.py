"""Pins for the CPU oracle: checks it against facts the paper and mathematics fix.

None of these tests needs a GPU.  Each check is chosen so that a plausible slip
in the oracle (a wrong mask order, a flipped kernel, swapped rows and columns,
a dropped term, '>' for '>=', the k-th distinct value instead of the k-th order
statistic, absolute instead of signed responses) fails at least one of them.
"""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi

from _golden import closed_forms
from oracle import aldp, ldp

RING = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]  # E, NE, N, ... SE


def _rng(seed):
    return np.random.default_rng(seed)


def _rand_img(rng, H, W, lo=0, hi=256):
    return rng.integers(lo, hi, size=(H, W), dtype=np.uint8)


def _adversarial_images():
    out = [np.full((5, 7), 9, np.uint8), np.zeros((3, 3), np.uint8), np.full((4, 4), 255, np.uint8)]
    r = _rng(11)
    for _ in range(4):
        a = np.zeros((9, 10), np.uint8)
        a[r.integers(0, 9), r.integers(0, 10)] = 255
        out.append(a)
    step = np.zeros((8, 8), np.uint8)
    step[:, 4:] = 255
    out += [step, np.ascontiguousarray(step.T)]
    sp = r.integers(0, 2, size=(12, 13)).astype(np.uint8) * 255
    out.append(sp)
    out.append(_rand_img(r, 10, 12, 0, 3))          # tiny alphabet: many ties
    return out


# ---------------------------------------------------------------- masks (Fig. 1)

def test_masks_are_the_kirsch_compass_set():
    """Section 2.2.1: M0 is the Kirsch East mask; each next mask is the previous
    one with its outer ring turned by 45 degrees counter-clockwise."""
    east = np.array([[-3, -3, 5], [-3, 0, 5], [-3, -3, 5]])
    assert (ldp.KIRSCH[0] == east).all()
    ring_cells = [(1 + dx, 1 + dy) for dx, dy in RING]
    for i in range(1, 8):
        prev, cur = ldp.KIRSCH[i - 1], ldp.KIRSCH[i]
        assert cur[1, 1] == 0
        for p in range(8):
            # the weight at ring position p+1 of mask i is the weight at p of mask i-1
            assert cur[ring_cells[(p + 1) % 8]] == prev[ring_cells[p]]


def test_masks_zero_sum_and_quarter_turns():
    for i in range(8):
        assert ldp.KIRSCH[i].sum() == 0
        # numpy rot90 turns counter-clockwise: a quarter turn is two compass steps
        assert (np.rot90(ldp.KIRSCH[i]) == ldp.KIRSCH[(i + 2) % 8]).all()


def test_first_columns_of_m0_m1_m7_coincide():
    """Section 2.3 (Fig. 2): the first columns of M0, M1 and M7 are the same."""
    c = ldp.KIRSCH[:, :, 0]
    assert (c[0] == c[1]).all() and (c[0] == c[7]).all()


# ---------------------------------------------------------------- Eq. 1

def _effective_weights(fn):
    """3x3 weights of a linear response function, found with unit impulses."""
    w = None
    for a in range(3):
        for b in range(3):
            img = np.zeros((3, 3), np.uint8)
            img[a, b] = 1
            r = fn(img)[:, 0, 0]
            if w is None:
                w = np.zeros((len(r), 3, 3), dtype=np.int64)
            w[:, a, b] = r
    return w


def test_eq1_is_a_plain_correlation_library_check():
    """scipy.ndimage.correlate is the textbook correlation (no kernel flip)."""
    r = _rng(1)
    for H, W in [(3, 3), (5, 9), (17, 11), (32, 33)]:
        img = _rand_img(r, H, W)
        resp = ldp.responses_direct(img)
        for i in range(8):
            ref = ndi.correlate(img.astype(np.int64), ldp.KIRSCH[i], mode="constant", cval=0)
            assert (resp[i] == ref[1:-1, 1:-1]).all()


def test_responses_sum_to_zero_and_stay_in_range():
    r = _rng(2)
    img = _rand_img(r, 40, 37)
    resp = ldp.responses_direct(img)
    assert (resp.sum(axis=0) == 0).all()
    assert resp.max() <= 15 * 255 and resp.min() >= -15 * 255
    full = np.zeros((3, 3), np.uint8)
    full[:, 2] = 255
    assert ldp.responses_direct(full)[0, 0, 0] == 3825


# ---------------------------------------------------------------- Eqs. 7-29

def test_correctly_printed_terms_reproduce_m0_m1_m2():
    """Eqs. 22, 23 and 24 use only terms printed correctly (A0..A6)."""
    r = _rng(3)
    img = _rand_img(r, 19, 23)
    printed = aldp.responses_from_terms(aldp.column_terms_as_printed(img))
    direct = ldp.responses_direct(img)
    for i in (0, 1, 2):
        assert (printed[i] == direct[i]).all()


def test_misprinted_terms_do_not_give_kirsch_masks():
    """As printed, m3..m7 (Eqs. 25-29) are not zero-sum masks, so the four
    corrected terms are a necessary reading."""
    w = _effective_weights(lambda im: aldp.responses_from_terms(aldp.column_terms_as_printed(im)))
    assert [int(w[i].sum()) for i in range(3, 8)] == [-5, -8, -3, -3, -3]
    for i in (0, 1, 2):
        assert (w[i] == ldp.KIRSCH[i]).all()


def test_corrected_scheme_weights_are_the_masks():
    w = _effective_weights(aldp.responses_aldp)
    assert (w == ldp.KIRSCH).all()


def test_corrected_terms_are_the_fifteen_distinct_columns():
    # six distinct left, three middle and six right columns: the fifteen terms
    # Section 2.3.1 counts
    cols = {(j, tuple(ldp.KIRSCH[i][:, j])) for i in range(8) for j in range(3)}
    assert len(cols) == 15
    terms = _effective_weights(lambda im: np.stack(aldp.column_terms(im)))
    got = set()
    for t in terms:
        nz = [j for j in range(3) if t[:, j].any()]
        assert len(nz) == 1                    # every term is one column
        got.add((nz[0], tuple(t[:, nz[0]])))
    want = {(j, tuple(ldp.KIRSCH[i][:, j])) for i in range(8) for j in range(3)}
    assert got == want


def test_scheme_equals_direct_on_random_and_adversarial_images():
    r = _rng(4)
    imgs = [_rand_img(r, int(r.integers(3, 30)), int(r.integers(3, 30))) for _ in range(30)]
    imgs += _adversarial_images()
    for img in imgs:
        assert (aldp.responses_aldp(img) == ldp.responses_direct(img)).all()


# ---------------------------------------------------------------- Eqs. 2-3

def test_closed_forms_golden():
    for case in closed_forms():
        got = ldp.ldp_codes(case["image"], case["k"])
        assert (got == case["codes"]).all(), (case["name"], case["why"], got)


def test_closed_forms_golden_c_oracle(oracle_c):
    for case in closed_forms():
        got = oracle_c.ldp_codes(case["image"], case["k"])
        assert (got == case["codes"]).all(), case["name"]


def _code_by_rank(m, k):
    """Bit i set when fewer than k responses are strictly larger than m_i: an
    equivalent statement of 'm_i >= k-th largest' that needs no sort."""
    code = 0
    for i in range(8):
        larger = sum(1 for j in range(8) if m[j] > m[i])
        if larger < k:
            code |= 1 << i
    return code


def test_bruteforce_rank_definition_tiny_images():
    r = _rng(5)
    imgs = [_rand_img(r, int(r.integers(3, 9)), int(r.integers(3, 9))) for _ in range(12)]
    imgs += [_rand_img(r, 7, 8, 0, 4), np.full((4, 3), 3, np.uint8)]
    for img in imgs:
        H, W = img.shape
        for k in range(1, 9):
            codes = ldp.ldp_codes(img, k)
            for x, y in itertools.product(range(1, H - 1), range(1, W - 1)):
                m = [int(sum(int(ldp.KIRSCH[i, a, b]) * int(img[x + a - 1, y + b - 1])
                             for a in range(3) for b in range(3))) for i in range(8)]
                assert codes[x - 1, y - 1] == _code_by_rank(m, k)


def _rotl8(c, s):
    c = c.astype(np.int64)
    return (((c << s) | (c >> (8 - s))) & 255).astype(np.uint8)


def _permute_bits(c, f):
    c = c.astype(np.int64)
    out = np.zeros_like(c)
    for i in range(8):
        out |= ((c >> i) & 1) << f(i)
    return out.astype(np.uint8)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7])
def test_symmetries_move_bits_as_directions_move(k):
    """Turning the image a quarter turn counter-clockwise turns every
    direction by two compass steps; mirrors reflect the compass."""
    r = _rng(6)
    img = _rand_img(r, 13, 17)
    c = ldp.ldp_codes(img, k)
    assert (ldp.ldp_codes(np.rot90(img), k) == np.rot90(_rotl8(c, 2))).all()
    assert (ldp.ldp_codes(np.fliplr(img), k) == np.fliplr(_permute_bits(c, lambda i: (4 - i) % 8))).all()
    assert (ldp.ldp_codes(np.flipud(img), k) == np.flipud(_permute_bits(c, lambda i: (8 - i) % 8))).all()
    t = np.ascontiguousarray(img.T)
    assert (ldp.ldp_codes(t, k) == _permute_bits(c, lambda i: (6 - i) % 8).T).all()


def test_offset_and_scale_leave_codes_unchanged():
    """The masks sum to zero (offset drops out) and ranking is scale-free."""
    r = _rng(7)
    img = _rand_img(r, 15, 16, 0, 100)
    for k in (2, 3, 4):
        c = ldp.ldp_codes(img, k)
        assert (ldp.ldp_codes(img + np.uint8(120), k) == c).all()
        assert (ldp.ldp_codes(img * np.uint8(2), k) == c).all()


def test_signed_responses_inverting_the_image_changes_codes():
    """Inverting the image negates every response: with signed responses the
    codes change (absolute responses would leave them unchanged)."""
    r = _rng(8)
    img = _rand_img(r, 20, 20)
    assert (ldp.ldp_codes(255 - img, 3) != ldp.ldp_codes(img, 3)).mean() > 0.5


@pytest.mark.parametrize("k", range(1, 9))
def test_popcount_at_least_k_with_equality_iff_no_tie(k):
    r = _rng(9)
    img = _rand_img(r, 30, 31)
    resp = ldp.responses_direct(img)
    desc = -np.sort(-resp, axis=0)
    codes = ldp.ldp_codes(img, k)
    pc = np.unpackbits(codes[..., None], axis=-1).sum(-1)
    assert (pc >= k).all()
    if k < 8:
        no_tie = desc[k - 1] > desc[k]
        assert ((pc == k) == no_tie).all()
    else:
        assert (codes == 255).all()


def test_argument_checks():
    with pytest.raises(ValueError):
        ldp.ldp_codes(np.zeros((2, 5), np.uint8), 3)
    with pytest.raises(ValueError):
        ldp.ldp_codes(np.zeros((5, 5), np.uint8), 0)
    with pytest.raises(ValueError):
        ldp.ldp_codes(np.zeros((5, 5), np.uint8), 9)
    with pytest.raises(ValueError):
        ldp.ldp_histograms(np.zeros((5, 5), np.uint8), 6, 1)


# ---------------------------------------------------------------- Eqs. 4-5

def test_histograms_mass_cells_and_library_counts():
    r = _rng(10)
    img = _rand_img(r, 490, 640)
    codes = ldp.ldp_codes(img, 3)
    hist = ldp.ldp_histograms(codes, 7, 6)
    assert hist.shape == (7, 6, 256) and hist.dtype == np.uint32
    assert int(hist.sum()) == 488 * 638
    # floor partition sizes, counted independently of the oracle's formula
    rows = [sum(1 for rr in range(488) if rr * 7 // 488 == cy) for cy in range(7)]
    cols = [sum(1 for cc in range(638) if cc * 6 // 638 == cx) for cx in range(6)]
    assert rows == [70, 70, 70, 69, 70, 70, 69] and cols == [107, 106, 106, 107, 106, 106]
    r0 = np.cumsum([0] + rows)
    c0 = np.cumsum([0] + cols)
    for cy in range(7):
        for cx in range(6):
            block = codes[r0[cy]:r0[cy + 1], c0[cx]:c0[cx + 1]]
            ref, _ = np.histogram(block, bins=256, range=(0, 256))
            assert (hist[cy, cx] == ref).all()
            assert hist[cy, cx].sum() == rows[cy] * cols[cx]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_histogram_bins_below_k_bits_are_empty(k):
    r = _rng(12)
    img = _rand_img(r, 40, 50)
    hist = ldp.ldp_histograms(ldp.ldp_codes(img, k), 3, 4)
    for v in range(256):
        if bin(v).count("1") < k:
            assert hist[..., v].sum() == 0


def test_single_cell_and_one_cell_per_pixel():
    r = _rng(13)
    img = _rand_img(r, 9, 12)
    codes = ldp.ldp_codes(img, 3)
    h1 = ldp.ldp_histograms(codes, 1, 1)
    assert (h1[0, 0] == np.bincount(codes.ravel(), minlength=256)).all()
    hp = ldp.ldp_histograms(codes, 7, 10)
    for x in range(7):
        for y in range(10):
            assert hp[x, y].sum() == 1 and hp[x, y, codes[x, y]] == 1


# ---------------------------------------------------------------- C oracle

def test_c_oracle_equals_numpy_oracle(oracle_c):
    r = _rng(14)
    for t in range(25):
        H, W = int(r.integers(3, 45)), int(r.integers(3, 45))
        pitch = W + int(r.integers(0, 9))
        base = _rand_img(r, H, pitch)
        img = base[:, :W]                                  # strided rows
        k = int(r.integers(1, 9))
        c_np = ldp.ldp_codes(np.ascontiguousarray(img), k)
        c_c = oracle_c.ldp_codes(img, k)
        assert (c_np == c_c).all()
        cy, cx = int(r.integers(1, H - 1)), int(r.integers(1, W - 1))
        assert (ldp.ldp_histograms(c_np, cy, cx) == oracle_c.ldp_histograms(c_c, cy, cx)).all()
    for img in _adversarial_images():
        for k in (2, 3, 4):
            assert (ldp.ldp_codes(img, k) == oracle_c.ldp_codes(img, k)).all()


def test_c_oracle_argument_checks(oracle_c):
    with pytest.raises(ValueError):
        oracle_c.ldp_codes(np.zeros((2, 9), np.uint8), 3)
    with pytest.raises(ValueError):
        oracle_c.ldp_codes(np.zeros((9, 9), np.uint8), 9)
    with pytest.raises(ValueError):
        oracle_c.ldp_histograms(np.zeros((3, 3), np.uint8), 4, 1)


def test_c_oracle_batch_equals_numpy_oracle_per_image(oracle_c):
    """The threaded batch call computes every image as the numpy definition
    does (strided rows, images of different sizes, any thread count)."""
    r = _rng(15)
    Hs = r.integers(3, 40, size=23).astype(np.int32)
    Ws = r.integers(3, 40, size=23).astype(np.int32)
    strides = Ws.astype(np.int64) + r.integers(0, 7, size=23)
    off = np.concatenate([[0], np.cumsum(Hs * strides + 5)])[:-1]
    buf = _rand_img(r, 1, int(off[-1] + Hs[-1] * strides[-1] + 8))[0]
    for k, mag in ((3, False), (1, True), (8, False)):
        want_c, want_h = [], []
        for j in range(len(Hs)):
            img = buf[off[j]:off[j] + Hs[j] * strides[j]].reshape(Hs[j], strides[j])[:, :Ws[j]]
            c = ldp.ldp_codes(np.ascontiguousarray(img), k, magnitude=mag)
            want_c.append(c.reshape(-1))
            want_h.append(ldp.ldp_histograms(c, 1, 1))
        for threads in (1, 4):
            codes, coff, hist = oracle_c.ldp_extract_batch(buf, off, Hs, Ws, strides, k, 1, 1,
                                                           magnitude=mag, threads=threads)
            for j in range(len(Hs)):
                assert (codes[coff[j]:coff[j + 1]] == want_c[j]).all(), (k, threads, j)
                assert (hist[j] == want_h[j]).all(), (k, threads, j)
    with pytest.raises(ValueError):       # a 2-row image anywhere in the batch
        bad = Hs.copy()
        bad[5] = 2
        oracle_c.ldp_extract_batch(buf, off, bad, Ws, strides, 3, 1, 1)
