"""Plain numpy oracle for Local Directional Pattern (LDP) codes and histograms.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

Everything here is the method's definition written out with no reuse of
partial sums, no blocking and no reordering, so that it can be checked against
the paper by eye.  Integer arithmetic is exact; there is no rounding anywhere.

Conventions (readings of the paper; each is listed with its justification in
the design notes of the repository):

* Image ``I`` has H rows and W columns; pixel ``(x, y)`` is row x, column y
  (Section 2.3 indexes the image as I_ij with i the row, and calls A0 a
  "column" term built from I(x-1, y-1), I(x, y-1), I(x+1, y-1)).
* The eight masks are the Kirsch compass masks (Section 2.2.1, Fig. 1), in the
  order East, North-East, North, North-West, West, South-West, South,
  South-East for M0..M7.  This is the only order consistent with the correctly
  printed Eqs. 22-24 and 26 and with the remark in Section 2.3 that the first
  columns of M0, M1 and M7 coincide.
* Eq. 1 is a correlation (no kernel flip): m_i = sum_{a,b in {-1,0,1}}
  M_i[a+1][b+1] * I[x+a][y+b].
* Responses are signed, as Eq. 2 is written (no absolute value).  The
  magnitude option ranks |m_i| instead: the convention of the original LDP
  descriptor that Section 2.2 builds on, offered as a variant.
* m_k is the k-th element of the eight responses sorted in descending order,
  duplicates kept (an order statistic).
* Eq. 3 sets bit i when m_i - m_k >= 0, so every response tied with m_k sets
  its bit; ties can set more than k bits.
* Bit i of the code belongs to response m_i (Section 2.2.1 lists the response
  vector as (m7, ..., m0)).
* Only interior pixels (1 <= x <= H-2, 1 <= y <= W-2) have a full 3x3
  neighbourhood and get a code; the code map is (H-2) x (W-2).
* Histograms (Eqs. 4-5) count raw 8-bit codes in 256 bins per cell of a
  cells_y x cells_x grid laid over the code map with a floor partition:
  code row r belongs to cell row floor(r * cells_y / (H-2)), code column c to
  cell column floor(c * cells_x / (W-2)).
"""
import numpy as np

# Kirsch compass masks, rows (x-1, x, x+1) top to bottom, columns
# (y-1, y, y+1) left to right.  Section 2.2.1, Fig. 1 (figure not reproduced in
# the text; the values are the standard Kirsch set named there).
KIRSCH = np.array(
    [
        # M0, East
        [[-3, -3, 5],
         [-3, 0, 5],
         [-3, -3, 5]],
        # M1, North-East
        [[-3, 5, 5],
         [-3, 0, 5],
         [-3, -3, -3]],
        # M2, North
        [[5, 5, 5],
         [-3, 0, -3],
         [-3, -3, -3]],
        # M3, North-West
        [[5, 5, -3],
         [5, 0, -3],
         [-3, -3, -3]],
        # M4, West
        [[5, -3, -3],
         [5, 0, -3],
         [5, -3, -3]],
        # M5, South-West
        [[-3, -3, -3],
         [5, 0, -3],
         [5, 5, -3]],
        # M6, South
        [[-3, -3, -3],
         [-3, 0, -3],
         [5, 5, 5]],
        # M7, South-East
        [[-3, -3, -3],
         [-3, 0, 5],
         [-3, 5, 5]],
    ],
    dtype=np.int64,
)

NUM_BINS = 256


def _as_image(img):
    a = np.asarray(img)
    if a.ndim != 2:
        raise ValueError("image must be 2-D (rows, columns)")
    if a.dtype != np.uint8:
        raise ValueError("image must be uint8")
    if a.shape[0] < 3 or a.shape[1] < 3:
        raise ValueError("image must have at least 3 rows and 3 columns")
    return a


def responses_direct(img):
    """Eight Kirsch responses of every interior pixel by direct correlation.

    Eq. 1 (Section 2.2.1): m_i(x, y) = sum_{a=-1..1} sum_{b=-1..1}
    M_i[a+1][b+1] * I(x+a, y+b), for every interior pixel.

    Returns int64 array of shape (8, H-2, W-2); element [i, x-1, y-1] is m_i at
    pixel (x, y).
    """
    a = _as_image(img).astype(np.int64)
    H, W = a.shape
    out = np.zeros((8, H - 2, W - 2), dtype=np.int64)
    for i in range(8):
        for da in range(3):
            for db in range(3):
                # I(x + da - 1, y + db - 1) for x in 1..H-2, y in 1..W-2
                out[i] += KIRSCH[i, da, db] * a[da:da + H - 2, db:db + W - 2]
    return out


def kth_largest(resp, k):
    """The k-th most outstanding response m_k (Section 2.2.2, Eq. 2).

    The k-th element of the eight responses sorted in descending order, with
    duplicates kept.  ``resp`` has the eight responses on axis 0.
    """
    if not 1 <= k <= 8:
        raise ValueError("k must be in 1..8")
    desc = -np.sort(-resp, axis=0)
    return desc[k - 1]


def codes_from_responses(resp, k):
    """LDP code of Eq. 2 with the step function of Eq. 3.

    code = sum_{i=0..7} s(m_i - m_k) * 2^i, with s(v) = 1 if v >= 0 else 0.
    """
    mk = kth_largest(resp, k)
    code = np.zeros(resp.shape[1:], dtype=np.int64)
    for i in range(8):
        code += (resp[i] - mk >= 0).astype(np.int64) << i
    return code.astype(np.uint8)


def ldp_codes(img, k=3, magnitude=False):
    """Interior LDP code map, uint8 array of shape (H-2, W-2).

    Eqs. 1-3 (Sections 2.2.1-2.2.2) applied to every interior pixel.  With
    ``magnitude`` the responses are ranked by absolute value: Eqs. 2-3 applied
    to |m_0|, ..., |m_7|.
    """
    resp = responses_direct(img)
    if magnitude:
        resp = np.abs(resp)
    return codes_from_responses(resp, k)


def cell_of(n, cells, idx):
    """Cell index of code row (or column) ``idx`` in a floor partition of
    ``n`` rows (columns) into ``cells`` cells."""
    return (idx * cells) // n


def ldp_histograms(codes, cells_y, cells_x):
    """Per-cell 256-bin histograms of a code map (Section 2.2.3, Eqs. 4-5).

    H_c[v] = number of code pixels of cell c whose code equals v.  Returns a
    uint32 array of shape (cells_y, cells_x, 256).
    """
    c = np.asarray(codes)
    if c.ndim != 2 or c.dtype != np.uint8:
        raise ValueError("codes must be a 2-D uint8 array")
    hc, wc = c.shape
    if not (1 <= cells_y <= hc and 1 <= cells_x <= wc):
        raise ValueError("cell grid must have 1..rows by 1..columns cells")
    hist = np.zeros((cells_y, cells_x, NUM_BINS), dtype=np.int64)
    cy = cell_of(hc, cells_y, np.arange(hc))
    cx = cell_of(wc, cells_x, np.arange(wc))
    for r in range(hc):
        for j in range(cells_x):
            sel = c[r, cx == j]
            hist[cy[r], j] += np.bincount(sel, minlength=NUM_BINS)
    return hist.astype(np.uint32)


def ldp_extract(img, k, cells_y, cells_x, magnitude=False):
    """Codes and per-cell histograms of one image (Eqs. 1-5)."""
    codes = ldp_codes(img, k, magnitude)
    return codes, ldp_histograms(codes, cells_y, cells_x)


def pattern_values(k):
    """Eq. 4's pattern values C_1, C_2, ...: the codes with exactly k bits set,
    in ascending order (C(8, k) of them; Eq. 6 lists 56 bins for k = 3)."""
    if not 1 <= k <= 8:
        raise ValueError("k must be in 1..8")
    return np.array([v for v in range(NUM_BINS) if bin(v).count("1") == k], dtype=np.int64)


def compact_histograms(hist, k):
    """Eq. 6's feature vector for every cell of ``hist`` (raw-code bins on the
    last axis): H_i of Eq. 4 for each pattern value C_i of pattern_values(k),
    followed by one bin counting the pixels whose code is no pattern value
    (a tie with m_k sets more than k bits).  Returns uint32, last axis
    C(8, k) + 1."""
    h = np.asarray(hist).astype(np.int64)
    if h.shape[-1] != NUM_BINS:
        raise ValueError("histograms must have 256 bins on the last axis")
    C = pattern_values(k)
    out = np.zeros(h.shape[:-1] + (len(C) + 1,), dtype=np.int64)
    for i, c in enumerate(C):
        out[..., i] = h[..., c]
    others = [v for v in range(NUM_BINS) if v not in set(C.tolist())]
    out[..., len(C)] = h[..., others].sum(axis=-1)
    return out.astype(np.uint32)


def window_counts(n, w):
    """Windows of w code rows (columns) over n: ceil(n / w), the last one
    partial when w does not divide n."""
    return -(-n // w)


def window_histograms(codes, win_y, win_x):
    """256-bin histograms per window of a code map (Section 3.2's windows):
    non-overlapping win_y x win_x windows tiling the code map from its first
    row and column; window (wy, wx) counts code rows wy*win_y .. and columns
    wx*win_x .., cut at the map's edge.  Returns uint32 of shape
    (ceil(rows / win_y), ceil(columns / win_x), 256)."""
    c = np.asarray(codes)
    if c.ndim != 2 or c.dtype != np.uint8:
        raise ValueError("codes must be a 2-D uint8 array")
    if win_y < 1 or win_x < 1:
        raise ValueError("window sides must be >= 1")
    hc, wc = c.shape
    ny, nx = window_counts(hc, win_y), window_counts(wc, win_x)
    hist = np.zeros((ny, nx, NUM_BINS), dtype=np.int64)
    for a in range(ny):
        for b in range(nx):
            block = c[a * win_y:(a + 1) * win_y, b * win_x:(b + 1) * win_x]
            hist[a, b] = np.bincount(block.ravel(), minlength=NUM_BINS)
    return hist.astype(np.uint32)

