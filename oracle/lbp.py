"""Plain numpy oracle for Local Binary Pattern (LBP) codes.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

Section 2.1: every pixel is labelled by thresholding its 3x3 neighbourhood at
the centre value and reading the results as a binary number; a 256-bin
histogram of the labels describes a region.  Readings (the paper gives no
neighbour order, threshold rule or border rule):

* bit i belongs to the neighbour in compass direction i, in the order the
  Kirsch masks use (East, North-East, North, North-West, West, South-West,
  South, South-East), with x the row and y the column;
* bit i is set when the neighbour is >= the centre (ties set the bit);
* only interior pixels get a label: the label map is (H-2) x (W-2), and its
  histograms use the same cells as the LDP code map.
"""
import numpy as np

# (row offset, column offset) of the neighbour in direction i
RING = ((0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1))


def lbp_codes(img):
    """Interior LBP label map, uint8 array of shape (H-2, W-2)."""
    a = np.asarray(img)
    if a.ndim != 2 or a.dtype != np.uint8 or a.shape[0] < 3 or a.shape[1] < 3:
        raise ValueError("image must be a 2-D uint8 array of at least 3x3")
    a = a.astype(np.int64)
    H, W = a.shape
    centre = a[1:H - 1, 1:W - 1]
    code = np.zeros(centre.shape, dtype=np.int64)
    for i, (dx, dy) in enumerate(RING):
        neighbour = a[1 + dx:H - 1 + dx, 1 + dy:W - 1 + dy]
        code += (neighbour >= centre).astype(np.int64) << i
    return code.astype(np.uint8)
