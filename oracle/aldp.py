"""The paper's acceleration scheme (ALDP), Section 2.3, as a CPU reference.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

Section 2.3.1 replaces the eight 3x3 mask products by fifteen partial column
terms A0..A14 (Eqs. 7-21), each the product of one distinct Kirsch mask
column with one image column; Section 2.3.2 adds three of them per response
(Eqs. 22-29).  Four of the printed column terms cannot be columns of any
Kirsch mask and make m3..m7 fail to be Kirsch responses (their weights do not
even sum to zero):

* Eq. 14 (A7) omits I(x, y-1); the column used by m3 is (5, 5, -3).
* Eq. 16 (A9) prints (5, 5, -3); the column used by m4 is (5, 5, 5).
* Eq. 18 (A11) prints -3(I(x-1,y) + I(x,y)) + 5 I(x+1,y-1); the column used by
  m5, m6 and m7 is the middle column (-3, 0, 5).
* Eq. 19 (A12) takes its +5 from I(x+1, y+1); the column used by m6 is the
  left column (-3, -3, 5).

``column_terms`` implements the corrected set: the fifteen distinct columns of
the eight masks (six left, three middle, six right), which is exactly the
count the paper states.  ``column_terms_as_printed`` keeps the printed forms
so a test can show that they do not reproduce the masks.

Coordinates: x is the row, y the column, as in the rest of the oracle.
"""
import numpy as np


def _shifts(img):
    """Return a function J(da, db) giving I(x+da, y+db) over all interior
    pixels (x, y) as an int64 array of shape (H-2, W-2)."""
    a = np.asarray(img)
    if a.ndim != 2 or a.dtype != np.uint8 or a.shape[0] < 3 or a.shape[1] < 3:
        raise ValueError("image must be a 2-D uint8 array of at least 3x3")
    a = a.astype(np.int64)
    H, W = a.shape

    def J(da, db):
        return a[1 + da:H - 1 + da, 1 + db:W - 1 + db]

    return J


def column_terms(img):
    """Corrected column terms A0..A14 (Section 2.3.1, Eqs. 7-21)."""
    J = _shifts(img)
    A = [None] * 15
    A[0] = -3 * (J(-1, -1) + J(0, -1) + J(1, -1))          # Eq. 7
    A[1] = -3 * (J(-1, 0) + J(1, 0))                       # Eq. 8
    A[2] = 5 * (J(-1, 1) + J(0, 1) + J(1, 1))              # Eq. 9
    A[3] = 5 * J(-1, 0) - 3 * J(1, 0)                      # Eq. 10
    A[4] = 5 * (J(-1, 1) + J(0, 1)) + (-3 * J(1, 1))       # Eq. 11
    A[5] = 5 * J(-1, -1) + (-3 * (J(0, -1) + J(1, -1)))    # Eq. 12
    A[6] = 5 * J(-1, 1) + (-3 * (J(0, 1) + J(1, 1)))       # Eq. 13
    A[7] = 5 * (J(-1, -1) + J(0, -1)) + (-3 * J(1, -1))    # Eq. 14, corrected
    A[8] = -3 * (J(-1, 1) + J(0, 1) + J(1, 1))             # Eq. 15
    A[9] = 5 * (J(-1, -1) + J(0, -1) + J(1, -1))           # Eq. 16, corrected
    A[10] = -3 * J(-1, -1) + 5 * (J(0, -1) + J(1, -1))     # Eq. 17
    A[11] = -3 * J(-1, 0) + 5 * J(1, 0)                    # Eq. 18, corrected
    A[12] = -3 * (J(-1, -1) + J(0, -1)) + 5 * J(1, -1)     # Eq. 19, corrected
    A[13] = -3 * (J(-1, 1) + J(0, 1)) + 5 * J(1, 1)        # Eq. 20
    A[14] = -3 * J(-1, 1) + 5 * (J(0, 1) + J(1, 1))        # Eq. 21
    return A


def column_terms_as_printed(img):
    """Column terms exactly as Eqs. 7-21 print them (four are misprints)."""
    J = _shifts(img)
    A = column_terms(img)
    A = list(A)
    A[7] = 5 * J(-1, -1) + (-3 * J(1, -1))                 # Eq. 14 as printed
    A[9] = 5 * (J(-1, -1) + J(0, -1)) + (-3 * J(1, -1))    # Eq. 16 as printed
    A[11] = -3 * (J(-1, 0) + J(0, 0)) + 5 * J(1, -1)       # Eq. 18 as printed
    A[12] = -3 * (J(-1, -1) + J(0, -1)) + 5 * J(1, 1)      # Eq. 19 as printed
    return A


def responses_from_terms(A):
    """Edge responses from column terms (Section 2.3.2, Eqs. 22-29)."""
    m = [
        A[0] + A[1] + A[2],      # Eq. 22
        A[0] + A[3] + A[4],      # Eq. 23
        A[5] + A[3] + A[6],      # Eq. 24
        A[7] + A[3] + A[8],      # Eq. 25
        A[9] + A[1] + A[8],      # Eq. 26
        A[10] + A[11] + A[8],    # Eq. 27
        A[12] + A[11] + A[13],   # Eq. 28
        A[0] + A[11] + A[14],    # Eq. 29
    ]
    return np.stack(m)


def responses_aldp(img):
    """Eight responses of every interior pixel via the corrected scheme."""
    return responses_from_terms(column_terms(img))
