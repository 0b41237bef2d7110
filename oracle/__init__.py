"""CPU oracle for Local Directional Pattern extraction.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything under this
directory.  Only the tests, the smoke entry point and the CPU-baseline leg of
the benchmark use it.

Contents
--------
``ldp.py``        plain numpy definition of the method: Kirsch responses by
                  direct mask correlation (Eq. 1), the k-th largest response and
                  the 8-bit code (Eqs. 2-3), per-cell code histograms (Eqs. 4-5).
``aldp.py``       the paper's acceleration scheme (Section 2.3): the fifteen
                  column terms A0..A14 (Eqs. 7-21, with four misprinted terms
                  corrected) and the eight responses assembled from them
                  (Eqs. 22-29).  Used only to check that the scheme and the
                  direct masks agree exactly.
``ldp_oracle.c``  the same definition as plain scalar C (direct masks, sort of
                  the eight responses, per-cell histograms) for inputs too
                  large for numpy loops and for CPU timing; loaded by
                  ``native.py`` through ctypes.
"""
