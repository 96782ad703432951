"""The D2Q9 tile kernel's row split of a slot index, checked exhaustively.

k_d2q9_tiles deals the cells of a step's region to its threads row by row:
slot r of a region w cells wide lies in row r / w. The kernel takes that
quotient as trunc((r + 1/2) * rcp(w)) in FP32 instead of an integer
division, where rcp is the hardware reciprocal, within 1 ulp of 1/w. This
checks, with every FP32 value within 1 ulp of 1/w standing in for rcp(w) and
a correctly rounded FP32 product, that the split equals the integer quotient
for every region width up to 256 and every slot below 2^11, the bounds the
kernel asserts at compile time.
"""

import numpy as np


def test_reciprocal_row_split_is_exact():
    r = np.arange(2048, dtype=np.int64)
    rf = r.astype(np.float32) + np.float32(0.5)
    for w in range(1, 257):
        near = np.float32(1.0) / np.float32(w)
        for inv_w in (np.nextafter(near, np.float32(0)), near, np.nextafter(near, np.float32(1))):
            q = (rf * inv_w).astype(np.float32).astype(np.int64)  # truncation toward zero
            assert np.array_equal(q, r // w), (w, inv_w)


def test_the_margin_the_split_relies_on():
    # (r + 1/2) / w keeps at least 1/(2w) from the integers, and a 1-ulp
    # reciprocal with a rounded product moves it by at most 2^-22 of itself:
    # under that margin
    r = np.arange(2048, dtype=np.float64)
    for w in (1, 7, 26, 30, 32, 64, 255, 256):
        v = (r + 0.5) / w
        gap = np.minimum(v - np.floor(v), np.ceil(v) - v).min()
        assert gap >= 0.5 / w - 1e-12
        assert (v * 2.0 ** -22).max() < gap
