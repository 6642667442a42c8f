"""Host checks of the index arithmetic the kernels rely on (no GPU).

The interval passes decode a row index r = x (2^n + 1) + k of a level into the
probe column x and direction k with a single-precision estimate of
r / (2^n + 1) followed by one correction in each direction, instead of an
integer division.  The estimate is the float product of r with the reciprocal
of the divisor, which the device computes to within one unit in the last
place; this checks, for every row of every level of every grid from 8^2 to
4096^2 and for reciprocals one unit below, at and above the correctly rounded
one, that the corrected estimate is the exact quotient.
"""
import numpy as np


def corrected_quotient(r: np.ndarray, d: int, rcp: np.float32) -> np.ndarray:
    x = (r.astype(np.float32) * rcp).astype(np.uint64)
    x = np.where(x * d > r, x - 1, x)
    return np.where((x + 1) * d <= r, x + 1, x)


def test_row_decode_is_exact_for_every_level():
    for N in range(3, 13):
        S = 1 << N
        for n in range(0, N + 1):
            d = (1 << n) + 1
            rows = (S >> n) * d
            r = np.arange(rows, dtype=np.uint64)
            rcp = np.float32(1.0) / np.float32(d)
            for approx in (np.nextafter(rcp, np.float32(0)), rcp, np.nextafter(rcp, np.float32(1))):
                np.testing.assert_array_equal(corrected_quotient(r, d, approx), r // d,
                                              err_msg=f"N={N} n={n}")
