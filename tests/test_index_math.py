"""Host checks of the kernels' integer-by-float index arithmetic.

The kernels split a flat index q into (q / d, q % d) with one FP32 multiply,
(int)((q + 1/2) * inv_d), where inv_d is 1/d rounded to FP32 or the hardware
reciprocal (within one ulp of 1/d).  The claim is that the truncation is the
exact integer quotient for q < 2^21; here every q < 2^16 and d <= 1024 is
checked in FP32 arithmetic with the correctly rounded inverse and with both of
its neighbours.
"""
import numpy as np


def _quotients(q, inv):
    prod = (q.astype(np.float32) + np.float32(0.5)) * np.float32(inv)
    assert prod.dtype == np.float32
    return prod.astype(np.int64)  # truncation toward zero, as the kernel's cast


def test_small_div_exact_with_one_ulp_inverses():
    q = np.arange(1 << 16, dtype=np.int64)
    for d in range(1, 1025):
        exact = q // d
        inv = np.float32(1.0) / np.float32(d)
        for v in (np.nextafter(inv, np.float32(0)), inv, np.nextafter(inv, np.float32(1))):
            np.testing.assert_array_equal(_quotients(q, v), exact, err_msg=f"d={d} inv={v!r}")


def test_small_div_near_the_stated_bound():
    # the largest quotients the bound covers, for the divisors the kernels use
    q = np.arange((1 << 21) - 4096, 1 << 21, dtype=np.int64)
    for d in list(range(1, 70)) + [127, 255, 1000]:
        inv = np.float32(1.0) / np.float32(d)
        for v in (np.nextafter(inv, np.float32(0)), inv, np.nextafter(inv, np.float32(1))):
            np.testing.assert_array_equal(_quotients(q, v), q // d, err_msg=f"d={d}")
