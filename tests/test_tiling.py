"""Host-side check of the arithmetic behind cell-contiguous tiles.

A workgroup of a cell-contiguous tile finds each lane's coordinates by
dividing a < d + 512 (the tile's start x or y plus an offset below 512) by
the row length or the plane height d <= 65535, as a float product with the
rounded reciprocal followed by one remainder test on each side.  This checks,
in IEEE single precision, that the result is the exact quotient at every
critical point: the multiples of d, their neighbours, and the ends of the
range."""
import numpy as np


def _div_small(a, d):
    a = np.asarray(a, dtype=np.uint32)
    inv = np.float32(1.0) / np.float32(d)                    # host: 1.0f / (float)d
    q = (a.astype(np.float32) * inv).astype(np.uint32)       # product rounded to float, truncated
    r = a.astype(np.int64) - q.astype(np.int64) * d
    neg = r < 0
    q = np.where(neg, q - 1, q)
    r = np.where(neg, r + d, r)
    return np.where(r >= d, q + 1, q)


def test_float_reciprocal_quotient_is_exact():
    for d in range(1, 65536):
        top = d + 512
        k = np.arange(0, top // d + 2, dtype=np.int64) * d
        a = np.concatenate([k - 1, k, k + 1, [0, top - 1, top - 2]])
        a = a[(a >= 0) & (a < top)]
        assert np.array_equal(_div_small(a, d), a // d), d


def test_float_reciprocal_quotient_dense_small_divisors():
    # every a for the divisors where the tile spans the most rows
    for d in range(1, 130):
        a = np.arange(0, d + 512, dtype=np.int64)
        assert np.array_equal(_div_small(a, d), a // d), d
