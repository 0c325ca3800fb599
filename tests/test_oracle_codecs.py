"""Pins of the reference 16-bit codecs against what the paper and mathematics
fix: Fig. 2 (code of 1.0), Table 2 (range, smallest values, epsilon, digits),
IEEE binary16 as implemented by numpy, exhaustive round trips, monotonicity,
the tie rule at every midpoint, and the paper's accuracy-interval claims for
the posit formats (Sec. 3.2.2)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FMTS = ("fp16", "fp16s", "fp16c", "p16_0s", "p16_1s", "p16_2c")
ALL_CODES = np.arange(65536, dtype=np.uint32).astype(np.uint16)


def _golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def _positive_values(orc, fmt):
    v = orc.decode(fmt, np.arange(0x8000, dtype=np.uint16))
    return v[np.isfinite(v)]


@pytest.mark.parametrize("fmt,bits,hexcode", [tuple(r) for r in _golden("format_one_codes.txt")])
def test_code_of_one_matches_fig2(orc, fmt, bits, hexcode):
    code = int(hexcode, 16)
    assert int(bits.replace("_", ""), 2) == code
    assert orc.decode(fmt, np.array([code]))[0] == 1.0
    assert int(orc.encode(fmt, np.array([1.0], np.float32))[0]) == code
    assert int(orc.encode(fmt, np.array([-1.0], np.float32))[0]) == code | 0x8000


@pytest.mark.parametrize("row", _golden("table2_formats.txt"), ids=lambda r: r[0])
def test_table2_constants(orc, row):
    fmt, n_m, digits, eps, vmax, smin_norm, smin = row
    pos = _positive_values(orc, fmt)
    # range and smallest positive value (denormal or minpos), to the printed
    # 7 digits (one unit of the last printed digit: the table rounds 2^-59 up)
    assert pos[-1] == pytest.approx(float(vmax), rel=1.5e-6)
    assert pos[1] == pytest.approx(float(smin), rel=1.5e-6)
    # epsilon and digits follow from the (largest) mantissa width
    assert float(f"{2.0 ** -int(n_m):.1e}") == float(eps)
    assert round(math.log10(2.0 ** (int(n_m) + 1)), 1) == float(digits)
    # the mantissa width is what the codes show: the finest step above a
    # power of two, relative to it
    k = np.nonzero(np.frexp(pos[1:-1])[0] == 0.5)[0] + 1
    rel = (pos[k + 1] - pos[k]) / pos[k]
    assert rel.min() == 2.0 ** -int(n_m)
    if smin_norm != "-":
        # smallest normal: first value from which the spacing is relative
        exp_min = {"fp16": -14, "fp16s": -29, "fp16c": -14}[fmt]
        assert 2.0 ** exp_min in set(pos.tolist())
        step = pos[2] - pos[1]
        assert pos[int(round(2.0 ** exp_min / step))] == 2.0 ** exp_min
        assert float(f"{2.0 ** exp_min:.2e}") == float(f"{float(smin_norm):.2e}")
        if fmt != "fp16s":
            assert float(f"{2.0 ** exp_min:.6e}") == float(smin_norm)


@pytest.mark.parametrize("fmt", FMTS)
def test_all_codes_round_trip(orc, fmt):
    v = orc.decode(fmt, ALL_CODES)
    finite = np.isfinite(v)
    # every finite value is exactly a float32
    assert np.all(v[finite].astype(np.float32).astype(np.float64) == v[finite])
    back = orc.encode(fmt, v[finite].astype(np.float32))
    assert np.array_equal(back, ALL_CODES[finite])
    if fmt in ("fp16", "fp16s"):
        assert np.count_nonzero(~finite) == 2 * 1024          # Inf and NaN codes
    else:
        assert np.all(finite)                                 # no Inf/NaN (Sec. 3.1.4, 3.2.3)


@pytest.mark.parametrize("fmt", FMTS)
def test_decode_monotone_and_symmetric(orc, fmt):
    pos = _positive_values(orc, fmt)
    assert pos[0] == 0.0 and np.all(np.diff(pos) > 0)
    neg = orc.decode(fmt, (np.arange(len(pos)) | 0x8000).astype(np.uint16))
    assert np.array_equal(neg, -pos)
    assert math.copysign(1.0, neg[0]) == -1.0                  # -0 exists (sign-magnitude)


@pytest.mark.parametrize("fmt", ("fp16", "fp16s"))
def test_ieee_half_matches_numpy(orc, fmt):
    rng = np.random.default_rng(1)
    scale = 32768.0 if fmt == "fp16s" else 1.0
    bits = rng.integers(0, 2 ** 32, size=400000, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    # plus values spread over the FP16 range, where most codes live
    x = np.concatenate([x, (rng.standard_normal(400000) * 10.0 ** rng.uniform(-9, 5, 400000)
                            / scale).astype(np.float32)])
    with np.errstate(over="ignore"):
        ref = (x.astype(np.float64) * scale).astype(np.float32).astype(np.float16).view(np.uint16)
    got = orc.encode(fmt, x)
    assert np.array_equal(got, ref)


def test_fp16c_normal_range_matches_bit_rounding(orc):
    """In its normal range FP16C is FP32 with 4 exponent bits (bias 15) and
    the mantissa cut to 11 bits; rounding half away from zero there is
    'add half an FP16C ulp to the FP32 bits and truncate'."""
    rng = np.random.default_rng(2)
    x = (rng.uniform(-1, 1, 300000) * 2.0 ** rng.uniform(-14, 0.99, 300000)).astype(np.float32)
    x = x[np.abs(x) >= 2.0 ** -14]
    b = x.view(np.uint32).astype(np.int64)
    sign = (b >> 16) & 0x8000
    mag = b & 0x7FFFFFFF
    code = ((mag - (112 << 23)) + 0x800) >> 12
    code = np.minimum(code, 0x7FFF)
    assert np.array_equal(orc.encode("fp16c", x), (sign | code).astype(np.uint16))


@pytest.mark.parametrize("fmt", FMTS)
def test_encode_is_nearest_exact_rational(orc, fmt):
    """Brute force on a sample: no other code is nearer than the chosen one
    (exact rational arithmetic), ties broken as the format prescribes."""
    rng = np.random.default_rng(3)
    pos = _positive_values(orc, fmt)
    top = pos[-1]
    x = (rng.uniform(0, 1, 3000) * top * 2.0 ** -rng.uniform(0, 40, 3000)).astype(np.float32)
    codes = orc.encode(fmt, x)
    for xi, c in zip(x.tolist(), codes.tolist()):
        X = Fraction(xi)
        d = abs(X - Fraction(pos[c]))
        for nb in (c - 1, c + 1):
            if 0 <= nb < len(pos):
                dn = abs(X - Fraction(pos[nb]))
                assert d <= dn, (fmt, xi, c, nb)


@pytest.mark.parametrize("fmt", FMTS)
def test_ties_and_neighbours_of_every_midpoint(orc, fmt):
    pos = _positive_values(orc, fmt)
    lo, hi = pos[:-1], pos[1:]
    mid = (lo + hi) / 2.0
    m32 = mid.astype(np.float32)
    assert np.all(m32.astype(np.float64) == mid)               # midpoints exact in FP32
    codes = orc.encode(fmt, m32).astype(np.int64)
    idx = np.arange(len(mid))
    if fmt in ("fp16", "fp16s"):
        expect = np.where(idx % 2 == 0, idx, idx + 1)          # ties to even
    else:
        expect = idx + 1                                       # ties away from zero
    assert np.array_equal(codes, expect)
    below = np.nextafter(m32, np.float32(0))
    above = np.nextafter(m32, np.float32(np.inf))
    assert np.array_equal(orc.encode(fmt, below).astype(np.int64), idx)
    assert np.array_equal(orc.encode(fmt, above).astype(np.int64), idx + 1)


def test_saturation_and_specials(orc):
    for fmt in ("fp16c", "p16_0s", "p16_1s", "p16_2c"):
        big = np.array([3.0, 1e30, np.inf, -np.inf, np.nan], np.float32)
        if fmt in ("p16_0s", "p16_1s"):
            big[0] = 3e7
        c = orc.encode(fmt, big)
        assert list(c[:3]) == [0x7FFF] * 3 and c[3] == 0xFFFF and (c[4] & 0x7FFF) == 0x7FFF
    f16 = orc.encode("fp16", np.array([65519.99, 65520.0, np.inf, np.nan], np.float32))
    assert list(f16[:3]) == [0x7BFF, 0x7C00, 0x7C00] and (f16[3] & 0x7C00) == 0x7C00 and (f16[3] & 0x3FF)
    tiny = orc.encode("fp16c", np.array([2.0 ** -26, np.nextafter(np.float32(2.0 ** -26), np.float32(0))],
                                        np.float32))
    assert list(tiny) == [1, 0]


def _min_digits(orc, fmt, lo, hi, n=20000):
    """Worst decimal digits -log10|log10(x_repr/x)| (appendix, measured format
    characteristics) over [lo, hi)."""
    x = np.exp(np.linspace(math.log(lo), math.log(hi), n)).astype(np.float32)
    v = orc.decode(fmt, orc.encode(fmt, x))
    with np.errstate(divide="ignore"):
        d = -np.log10(np.abs(np.log10(v / x.astype(np.float64))))
    return d[np.isfinite(d)].min()


@pytest.mark.parametrize("better,worse,lo_exp,hi_exp", [
    ("p16_0s", "fp16s", -11, -3), ("p16_0s", "fp16c", -10, -4),
    ("p16_1s", "fp16s", -13, -1), ("p16_1s", "fp16c", -11, -3),
    ("p16_2c", "fp16c", -7, 1), ("p16_2c", "fp16s", -11, 1),
    ("fp16c", "fp16", -14, 1),
])
def test_accuracy_interval_claims(orc, better, worse, lo_exp, hi_exp):
    """Sec. 3.2.2 and 3.1.2: in the stated intervals the first format is at
    least as accurate as the second (compared binade by binade), and strictly
    more accurate somewhere inside."""
    strictly = False
    for e in range(lo_exp, hi_exp):
        a = _min_digits(orc, better, 2.0 ** e, 2.0 ** (e + 1) * 0.99999)
        b = _min_digits(orc, worse, 2.0 ** e, 2.0 ** (e + 1) * 0.99999)
        assert a >= b - 1e-9, (better, worse, e, a, b)
        strictly |= a > b + 1e-6
    assert strictly
