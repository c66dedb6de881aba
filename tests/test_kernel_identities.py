"""Host-side checks of identities the kernels rely on (no GPU)."""
import numpy as np

import paper_1102_0148_amd as corr


def test_int16_digit_rule_by_nearest_integer():
    """The F-stage forms the high base-255 digit of an int16 code q as the
    integer nearest q * fl(1/255), rounded by adding 1.5 * 2^23 in one fused
    operation. For every code |q| <= 32512 that equals the defining
    floor((q + 127.5) / 255), and the low digit q - 255 h lies in [-127, 127]
    (the product is formed exactly in float64 here; no value lands on a
    rounding tie, so rounding the sum to float32 once gives the fused result)."""
    q = np.arange(-32512, 32513, dtype=np.float64)
    c = np.float64(np.float32(1.0 / 255.0))
    magic = np.float64(12582912.0)
    hm = (q * c + magic).astype(np.float32).astype(np.float64)
    h = hm - magic
    np.testing.assert_array_equal(h, np.floor((q + 127.5) / 255.0))
    frac = np.abs(q * c - np.round(q * c))
    assert np.all(np.abs(frac - 0.5) > 1e-3)  # far from a tie
    l = q - 255.0 * h
    assert l.min() >= -127 and l.max() <= 127
    hh, ll = corr.int16_digits(q.astype(np.int64))
    np.testing.assert_array_equal(hh, h)
    np.testing.assert_array_equal(ll, l)


def test_int16_low_digit_byte_from_biased_bits():
    """The F-stage writes the low digit's byte as the low byte of the sum of
    the bit patterns of 1.5 * 2^23 + q and 1.5 * 2^23 + h (both exact
    floats): for every code that byte is l = q - 255 h as a two's-complement
    int8."""
    q = np.arange(-32512, 32513, dtype=np.int64)
    h = np.floor((q + 127.5) / 255.0).astype(np.int64)
    l = q - 255 * h
    magic = np.float32(12582912.0)
    qm = (magic + q.astype(np.float32)).view(np.uint32).astype(np.int64)
    hm = (magic + h.astype(np.float32)).view(np.uint32).astype(np.int64)
    bias = int(np.float32(magic).view(np.uint32))
    np.testing.assert_array_equal(qm - bias, q)
    np.testing.assert_array_equal(hm - bias, h)
    assert bias & 0xFF == 0
    byte = ((qm + hm) & 0xFF).astype(np.uint8).view(np.int8)
    np.testing.assert_array_equal(byte, l.astype(np.int8))

