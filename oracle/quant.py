"""Reduced-precision storage codes for the feature table (bfloat16, OCP e4m3).

The paper does not fix a precision; these are storage formats for the
feature table F (Sec. 4.1), decoded to FP32 before blending.

* bfloat16: the upper 16 bits of the float32 pattern after round-to-nearest,
  ties-to-even on the dropped 16 bits.
* OCP FP8 e4m3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits, no
  infinities, 0x7F / 0xFF are NaN, largest finite magnitude 448. Each
  Gaussian row i has a float32 scale s_i = max_d |f_id| / 448 (1 for an
  all-zero row); the code is the e4m3 value nearest to the float32 quotient
  f_id / s_i (ties to the even code), and the decoded value is code * s_i.
"""

from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_encode(x) -> np.ndarray:
    """float32 -> uint16 bfloat16 codes (RNE)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    return ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_decode(c) -> np.ndarray:
    c = np.asarray(c, dtype=np.uint16).astype(np.uint32) << 16
    return c.view(np.float32).astype(np.float64)


def e4m3_decode_code(code: int) -> float:
    """Value of one e4m3 code, from the format definition."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return s * (m / 8.0) * 2.0 ** (-6)
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


E4M3_TABLE = np.array([e4m3_decode_code(c) for c in range(256)])


def e4m3_decode(c) -> np.ndarray:
    return E4M3_TABLE[np.asarray(c, dtype=np.uint8).astype(np.int64)]


def e4m3_encode(x) -> np.ndarray:
    """Nearest e4m3 code to each value (ties to even code), saturating at 448."""
    x = np.asarray(x, dtype=np.float64)
    pos_codes = np.arange(0, 0x7F)  # 0x00..0x7E: every finite non-negative value
    pos_vals = E4M3_TABLE[pos_codes]  # increasing
    mag = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.searchsorted(pos_vals, mag, side="left")  # first value >= mag
    hi = np.minimum(hi, pos_codes.size - 1)
    lo = np.maximum(hi - 1, 0)
    d_hi = pos_vals[hi] - mag
    d_lo = mag - pos_vals[lo]
    pick_lo = (d_lo < d_hi) | ((d_lo == d_hi) & (pos_codes[lo] % 2 == 0))
    code = np.where(pick_lo, pos_codes[lo], pos_codes[hi])
    code = np.where(mag == pos_vals[hi], pos_codes[hi], code)
    sign = np.where(np.signbit(x), 0x80, 0)
    # -0.0 stays 0x80; a negative value rounding to zero keeps its sign bit
    return (code | sign).astype(np.uint8)


def e4m3_row_scales(features) -> np.ndarray:
    f = np.asarray(features, dtype=np.float32)
    m = np.max(np.abs(f), axis=1)
    s = (m / np.float32(E4M3_MAX)).astype(np.float32)
    return np.where(m > 0, s, np.float32(1.0)).astype(np.float32)


def e4m3_quantize(features):
    """(codes uint8 [N,D], scales float32 [N]) for a float32 feature table."""
    f = np.asarray(features, dtype=np.float32)
    s = e4m3_row_scales(f)
    q = (f / s[:, None]).astype(np.float32)
    return e4m3_encode(q), s


def e4m3_dequantize(codes, scales) -> np.ndarray:
    return e4m3_decode(codes) * np.asarray(scales, np.float64)[:, None]
