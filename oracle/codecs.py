"""Number formats for the oracle -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's quantized estimate (qCH, Sec. 4.5; quantization in Sec. 4.2)
replaces every vector by a coarse code before scoring. Here the code is an
OCP FP8 E4M3 ("e4m3fn") vector with one power-of-two float32 scale per vector,
and the exact paths may run on bfloat16 operands. Everything below is written
from the format definitions, in plain NumPy:

  * bfloat16: the top 16 bits of an IEEE binary32, rounded to nearest, ties to
    even on the dropped 16 bits; and the split of a float32 into two bfloat16
    parts (hi, lo) that lets float32 products run as three bfloat16 products.
  * OCP FP8 E4M3 (OCP 8-bit Floating Point Specification, 2023): 1 sign bit,
    4 exponent bits with bias 7, 3 mantissa bits; exponent field 0 encodes
    subnormals 2^-6 * m/8; S.1111.111 is NaN; there is no infinity; the largest
    finite magnitude is 1.75 * 2^8 = 448.
  * per-vector scale: the smallest power of two s = 2^e with amax <= 448 * s,
    where amax is the largest |component| of the vector (s = 1 when amax = 0);
    e is clamped to [-126, 127] so that s stays a normal float32.
  * encoding: round x / s to the nearest E4M3 value, ties to the even code,
    saturating magnitudes above 448 to 448; NaN encodes as 0x7F.
"""
from __future__ import annotations

import math

import numpy as np

E4M3_MAX = 448.0


def bf16_round_bits(x) -> np.ndarray:
    """float32 array -> bfloat16 bit patterns (uint16), round to nearest even."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) & 0xFFFF
    nan = np.isnan(x)
    if nan.any():
        sign = (bits >> 16) & 0x8000
        rounded = np.where(nan, sign | 0x7FC0, rounded)
    return rounded.astype(np.uint16)


def bf16_decode(bits) -> np.ndarray:
    """bfloat16 bit patterns (uint16) -> float64 values (exact)."""
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint16)).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def split_bf16x3(x) -> tuple[np.ndarray, np.ndarray]:
    """float32 array -> bfloat16 bit patterns (hi, lo) of the split x = hi + lo + e:
    hi = bf16(x), lo = bf16(x - hi), each rounded to nearest even. x - hi is
    exact in float32 (both are multiples of x's float32 ulp and the difference
    is at most half a bfloat16 ulp of x), so |e| <= 2^-8 |x - hi| <= 2^-16 |x|."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    hi = bf16_round_bits(x)
    rest = (x.astype(np.float64) - bf16_decode(hi)).astype(np.float32)
    return hi, bf16_round_bits(rest)


def e4m3_decode(code: int) -> float:
    """One OCP E4M3 code (0..255) -> its value, from the format definition."""
    code = int(code) & 0xFF
    sign = -1.0 if code & 0x80 else 1.0
    exp = (code >> 3) & 0xF
    man = code & 0x7
    if exp == 0xF and man == 0x7:
        return math.nan
    if exp == 0:
        return sign * math.ldexp(man / 8.0, 1 - 7)
    return sign * math.ldexp(1.0 + man / 8.0, exp - 7)


def e4m3_decode_table() -> np.ndarray:
    """All 256 codes decoded (float64; NaN for the two NaN codes)."""
    return np.array([e4m3_decode(c) for c in range(256)], dtype=np.float64)


_TABLE = e4m3_decode_table()
# Codes 0x00..0x7E are the non-negative finite values, increasing with the code.
_POS_VALUES = _TABLE[:0x7F]


def e4m3_decode_array(codes) -> np.ndarray:
    return _TABLE[np.asarray(codes, dtype=np.uint8)]


def e4m3_encode(x) -> np.ndarray:
    """float64 array -> E4M3 codes (uint8): nearest value, ties to even code, saturating."""
    x = np.asarray(x, dtype=np.float64)
    mag = np.abs(x)
    sign = np.where(np.signbit(x), 0x80, 0x00).astype(np.int64)
    hi = np.searchsorted(_POS_VALUES, mag, side="left")      # first value >= mag
    hi = np.clip(hi, 0, len(_POS_VALUES) - 1)
    lo = np.clip(hi - 1, 0, len(_POS_VALUES) - 1)
    d_hi = np.abs(_POS_VALUES[hi] - mag)
    d_lo = np.abs(mag - _POS_VALUES[lo])
    pick = np.where(d_lo < d_hi, lo, hi)
    tie = (d_lo == d_hi) & (lo != hi)
    pick = np.where(tie, np.where(lo % 2 == 0, lo, hi), pick)
    pick = np.where(mag >= E4M3_MAX, 0x7E, pick)             # saturate to 448
    code = (pick | sign).astype(np.uint8)
    code = np.where(np.isnan(x), np.uint8(0x7F), code)
    return code.astype(np.uint8)


def pow2_scale(amax: float) -> float:
    """Smallest power of two s with amax <= 448 * s (s = 1 for amax = 0), e in [-126, 127]."""
    amax = float(amax)
    if amax == 0.0:
        return 1.0
    _, E = math.frexp(amax)              # amax = f * 2^E, 0.5 <= f < 1
    e = E - 12
    while amax > E4M3_MAX * math.ldexp(1.0, e):
        e += 1
    e = max(-126, min(127, e))
    return math.ldexp(1.0, e)


def quantize_fp8(vecs) -> tuple[np.ndarray, np.ndarray]:
    """float32 rows -> (E4M3 codes uint8 [n, d], power-of-two scales float32 [n])."""
    v = np.asarray(vecs, dtype=np.float32)
    n = v.shape[0]
    amax = np.abs(v).max(axis=1) if v.shape[1] else np.zeros(n, np.float32)
    scales = np.array([pow2_scale(a) for a in amax], dtype=np.float64)
    codes = e4m3_encode(v.astype(np.float64) / scales[:, None])
    return codes, scales.astype(np.float32)


def dequantize_fp8(codes, scales) -> np.ndarray:
    """(codes, scales) -> float64 rows s * decode(code) (exact)."""
    return e4m3_decode_array(codes) * np.asarray(scales, dtype=np.float64)[:, None]
