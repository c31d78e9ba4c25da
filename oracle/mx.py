"""MXFP4 and MXFP6 (OCP Microscaling, E2M1 / E2M3 elements) for the oracle --
TEST INFRASTRUCTURE ONLY.

The paper names ultra-low-bit quantization as the next step for its quantized
estimate (Sec. 6, conclusion). The formats here are written from the OCP
Microscaling Formats specification (v1.0, 2023).

MXFP4:

  * element E2M1: 1 sign bit, 2 exponent bits with bias 1, 1 mantissa bit;
    exponent field 0 holds the subnormals 0 and 0.5; the magnitudes are
    0, 0.5, 1, 1.5, 2, 3, 4, 6; there is no infinity and no NaN;
  * block: 32 consecutive elements of a vector share one E8M0 scale 2^e
    (an exponent byte e + 127);
  * reading of the block scale (the specification leaves it to the encoder):
    the smallest 2^e with amax <= 6 * 2^e, e in [-127, 127], 2^0 for an
    all-zero block, so that no element is clipped;
  * element encoding: the E2M1 value nearest to x / 2^e, ties to the even code.

MXFP6 (E2M3 elements):

  * element E2M3: 1 sign bit, 2 exponent bits with bias 1, 3 mantissa bits;
    exponent field 0 holds the subnormals m / 8 (m = 0..7); the largest
    magnitude is 7.5; there is no infinity and no NaN; a code is
    sign << 5 | exponent << 3 | mantissa;
  * block: as for MXFP4, 32 elements share one E8M0 scale 2^e;
  * reading of the block scale: the smallest 2^e with amax <= 7.5 * 2^e,
    e in [-127, 127], 2^0 for an all-zero block (no element is clipped);
  * element encoding: the E2M3 value nearest to x / 2^e, ties to the even code.
"""
from __future__ import annotations

import math

import numpy as np

E2M1_MAX = 6.0
E2M3_MAX = 7.5
BLOCK = 32


def e2m1_decode(code: int) -> float:
    """Value of a 4-bit E2M1 code, from the field definitions."""
    code = int(code) & 0xF
    sign = -1.0 if code & 0x8 else 1.0
    e = (code >> 1) & 0x3
    m = code & 0x1
    if e == 0:
        return sign * (m / 2.0)                       # subnormal: 0.m * 2^(1 - bias), bias 1
    return sign * (1.0 + m / 2.0) * 2.0 ** (e - 1)


def e2m1_table() -> np.ndarray:
    return np.array([e2m1_decode(c) for c in range(16)], dtype=np.float64)


def e2m1_encode(y) -> np.ndarray:
    """Nearest E2M1 code to each y (|y| <= 6 expected), ties to the even code;
    magnitudes beyond 6 take the largest code. Brute force over the 8 magnitudes."""
    y = np.asarray(y, dtype=np.float64)
    mags = e2m1_table()[:8]
    a = np.minimum(np.abs(y), E2M1_MAX)
    d = np.abs(a[..., None] - mags)                   # distance to every magnitude
    best = d.min(axis=-1, keepdims=True)
    cand = d == best
    # among the nearest magnitudes (one, or two at a midpoint) take the even code
    even = cand & (np.arange(8) % 2 == 0)
    pick = np.where(even.any(axis=-1), np.argmax(even, axis=-1), np.argmax(cand, axis=-1))
    sign = np.where(np.signbit(y) & (pick > 0), 8, 0)
    return (pick | sign).astype(np.uint8)


def block_exponent(amax: float, top: float = E2M1_MAX) -> int:
    """Smallest e in [-127, 127] with amax <= top * 2^e (0 for amax = 0); top is
    the element format's largest magnitude (6 for E2M1, 7.5 for E2M3)."""
    amax = float(amax)
    if amax == 0.0:
        return 0
    _, E = math.frexp(amax)                           # amax = f * 2^E, 0.5 <= f < 1
    e = E - 4                                         # below the answer for top < 8
    while amax > top * math.ldexp(1.0, e):
        e += 1
    return max(-127, min(127, e))


def quantize_mxfp4(vecs) -> tuple[np.ndarray, np.ndarray]:
    """float32 rows [n, d] (d a multiple of 32) -> (E2M1 codes uint8 [n, d], one
    per element, and block exponents int32 [n, d / 32])."""
    v = np.asarray(vecs, dtype=np.float32).astype(np.float64)
    n, d = v.shape
    blocks = v.reshape(n, d // BLOCK, BLOCK)
    amax = np.abs(blocks).max(axis=2)
    exps = np.array([[block_exponent(a) for a in row] for row in amax], dtype=np.int32).reshape(n, d // BLOCK)
    scaled = blocks / np.ldexp(1.0, exps)[..., None]
    codes = e2m1_encode(scaled).reshape(n, d)
    return codes, exps


def dequantize_mxfp4(codes, exps) -> np.ndarray:
    """(codes, block exponents) -> float64 rows (exact)."""
    codes = np.asarray(codes, dtype=np.uint8)
    n, d = codes.shape
    vals = e2m1_table()[codes].reshape(n, d // BLOCK, BLOCK)
    return (vals * np.ldexp(1.0, np.asarray(exps, np.int64))[..., None]).reshape(n, d)


# ---------------------------------------------------------------------- MXFP6
def e2m3_decode(code: int) -> float:
    """Value of a 6-bit E2M3 code, from the field definitions."""
    code = int(code) & 0x3F
    sign = -1.0 if code & 0x20 else 1.0
    e = (code >> 3) & 0x3
    m = code & 0x7
    if e == 0:
        return sign * (m / 8.0)                       # subnormal: 0.mmm * 2^(1 - bias), bias 1
    return sign * (1.0 + m / 8.0) * 2.0 ** (e - 1)


def e2m3_table() -> np.ndarray:
    return np.array([e2m3_decode(c) for c in range(64)], dtype=np.float64)


def e2m3_encode(y) -> np.ndarray:
    """Nearest E2M3 code to each y (|y| <= 7.5 expected), ties to the even code;
    magnitudes beyond 7.5 take the largest code. Brute force over the 32 magnitudes."""
    y = np.asarray(y, dtype=np.float64)
    mags = e2m3_table()[:32]
    a = np.minimum(np.abs(y), E2M3_MAX)
    d = np.abs(a[..., None] - mags)
    best = d.min(axis=-1, keepdims=True)
    cand = d == best
    even = cand & (np.arange(32) % 2 == 0)
    pick = np.where(even.any(axis=-1), np.argmax(even, axis=-1), np.argmax(cand, axis=-1))
    sign = np.where(np.signbit(y) & (pick > 0), 0x20, 0)
    return (pick | sign).astype(np.uint8)


def quantize_mxfp6(vecs) -> tuple[np.ndarray, np.ndarray]:
    """float32 rows [n, d] (d a multiple of 32) -> (E2M3 codes uint8 [n, d], one
    per element, and block exponents int32 [n, d / 32])."""
    v = np.asarray(vecs, dtype=np.float32).astype(np.float64)
    n, d = v.shape
    blocks = v.reshape(n, d // BLOCK, BLOCK)
    amax = np.abs(blocks).max(axis=2)
    exps = np.array([[block_exponent(a, E2M3_MAX) for a in row] for row in amax],
                    dtype=np.int32).reshape(n, d // BLOCK)
    scaled = blocks / np.ldexp(1.0, exps)[..., None]
    codes = e2m3_encode(scaled).reshape(n, d)
    return codes, exps


def dequantize_mxfp6(codes, exps) -> np.ndarray:
    """(codes, block exponents) -> float64 rows (exact)."""
    codes = np.asarray(codes, dtype=np.uint8)
    n, d = codes.shape
    vals = e2m3_table()[codes].reshape(n, d // BLOCK, BLOCK)
    return (vals * np.ldexp(1.0, np.asarray(exps, np.int64))[..., None]).reshape(n, d)
