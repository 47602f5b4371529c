"""Reduced-precision references (test infrastructure only).

Low-precision EHYB plans store values as binary32 or bfloat16 and multiply
binary32 x with binary32 accumulation.  Two references separate the two
sources of error:

* the FP64 product of the original matrix and x (O1): the total error of the
  low-precision result, which is stated, not bounded by 1e-12;
* the FP64 product of the *quantized* values and the binary32-rounded x: the
  low-precision result must agree with it within the accumulation bound
  gamma_m(u = 2^-24) * sum |a_q x_q| (every quantized value and product is
  exact in FP64, so only the binary32 sum rounds).

bfloat16 here means 1 sign, 8 exponent and 7 stored mantissa bits, values
rounded to nearest with ties to even directly from binary64 (no intermediate
binary32 rounding).
"""
from __future__ import annotations

import numpy as np


def to_float32(v: np.ndarray) -> np.ndarray:
    """binary64 -> binary32, round to nearest even (IEEE conversion)."""
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def to_bf16_bits(v: np.ndarray) -> np.ndarray:
    """binary64 -> bfloat16 bit patterns (uint16), round to nearest, ties to
    even, computed on the exact binary64 value.

    For a finite nonzero |v| with exponent e (2^e <= |v| < 2^(e+1)) the
    bfloat16 spacing is 2^(e-7) (never below 2^-133, the subnormal spacing);
    |v| / spacing is exact in binary64, numpy's rint rounds it half to even,
    and the scaled-back result is a bfloat16 value (or overflows to inf)."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    out = np.zeros(v.shape, dtype=np.float64)
    nz = (a > 0) & np.isfinite(a)
    e = np.floor(np.log2(a[nz]))
    # guard log2 rounding at binade edges
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > a[nz], e - 1, e)
    e = np.where(np.ldexp(1.0, (e + 1).astype(np.int64)) <= a[nz], e + 1, e)
    sp = np.maximum(e - 7, -133).astype(np.int64)
    q = np.rint(np.ldexp(a[nz], -sp))
    out[nz] = np.ldexp(q, sp)
    out[~np.isfinite(a)] = a[~np.isfinite(a)]
    big = out > 3.3895313892515355e38    # largest finite bfloat16
    out[big] = np.inf
    f = out.astype(np.float32)            # exact: every bfloat16 is a binary32
    bits = (f.view(np.uint32) >> 16).astype(np.uint16)
    bits |= np.where(np.signbit(v), np.uint16(0x8000), np.uint16(0))
    bits[np.isnan(v)] = 0x7FC0
    return bits


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def quantize(v: np.ndarray, dtype: str) -> np.ndarray:
    """Values as stored by a plan of `dtype` ('f64', 'f32', 'bf16'), as float64."""
    if dtype == "f64":
        return np.asarray(v, dtype=np.float64)
    if dtype == "f32":
        return to_float32(v).astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f64(to_bf16_bits(v))
    raise ValueError(dtype)


def gamma32(m) -> np.ndarray:
    u = 2.0 ** -24
    m = np.asarray(m, dtype=np.float64)
    return m * u / (1.0 - m * u)
