"""Storage quantisation and value range (test infrastructure).

* float16: numpy's IEEE binary16 conversion (round to nearest, ties to even).
* bfloat16: round-to-nearest-even on the top 16 bits of the binary32 pattern, NaN kept NaN.
* ``finite_minmax``: minimum and maximum over finite values (the colour-map domain
  default; DATAMIN = the minimum).
"""
from __future__ import annotations

import numpy as np


def to_f16(a):
    return np.asarray(a, dtype=np.float32).astype(np.float16)


def to_bf16_bits(a):
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = np.isnan(np.asarray(a, dtype=np.float32))
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(nan, (u >> 16) | 0x0040, r)
    return r.astype(np.uint16)


def bf16_bits_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def to_bf16_as_f32(a):
    return bf16_bits_to_f32(to_bf16_bits(a))


def dequantize(a, storage):
    """Values a cube holds once stored as ``storage`` ('f32', 'f16' or 'bf16'), as float32."""
    a = np.asarray(a, dtype=np.float32)
    if storage == "f32":
        return a.copy()
    if storage == "f16":
        return to_f16(a).astype(np.float32)
    if storage == "bf16":
        return to_bf16_as_f32(a)
    raise ValueError(storage)


def finite_minmax(a):
    a = np.asarray(a)
    f = a[np.isfinite(a)]
    if f.size == 0:
        return float("nan"), float("nan")
    return float(f.min()), float(f.max())
