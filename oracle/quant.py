"""Rounding emulation for reduced-precision formats -- TEST INFRASTRUCTURE.

The paper states no numeric precision.  The reduced-precision GPU paths store
network operands in bfloat16 (8-bit exponent, 7 stored mantissa bits) or in
OCP FP8 E4M3FN (bias 7, 3 mantissa bits, largest finite 448, no infinities),
both rounded to nearest with ties to even; E4M3 values beyond +-448 saturate.
These functions produce the float64 value of the rounded number so that the
oracle can repeat a reduced-precision computation exactly where it rounds.
"""
from __future__ import annotations

import numpy as np


def round_bf16(a) -> np.ndarray:
    """float64 value of round-to-nearest-even bfloat16(float32(a))."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0


def round_e4m3(a) -> np.ndarray:
    """float64 value of saturating round-to-nearest-even E4M3FN(a)."""
    a = np.asarray(a, dtype=np.float64)
    mag = np.abs(a)
    # exponent of the binade; values below 2^-6 use the subnormal quantum 2^-9
    e = np.floor(np.log2(np.maximum(mag, 2.0 ** -6)))
    quantum = 2.0 ** (e - 3)
    r = np.round(mag / quantum) * quantum  # numpy rounds halves to even
    r = np.minimum(r, E4M3_MAX)
    return np.sign(a) * r
