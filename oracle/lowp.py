"""BF16 rounding with integer operations (test infrastructure only).

The precision form streams a BF16 copy of X = [A, -b] through the sampling
pass.  BF16 keeps the top 16 bits of an IEEE FP32 word; rounding is to
nearest, ties to even, done here on the bit pattern: add 0x7FFF plus the
lowest kept bit, then drop the low 16 bits.  Inputs are finite.
"""
from __future__ import annotations

import numpy as np


def f32_to_bf16_bits(x) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    return ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)


def bf16_bits_to_f64(h) -> np.ndarray:
    u = np.asarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    """FP32 values rounded to BF16, returned as FP64."""
    return bf16_bits_to_f64(f32_to_bf16_bits(x))
