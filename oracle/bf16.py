"""Bit-exact emulation of the split-bfloat16 operand format (oracle, test
infrastructure only).

The mixed-precision projection/rotation GEMMs take FP32 operands as an
unevaluated sum of two bfloat16 numbers and form three products with FP32
accumulation ("bf16x3", Henry, Tang & Heinecke 2019):
  a_hi = bf16_rne(a),  a_lo = bf16_rne(a - a_hi)   (the subtraction is exact in FP32)
  a*b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi.
bf16_rne is IEEE round-to-nearest-even of the FP32 bit pattern to its top
16 bits.  NaN and Inf inputs are out of scope (the path never feeds them).
Pins: torch's own float32 -> bfloat16 conversion (also RNE), hand-picked
tie cases, and |a - a_hi - a_lo| <= 2^-16 |a| (tests/test_oracle_bf16.py).
"""
from __future__ import annotations

import numpy as np


def bf16_rne_bits(a: np.ndarray) -> np.ndarray:
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    return ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def split(a: np.ndarray):
    """(hi bits, lo bits) as uint16 arrays."""
    a = np.asarray(a, dtype=np.float32)
    hi = bf16_rne_bits(a)
    rem = (a - bf16_to_f32(hi)).astype(np.float32)
    lo = bf16_rne_bits(rem)
    return hi, lo


def split_values(a: np.ndarray):
    hi, lo = split(a)
    return bf16_to_f32(hi), bf16_to_f32(lo)
