"""Oracle of the low-precision copies of A streamed by the mixed-precision modes.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, written from the
definitions:

* FP32 copy: every element rounded to the nearest FP32 value, ties to even (the
  IEEE 754 default rounding; numpy's float64 -> float32 cast).
* BF16x2 copy: ``hi`` is the element rounded to the nearest BF16 value, ties to
  even, in one rounding from the double; ``lo`` is ``A - hi`` (exact in FP64)
  rounded the same way.  BF16 has 8 significant bits (1 implicit + 7 stored) and
  FP32's exponent range.  These functions cover normal BF16 magnitudes,
  2**-126 <= |a| < 2**128, and zero; nothing smaller is rounded to a BF16
  subnormal here.

The mixed-precision refinement loop itself has no oracle trajectory: its iterates
legitimately differ from any FP64 run.  Its results are pinned by the explicit FP64
residual (``oracle.residual``) and by the distance to the direct solution.
"""
from __future__ import annotations

import numpy as np


def to_f32(A: np.ndarray) -> np.ndarray:
    """A rounded elementwise to FP32, nearest even."""
    return np.asarray(A, dtype=np.float64).astype(np.float32)


def bf16_rne(a: np.ndarray) -> np.ndarray:
    """Nearest BF16 value of every element (ties to even), returned as float64.

    Write a = m * 2**e with 0.5 <= |m| < 1; the BF16 neighbours of a are the
    multiples of 2**(e - 8) (8 significant bits), so the rounded value is
    rint(m * 256) * 2**(e - 8), where rint rounds halves to the even integer."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)
    q = np.rint(m * 256.0)
    return np.ldexp(q, e - 8)


def to_bf16x2(A: np.ndarray):
    """(hi, lo) as float64 arrays: hi = bf16(A), lo = bf16(A - hi)."""
    A = np.asarray(A, dtype=np.float64)
    hi = bf16_rne(A)
    lo = bf16_rne(A - hi)
    return hi, lo


def bf16_bits(v: np.ndarray) -> np.ndarray:
    """uint16 BF16 bit patterns of float64 values that are exactly BF16 numbers."""
    f = np.asarray(v, dtype=np.float64).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """float64 values of uint16 BF16 bit patterns."""
    u = np.asarray(bits).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)
