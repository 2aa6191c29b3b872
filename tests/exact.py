"""Exact rational/integer helpers used to pin the oracle independently of its C code.

Python integers and fractions.Fraction are exact, so these re-derive the
integer decisions the paper defines (round-to-nearest of a real magnitude,
round-half-up of a real level coordinate) by a different method than the
oracle's floating-point + expansion arithmetic.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction


def f32(v: float) -> float:
    return struct.unpack("<f", struct.pack("<f", v))[0]


def f32_bits(v: float) -> int:
    return struct.unpack("<I", struct.pack("<f", v))[0]


def exact_sq_norm(x: float, y: float, z: float) -> Fraction:
    return Fraction(x) ** 2 + Fraction(y) ** 2 + Fraction(z) ** 2


def floor_log2(S: Fraction) -> int:
    """floor(log2 S) for rational S > 0."""
    n, d = S.numerator, S.denominator
    k = n.bit_length() - d.bit_length()
    if k >= 0:
        if n < (d << k):
            k -= 1
    elif (n << -k) < d:
        k -= 1
    return k


def round_sqrt(S: Fraction, prec: int, min_spacing: Fraction | None = None) -> Fraction:
    """Exact round-to-nearest-even of sqrt(S) to `prec` significant bits; the grid
    spacing is never finer than `min_spacing` (gradual underflow)."""
    if S == 0:
        return Fraction(0)
    e = floor_log2(S) // 2                      # 2^e <= sqrt(S) < 2^(e+1)
    u = Fraction(2) ** (e - (prec - 1))
    if min_spacing is not None and u < min_spacing:
        u = min_spacing
    T = S / (u * u)                             # sqrt(T) = sqrt(S)/u
    j = math.isqrt(T.numerator // T.denominator)   # floor(sqrt(T))
    mid = Fraction(2 * j + 1, 2)
    if T > mid * mid:
        j += 1
    elif T == mid * mid and j % 2 == 1:
        j += 1
    return j * u


def nint(v: Fraction) -> int:
    """Round half up: ceil(floor(2v)/2) (§2.1)."""
    return math.ceil(Fraction(math.floor(2 * v), 2))
