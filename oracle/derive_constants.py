"""Exact derivation of the binary32 constants of cospi_f32 / exp_f32.

Each constant is defined mathematically and rounded once to the nearest
binary32 (ties to even):
  cos(pi a) = sum_k (-1)^k pi^(2k) a^(2k) / (2k)!        k = 0..5
  sin(pi a) = sum_k (-1)^k pi^(2k+1) a^(2k+1) / (2k+1)!  k = 0..4
  exp(r)    = sum_k r^k / k!                              k = 0..8
  LN2_HI = rn(ln 2), LN2_LO = rn(ln 2 - LN2_HI), LOG2E = rn(1 / ln 2)
pi comes from Machin's formula and ln 2 from sum 1/(k 2^k), both in exact
rational arithmetic to far more digits than binary32 needs.  Test
infrastructure: the oracle tests compare the constants in pso_oracle.c with
these values.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction


def pi_fraction(digits: int = 60) -> Fraction:
    scale = 10 ** (digits + 10)

    def atan_inv(x: int) -> int:
        total, term, n, sign, x2 = 0, scale // x, 1, 1, x * x
        while term:
            total += sign * (term // n)
            term //= x2
            n += 2
            sign = -sign
        return total

    return Fraction(16 * atan_inv(5) - 4 * atan_inv(239), scale)


def ln2_fraction(terms: int = 240) -> Fraction:
    return sum((Fraction(1, k * 2 ** k) for k in range(1, terms)), Fraction(0))


def _f32_bits_to_float(b: int) -> float:
    return struct.unpack("<f", struct.pack("<I", b))[0]


def round_f32(q: Fraction) -> float:
    """Round an exact rational to the nearest binary32 (ties to even)."""
    if q == 0:
        return 0.0
    sign = -1.0 if q < 0 else 1.0
    a = abs(q)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    # fix e so that 2^e <= a < 2^(e+1)
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp
    n = math.floor(m)
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * float(n * ulp)


def cos_pi_coeffs():
    pi = pi_fraction()
    return [round_f32((-1) ** k * pi ** (2 * k) / math.factorial(2 * k)) for k in range(6)]


def sin_pi_coeffs():
    pi = pi_fraction()
    return [round_f32((-1) ** k * pi ** (2 * k + 1) / math.factorial(2 * k + 1)) for k in range(5)]


def exp_coeffs():
    return [round_f32(Fraction(1, math.factorial(k))) for k in range(9)]


def ln2_split():
    ln2 = ln2_fraction()
    hi = round_f32(ln2)
    lo = round_f32(ln2 - Fraction(hi))
    return hi, lo, round_f32(1 / ln2)


if __name__ == "__main__":
    print("cos", [c.hex() for c in cos_pi_coeffs()])
    print("sin", [c.hex() for c in sin_pi_coeffs()])
    print("exp", [c.hex() for c in exp_coeffs()])
    print("ln2_hi, ln2_lo, log2e", [c.hex() for c in ln2_split()])
