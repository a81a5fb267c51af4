"""Exact Wigner 3j symbols for the oracle (test infrastructure only).

The coupling coefficients of the isotropic basis (Section 2.1, eq. basis-coupling)
are chains of Wigner 3j symbols.  The oracle evaluates each 3j symbol with the
Racah single-sum formula (DLMF 34.2.4) in exact rational arithmetic: the square of
the symbol is an exact Fraction, so the only rounding is one final square root.

Pinned against sympy.physics.wigner.wigner_3j (an independent implementation) in
tests/test_oracle_pins.py.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial, sqrt

__all__ = ["wigner3j", "wigner3j_sq_signed"]


def _triangle(a: int, b: int, c: int) -> bool:
    return abs(a - b) <= c <= a + b


@lru_cache(maxsize=None)
def wigner3j_sq_signed(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int):
    """Return (sign, square) with (j1 j2 j3; m1 m2 m3) = sign * sqrt(square).

    Integer angular momenta only (all the basis needs).  square is a Fraction.
    """
    if m1 + m2 + m3 != 0:
        return 0, Fraction(0)
    if not _triangle(j1, j2, j3):
        return 0, Fraction(0)
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0, Fraction(0)
    f = factorial
    # Triangle coefficient Delta(j1 j2 j3)
    delta = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3), f(j1 + j2 + j3 + 1))
    pref = f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3)
    # Racah sum over k: every factorial argument must be non-negative.
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for k in range(kmin, kmax + 1):
        den = (f(k) * f(j3 - j2 + k + m1) * f(j3 - j1 + k - m2) * f(j1 + j2 - j3 - k)
               * f(j1 - k - m1) * f(j2 - k + m2))
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0, Fraction(0)
    phase = -1 if (j1 - j2 - m3) % 2 else 1
    sign = phase * (1 if s > 0 else -1)
    return sign, delta * pref * s * s


@lru_cache(maxsize=None)
def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    """(j1 j2 j3; m1 m2 m3) as a float, correctly rounded up to one sqrt."""
    sign, sq = wigner3j_sq_signed(j1, j2, j3, m1, m2, m3)
    if sign == 0:
        return 0.0
    return sign * sqrt(sq)
