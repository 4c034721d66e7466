"""Exact rational round-to-nearest-even into binary formats (test helper).

Written from the IEEE 754 definition with Python's ``fractions``; it shares no
code with the oracle and is used to pin the oracle's FMA emulation.
"""
from fractions import Fraction
import math

HALF = (10, -14, 15)     # (fraction bits, emin, emax)
SINGLE = (23, -126, 127)


def rne(q: Fraction, fmt=HALF) -> float:
    mbits, emin, emax = fmt
    if q == 0:
        return 0.0
    s = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    ulp = Fraction(2) ** (e - mbits)
    k = a / ulp
    fl = math.floor(k)
    rem = k - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    v = fl * ulp
    if v >= Fraction(2) ** (emax + 1):
        return s * math.inf
    return s * float(v)
