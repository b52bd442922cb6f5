"""Clebsch-Gordan coefficients for the oracle (test infrastructure).

The paper cites the two-body matrix elements without fixing conventions; the
oracle uses the textbook Condon-Shortley coefficients from Racah's closed
formula, evaluated in exact rational arithmetic and square-rooted last.
All angular momenta are passed doubled (2j, 2m).
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache


def _f(x2: int) -> int:
    """Factorial of x2/2 for an even doubled argument; -1 flags a negative argument."""
    if x2 % 2:
        raise ValueError("half-integer factorial argument")
    x = x2 // 2
    return -1 if x < 0 else math.factorial(x)


@lru_cache(maxsize=None)
def cg(tj1: int, tm1: int, tj2: int, tm2: int, tJ: int, tM: int) -> float:
    """<j1 m1 j2 m2 | J M> (Racah's formula), doubled arguments."""
    if tm1 + tm2 != tM:
        return 0.0
    if tJ < abs(tj1 - tj2) or tJ > tj1 + tj2 or (tj1 + tj2 + tJ) % 2:
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    if (tj1 + tm1) % 2 or (tj2 + tm2) % 2 or (tJ + tM) % 2:
        return 0.0
    pref = Fraction((tJ + 1) * _f(tj1 + tj2 - tJ) * _f(tj1 - tj2 + tJ) * _f(-tj1 + tj2 + tJ),
                    _f(tj1 + tj2 + tJ + 2))
    pref *= (_f(tj1 + tm1) * _f(tj1 - tm1) * _f(tj2 + tm2) * _f(tj2 - tm2) * _f(tJ + tM) * _f(tJ - tM))
    s = Fraction(0)
    for k in range(0, (tj1 + tj2) // 2 + 2):
        args = (2 * k, tj1 + tj2 - tJ - 2 * k, tj1 - tm1 - 2 * k, tj2 + tm2 - 2 * k,
                tJ - tj2 + tm1 + 2 * k, tJ - tj1 - tm2 + 2 * k)
        if min(args) < 0:
            continue
        den = 1
        for a in args:
            den *= _f(a)
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0.0
    val = math.sqrt(pref * s * s)
    return val if s > 0 else -val
