"""Exact SU(2) 6j symbols by the Racah formula (oracle; test infrastructure only).

The paper evaluates its 6j symbols with exact multiword arithmetic (Sec. 3, first paragraph:
the WIGXJPF / FASTWIGXJ libraries).  The oracle does the same thing in the plainest possible
way: Python big integers and ``fractions.Fraction``, rounded once to the nearest FP64 value.

All spins are passed as *twice* their value (``two_a = 2 a``), so half-integers are exact.

Racah's single-sum formula (Racah 1942; Edmonds, "Angular Momentum in Quantum Mechanics",
Sec. 6.3):

    {a b c}  = D(abc) D(aef) D(dbf) D(dec)
    {d e f}    * sum_t (-1)^t (t+1)! / [ (t-a-b-c)! (t-a-e-f)! (t-d-b-f)! (t-d-e-c)!
                                         (a+b+d+e-t)! (a+c+d+f-t)! (b+c+e+f-t)! ]

    D(abc)^2 = (a+b-c)! (a-b+c)! (-a+b+c)! / (a+b+c+1)!

The symbol vanishes unless the four triads (abc), (aef), (dbf), (dec) satisfy the triangle
inequalities with an integer sum.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial, isqrt

__all__ = ["triad", "sixj_exact", "sixj", "sqrt_fraction_to_float"]


def triad(two_a: int, two_b: int, two_c: int) -> bool:
    """True when (a, b, c) close a triangle with an integer sum a + b + c."""
    if two_a < 0 or two_b < 0 or two_c < 0:
        return False
    if (two_a + two_b + two_c) % 2:
        return False
    return abs(two_a - two_b) <= two_c <= two_a + two_b


@lru_cache(maxsize=None)
def _fact(n: int) -> int:
    return factorial(n)


def _delta_sq(two_a: int, two_b: int, two_c: int) -> Fraction:
    """D(abc)^2 as an exact rational (all arguments in two-units, triad assumed valid)."""
    return Fraction(
        _fact((two_a + two_b - two_c) // 2)
        * _fact((two_a - two_b + two_c) // 2)
        * _fact((-two_a + two_b + two_c) // 2),
        _fact((two_a + two_b + two_c) // 2 + 1),
    )


@lru_cache(maxsize=None)
def sixj_exact(two_a: int, two_b: int, two_c: int, two_d: int, two_e: int, two_f: int):
    """Return ``(S, P)`` with {a b c; d e f} = S * sqrt(P) exactly.

    ``S`` is the (signed) Racah sum, ``P`` the product of the four squared triangle
    coefficients; both are ``Fraction``.  ``(0, 0)`` when a triad fails.
    """
    if not (triad(two_a, two_b, two_c) and triad(two_a, two_e, two_f)
            and triad(two_d, two_b, two_f) and triad(two_d, two_e, two_c)):
        return Fraction(0), Fraction(0)
    a1 = (two_a + two_b + two_c) // 2
    a2 = (two_a + two_e + two_f) // 2
    a3 = (two_d + two_b + two_f) // 2
    a4 = (two_d + two_e + two_c) // 2
    b1 = (two_a + two_b + two_d + two_e) // 2
    b2 = (two_a + two_c + two_d + two_f) // 2
    b3 = (two_b + two_c + two_e + two_f) // 2
    s = Fraction(0)
    for t in range(max(a1, a2, a3, a4), min(b1, b2, b3) + 1):
        num = _fact(t + 1)
        den = (_fact(t - a1) * _fact(t - a2) * _fact(t - a3) * _fact(t - a4)
               * _fact(b1 - t) * _fact(b2 - t) * _fact(b3 - t))
        s += Fraction(-num if t % 2 else num, den)
    p = (_delta_sq(two_a, two_b, two_c) * _delta_sq(two_a, two_e, two_f)
         * _delta_sq(two_d, two_b, two_f) * _delta_sq(two_d, two_e, two_c))
    return s, p


def sqrt_fraction_to_float(q: Fraction) -> float:
    """Correctly rounded FP64 value of sqrt(q) for a non-negative rational q."""
    if q < 0:
        raise ValueError("negative argument")
    if q == 0:
        return 0.0
    p, d = q.numerator, q.denominator
    # Scale so that the integer square root carries at least 70 significant bits.
    k = max(0, (140 - (p.bit_length() - d.bit_length())) // 2 + 1)
    n = p << (2 * k)
    y = isqrt(n // d)
    if y * y * d != n:
        # Not exact: append a sticky bit so the final rounding to 53 bits is correct.
        y = (y << 1) | 1
        k += 1
    return float(Fraction(y, 1 << k))


@lru_cache(maxsize=None)
def sixj(two_a: int, two_b: int, two_c: int, two_d: int, two_e: int, two_f: int) -> float:
    """{a b c; d e f} rounded once to the nearest FP64 number."""
    s, p = sixj_exact(two_a, two_b, two_c, two_d, two_e, two_f)
    if s == 0:
        return 0.0
    mag = sqrt_fraction_to_float(s * s * p)
    return mag if s > 0 else -mag
