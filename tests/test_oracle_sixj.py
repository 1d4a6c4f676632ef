"""Pins of the oracle's exact 6j symbols against the textbook and an independent library.

* sympy's ``wigner_6j`` (an independent exact implementation) on a random sample;
* the 24 tetrahedral symmetries and the Regge symmetry;
* orthogonality  sum_x (2x+1)(2f+1) {a b x; c d f}{a b x; c d f'} = delta(f, f');
* the Racah sum rule  sum_x (-1)^{p+q+x} (2x+1) {a b x; c d p}{a b x; d c q} = {a c q; b d p};
* the Biedenharn-Elliott identity;
* the closed form {a b c; 0 c b} = (-1)^{a+b+c} / sqrt((2b+1)(2c+1)).
(Edmonds, "Angular Momentum in Quantum Mechanics", Ch. 6; Regge 1959.)
"""
import itertools
import math
import random

import pytest
from sympy import Rational
from sympy.physics.wigner import wigner_6j

from oracle.wigner import sixj, sixj_exact, triad, sqrt_fraction_to_float
from fractions import Fraction


def admissible(a, b, c, d, e, f):
    return triad(a, b, c) and triad(a, e, f) and triad(d, b, f) and triad(d, e, c)


def random_admissible(rng, top, count):
    out = []
    while len(out) < count:
        s = [rng.randint(0, top) for _ in range(6)]
        if admissible(*s):
            out.append(tuple(s))
    return out


def test_sqrt_rounding():
    assert sqrt_fraction_to_float(Fraction(2)) == math.sqrt(2.0)
    assert sqrt_fraction_to_float(Fraction(1, 3)) == math.sqrt(1.0 / 3.0)
    assert sqrt_fraction_to_float(Fraction(9, 4)) == 1.5


def test_against_sympy():
    rng = random.Random(7)
    for s in random_admissible(rng, 24, 150):
        # sympy's exact value, evaluated to 40 digits, then rounded once to FP64
        ref = float(wigner_6j(*[Rational(v, 2) for v in s]).evalf(40))
        assert sixj(*s) == ref, s


def test_non_admissible_is_zero():
    assert sixj(2, 2, 2, 2, 2, 9) == 0.0        # non-integer triad sum
    assert sixj(2, 2, 10, 2, 2, 2) == 0.0       # triangle violated


def tetrahedral_images(a, b, c, d, e, f):
    cols = [(a, d), (b, e), (c, f)]
    out = set()
    for perm in itertools.permutations(range(3)):
        pc = [cols[p] for p in perm]
        # swapping upper and lower entries in any two columns
        for flip in [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)]:
            top = [pc[n][flip[n]] for n in range(3)]
            bot = [pc[n][1 - flip[n]] for n in range(3)]
            out.add(tuple(top + bot))
    return out


def test_tetrahedral_symmetry():
    rng = random.Random(11)
    for s in random_admissible(rng, 16, 60):
        images = tetrahedral_images(*s)
        assert len(images) <= 24
        for img in images:
            assert sixj_exact(*img) == sixj_exact(*s)


def test_regge_symmetry():
    rng = random.Random(12)
    for a, b, c, d, e, f in random_admissible(rng, 18, 80):
        # {a b c; d e f} = {a, (b+c+e-f)/2, (b+c-e+f)/2; d, (e+f+b-c)/2, (e+f-b+c)/2}
        img = (a, (b + c + e - f) // 2, (b + c - e + f) // 2, d, (e + f + b - c) // 2, (e + f - b + c) // 2)
        assert sixj(*img) == pytest.approx(sixj(a, b, c, d, e, f), rel=1e-15, abs=1e-300)


def test_orthogonality():
    for a, b, c, d in [(2, 4, 3, 5), (6, 6, 6, 6), (1, 4, 3, 2), (8, 5, 7, 4), (10, 10, 6, 8)]:
        fs = [f for f in range(0, 40) if any(admissible(a, b, x, c, d, f) for x in range(0, 40))]
        xs = range(0, 40)
        for f in fs:
            for g in fs:
                s = math.fsum((x + 1) * (f + 1) * sixj(a, b, x, c, d, f) * sixj(a, b, x, c, d, g) for x in xs)
                assert s == pytest.approx(1.0 if f == g else 0.0, abs=1e-13), (a, b, c, d, f, g)


def test_racah_sum_rule():
    rng = random.Random(3)
    n = 0
    while n < 40:
        a, b, c, d, p, q = (rng.randint(0, 10) for _ in range(6))
        if not admissible(a, c, q, b, d, p):
            continue
        n += 1
        lhs = math.fsum((-1) ** ((p + q + x) // 2) * (x + 1) * sixj(a, b, x, c, d, p) * sixj(a, b, x, d, c, q)
                        for x in range(0, 30) if (p + q + x) % 2 == 0)
        assert lhs == pytest.approx(sixj(a, c, q, b, d, p), abs=1e-13)


def test_biedenharn_elliott():
    rng = random.Random(5)
    n = 0
    while n < 30:
        a, b, c, d, e, f, p, q, r = (rng.randint(0, 8) for _ in range(9))
        rhs = sixj(p, q, r, e, a, d) * sixj(p, q, r, f, b, c)
        if not (admissible(p, q, r, e, a, d) and admissible(p, q, r, f, b, c)):
            continue
        n += 1
        s2 = a + b + c + d + e + f + p + q + r
        lhs = math.fsum((-1) ** ((s2 + x) // 2) * (x + 1) * sixj(a, b, x, c, d, p) * sixj(c, d, x, e, f, q)
                        * sixj(e, f, x, b, a, r) for x in range(0, 30) if (s2 + x) % 2 == 0)
        assert lhs == pytest.approx(rhs, abs=1e-13), (a, b, c, d, e, f, p, q, r)


def test_closed_form_zero_entry():
    for a in range(0, 9):
        for b in range(0, 9):
            for c in range(0, 9):
                if not triad(a, b, c):
                    continue
                ref = (-1) ** ((a + b + c) // 2) / math.sqrt((b + 1) * (c + 1))
                assert sixj(a, b, c, 0, c, b) == pytest.approx(ref, rel=1e-15)
