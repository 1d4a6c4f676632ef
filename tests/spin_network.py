"""Brute-force SU(2) spin-network evaluation from Wigner 3jm symbols (test helper).

Independent of the oracle: 3jm values come from sympy, and the {15j} / BF vertex is obtained
by summing over every magnetic number of the 4-simplex boundary graph, not from 6j symbols.

A normalised 4-valent intertwiner on links (p q)(r s) with virtual spin i is

    iota_i[m_p, m_q, m_r, m_s] = sqrt(2i+1) sum_m (-1)^{i-m} (p q i; m_p m_q m) (i r s; -m m_r m_s)

(orthonormal in i).  The 4-simplex evaluation contracts the five node intertwiners along the
ten links, with the link metric (-1)^{j-m} delta(m, -m'): the magnetic index of link ab enters
node a as m and node b as -m.
"""
from functools import lru_cache

import numpy as np
from sympy import Rational
from sympy.physics.wigner import wigner_3j

LINKS = ("12", "13", "14", "15", "23", "24", "25", "34", "35", "45")
EDGE_LINKS = {
    1: ("12", "13", "14", "15"),
    2: ("23", "24", "25", "12"),
    3: ("34", "35", "13", "23"),
    4: ("45", "14", "24", "34"),
    5: ("15", "25", "35", "45"),
}


@lru_cache(maxsize=None)
def w3j(two_a, two_b, two_c, two_ma, two_mb, two_mc):
    if two_ma + two_mb + two_mc != 0:
        return 0.0
    return float(wigner_3j(Rational(two_a, 2), Rational(two_b, 2), Rational(two_c, 2),
                           Rational(two_ma, 2), Rational(two_mb, 2), Rational(two_mc, 2)))


def _ms(two_j):
    return list(range(-two_j, two_j + 1, 2))


@lru_cache(maxsize=None)
def intertwiner(two_p, two_q, two_r, two_s, two_i):
    """iota_i as a dense array over (m_p, m_q, m_r, m_s), m ascending."""
    out = np.zeros((two_p + 1, two_q + 1, two_r + 1, two_s + 1))
    for a, mp in enumerate(_ms(two_p)):
        for b, mq in enumerate(_ms(two_q)):
            m = -(mp + mq)
            if abs(m) > two_i:
                continue
            for c, mr in enumerate(_ms(two_r)):
                for d, ms in enumerate(_ms(two_s)):
                    if mr + ms != m:
                        continue
                    ph = -1.0 if ((two_i - m) // 2) % 2 else 1.0
                    out[a, b, c, d] = ph * w3j(two_p, two_q, two_i, mp, mq, m) * w3j(two_i, two_r, two_s, -m, mr, ms)
    return out * np.sqrt(two_i + 1.0)


def simplex_evaluation(two_spins, two_intertwiners):
    """Contract five normalised intertwiners (node e on its four links) along the ten links.

    ``two_spins`` maps link name -> two_j, ``two_intertwiners`` is [two_i1 .. two_i5].
    """
    letters = {name: chr(ord("a") + n) for n, name in enumerate(LINKS)}
    ops = []
    specs = []
    for e in range(1, 6):
        names = EDGE_LINKS[e]
        t = intertwiner(*(two_spins[n] for n in names), two_intertwiners[e - 1])
        # Node e is the first endpoint of link "ab" when e == a: it takes m; else -m.
        for axis, name in enumerate(names):
            if int(name[0]) != e:
                t = np.flip(t, axis=axis)       # index by m of the link, entry uses -m
        ops.append(t)
        specs.append("".join(letters[n] for n in names))
    for name in LINKS:
        two_j = two_spins[name]
        ops.append(np.array([-1.0 if ((two_j - m) // 2) % 2 else 1.0 for m in _ms(two_j)]))
        specs.append(letters[name])
    return float(np.einsum(",".join(specs) + "->", *ops, optimize="greedy"))


def simplex_tensor(two_spins, node_stacks):
    """Like ``simplex_evaluation`` but each node carries a stack of 4-valent tensors.

    ``node_stacks[e-1]`` has shape (n_e, m_p, m_q, m_r, m_s) on the links of node e; the result
    is the 5-index tensor over the stack indices of nodes 1..5.
    """
    letters = {name: chr(ord("a") + n) for n, name in enumerate(LINKS)}
    outs = "vwxyz"
    ops, specs = [], []
    for e in range(1, 6):
        names = EDGE_LINKS[e]
        t = node_stacks[e - 1]
        for axis, name in enumerate(names):
            if int(name[0]) != e:
                t = np.flip(t, axis=axis + 1)
        ops.append(t)
        specs.append(outs[e - 1] + "".join(letters[n] for n in names))
    for name in LINKS:
        two_j = two_spins[name]
        ops.append(np.array([-1.0 if ((two_j - m) // 2) % 2 else 1.0 for m in _ms(two_j)]))
        specs.append(letters[name])
    return np.einsum(",".join(specs) + "->" + outs, *ops, optimize="greedy")


def intertwiner_stack(two_p, two_q, two_r, two_s):
    """(two_lo, stack) of all normalised intertwiners of (p q)(r s), ascending."""
    lo = max(abs(two_p - two_q), abs(two_r - two_s))
    hi = min(two_p + two_q, two_r + two_s)
    vals = list(range(lo, hi + 1, 2))
    return lo, np.stack([intertwiner(two_p, two_q, two_r, two_s, i) for i in vals])
