"""The {15j} symbol of the first kind, eq. (15j) (oracle; test infrastructure only).

Eq. (15j) writes the symbol with rows

    ( i1   j14  k4   l24  k2  )
    ( j15  l45  l34  l23  j12 )
    ( l25  k5   l35  k3   j13 )

as a single sum over x of (2x+1), a phase, and five 6j symbols

    {i1 l25 x; k5 j14 j15} {j14 k5 x; l35 k4 l45} {k4 l35 x; k3 l24 l34}
    {l24 k3 x; j13 k2 l23} {k2 j13 x; i1 l25 j12}.

The phase is printed garbled in the source.  It is read here as (-1)^R with R the sum of all
fifteen entries, the phase of the general first-kind 3nj symbol, whose x-dependent part
(-1)^{(n-1) x} is 1 for n = 5.  R is an integer: the fifteen entries split into the five
closed triads (i1 j12 j13), (k2 l23 l24), (k3 l34 l35), (k4 j14 l45), (k5 j15 l25).

x runs in unit steps over the values allowed by the five triads that contain it:
(i1 l25 x), (k5 j14 x), (l35 k4 x), (l24 k3 x), (j13 k2 x).
"""
import numpy as np

from .wigner import sixj, triad
from .ranges import LINK

__all__ = ["fifteenj", "x_range", "phase15"]


def _j(two_l, name):
    return two_l[LINK[name]]


def x_range(two_i1, two_k2, two_k3, two_k4, two_k5, two_l):
    """List of two_x allowed by all five x triads (may be empty)."""
    pairs = [(two_i1, _j(two_l, "25")), (two_k5, _j(two_l, "14")), (_j(two_l, "35"), two_k4),
             (_j(two_l, "24"), two_k3), (_j(two_l, "13"), two_k2)]
    lo = max(abs(a - b) for a, b in pairs)
    hi = min(a + b for a, b in pairs)
    return [x for x in range(lo, hi + 1, 2) if all(triad(a, b, x) for a, b in pairs)]


def phase15(two_i1, two_k2, two_k3, two_k4, two_k5, two_l):
    """(-1)^R, R = sum of all fifteen entries of the symbol."""
    two_r = two_i1 + two_k2 + two_k3 + two_k4 + two_k5 + sum(two_l)
    assert two_r % 2 == 0, "the fifteen entries must have an integer sum"
    return -1 if (two_r // 2) % 2 else 1


def fifteenj(two_i1, two_k2, two_k3, two_k4, two_k5, two_l):
    """{15j} of eq. (15j) in FP64; ``two_l`` are the ten virtual spins in link order.

    The first four entries of ``two_l`` are the gauge-fixed j12..j15.
    """
    l = lambda n: _j(two_l, n)  # noqa: E731
    total = 0.0
    for x in x_range(two_i1, two_k2, two_k3, two_k4, two_k5, two_l):
        total += ((x + 1)
                  * sixj(two_i1, l("25"), x, two_k5, l("14"), l("15"))
                  * sixj(l("14"), two_k5, x, l("35"), two_k4, l("45"))
                  * sixj(two_k4, l("35"), x, two_k3, l("24"), l("34"))
                  * sixj(l("24"), two_k3, x, l("13"), two_k2, l("23"))
                  * sixj(two_k2, l("13"), x, two_i1, l("25"), l("12")))
    return phase15(two_i1, two_k2, two_k3, two_k4, two_k5, two_l) * total


def fifteenj_block(ranges_i1, ranges_k, two_l):
    """W[i1, k2, k3, k4, k5] for one shell: step 6(i) of the framed algorithm, Sec. 3.1.

    ``ranges_i1`` = (two_lo, dim) of i1, ``ranges_k`` = four (two_lo, dim) for k2..k5.
    The five 6j slices are tabulated over a common x window and summed with ``einsum``;
    entries outside a triad are zero, so the window only has to contain every allowed x.
    """
    (i_lo, i_n), ((k2_lo, k2_n), (k3_lo, k3_n), (k4_lo, k4_n), (k5_lo, k5_n)) = ranges_i1, ranges_k
    l = lambda n: _j(two_l, n)  # noqa: E731
    i1s = [i_lo + 2 * a for a in range(i_n)]
    k2s = [k2_lo + 2 * a for a in range(k2_n)]
    k3s = [k3_lo + 2 * a for a in range(k3_n)]
    k4s = [k4_lo + 2 * a for a in range(k4_n)]
    k5s = [k5_lo + 2 * a for a in range(k5_n)]
    # x window: union over the index ranges of each x-triad, intersected over the triads.
    lo = max(min(abs(a - l("25")) for a in i1s), min(abs(a - l("14")) for a in k5s),
             min(abs(a - l("35")) for a in k4s), min(abs(a - l("24")) for a in k3s),
             min(abs(a - l("13")) for a in k2s))
    hi = min(max(a + l("25") for a in i1s), max(a + l("14") for a in k5s),
             max(a + l("35") for a in k4s), max(a + l("24") for a in k3s),
             max(a + l("13") for a in k2s))
    shape = (i_n, k2_n, k3_n, k4_n, k5_n)
    if lo > hi:
        return np.zeros(shape)
    xs = list(range(lo, hi + 1, 2))
    nx = len(xs)
    s1 = np.array([[[sixj(a, l("25"), x, e, l("14"), l("15")) for x in xs] for e in k5s] for a in i1s]).reshape(i_n, k5_n, nx)
    s2 = np.array([[[sixj(l("14"), e, x, l("35"), d, l("45")) for x in xs] for d in k4s] for e in k5s]).reshape(k5_n, k4_n, nx)
    s3 = np.array([[[sixj(d, l("35"), x, c, l("24"), l("34")) for x in xs] for c in k3s] for d in k4s]).reshape(k4_n, k3_n, nx)
    s4 = np.array([[[sixj(l("24"), c, x, l("13"), b, l("23")) for x in xs] for b in k2s] for c in k3s]).reshape(k3_n, k2_n, nx)
    s5 = np.array([[[sixj(b, l("13"), x, a, l("25"), l("12")) for x in xs] for a in i1s] for b in k2s]).reshape(k2_n, i_n, nx)
    dimx = np.array([x + 1 for x in xs], dtype=np.float64)
    w = np.einsum("aex,edx,dcx,cbx,bax,x->abcde", s1, s2, s3, s4, s5, dimx)
    # (-1)^R factorises over the five intertwiners and the ten spins.
    base = sum(two_l) + i_lo + k2_lo + k3_lo + k4_lo + k5_lo
    assert base % 2 == 0
    sign0 = -1.0 if (base // 2) % 2 else 1.0
    alt = [np.array([(-1.0) ** n for n in range(m)]) for m in shape]
    ph = sign0 * np.einsum("a,b,c,d,e->abcde", *alt)
    return w * ph
