"""Booster functions of eq. (booster) by FP64 quadrature (oracle; test infrastructure only).

The booster of an edge with boundary spins j_1..j_4 (intertwiner i) and virtual spins
l_1..l_4 (intertwiner k) is

    B4 = sum_{m_1..m_4} 4jm(j; m; i) 4jm(l; m; k)
           * int_0^inf dr sinh^2(r) / (4 pi) prod_a d^{(rho_a, k_a)}_{j_a l_a m_a}(r)

with the Y-map (rho_a, k_a) = (gamma (j_a + 1), j_a) of eq. (booster).  The paper evaluates the
boost matrix elements d by a finite sum of exponentials whose coefficients it does not print,
so they are computed here from a definition that can be checked by hand:

* SL(2,C) principal series (rho, k) on functions on SU(2) with left covariance k, canonical
  basis sqrt(2j+1) D^j_{k m}(u).  A boost h_r = diag(e^{r/2}, e^{-r/2}) acts as
  f(u) -> lambda^{2 i rho - 2} f(u'), where u h_r = b u' (b lower triangular, first diagonal
  entry lambda > 0); it keeps the Euler angles alpha, gamma of u and maps the polar angle by
  cos(beta'/2) = e^{r/2} cos(beta/2) / lambda.  The modulus lambda^{-2} is the square root of
  the Jacobian of beta -> beta', so the action is unitary.  With s = log(lambda^2) this gives

      d_{jlm}(r) = sqrt((2j+1)(2l+1)) / (2 sinh r) * int_{-r}^{r} ds e^{i rho s}
                   d^j_{km}(beta(s)) d^l_{km}(beta'(s)),
      cos^2(beta/2) = (e^s - e^{-r}) / (2 sinh r),  sin^2(beta/2) = (e^r - e^s) / (2 sinh r),
      cos^2(beta'/2) = e^{r-s} cos^2(beta/2),       sin^2(beta'/2) = e^{-r-s} sin^2(beta/2),

  evaluated by Gauss-Legendre quadrature in s (the integrand is analytic in s).  For k = 0 and
  j = l = 0 it reduces to the spherical function sin(rho r) / (rho sinh r).
* SU(2) small d^j(beta) = exp(-i beta J_y) in the |j m> basis (Condon-Shortley phases), from
  the eigendecomposition of J_y (the eigenvalues are -j..j), stable in FP64.
* 3jm by Racah's formula in exact rational arithmetic, rounded once; 4jm couples the first two
  and the last two spins: 4jm(j; m; i) = (-1)^(i - m) (j1 j2 i; m1 m2 m)(i j3 j4; -m m3 m4),
  m = -(m1 + m2).
* The r integral follows the booster quadrature of Sec. 3.1: u = e^{-r} maps it to (0, 1],
  which is cut into n subintervals growing linearly from u = 0 (|I_k| = k * 2 / (n (n+1))).
  Each subinterval gets Gauss-Legendre rules of 30 and 61 points (the paper's Gauss-Kronrod
  pair nests its nodes; two Gauss rules serve the same purpose), the sum of the 61-point
  results is the value and the sum of |G61 - G30| the error estimate; n doubles until the
  estimate is below the tolerance.

All spins are passed as twice their value.  Boosters of a configuration are returned in the
packed layout of ``ranges.booster_layout`` (edge 2..5, offset triple, rows i, columns k).
"""
from fractions import Fraction
from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np

from . import ranges as R
from .wigner import sqrt_fraction_to_float

__all__ = ["threejm", "fourjm", "su2_d", "boost_d", "booster_block", "boosters"]


@lru_cache(maxsize=None)
def _f(n):
    return factorial(n)


@lru_cache(maxsize=None)
def threejm(two_j1, two_j2, two_j3, two_m1, two_m2, two_m3):
    """Wigner 3jm symbol (j1 j2 j3; m1 m2 m3) by Racah's formula, exact then rounded."""
    if two_m1 + two_m2 + two_m3 != 0:
        return 0.0
    if any(abs(m) > j for m, j in ((two_m1, two_j1), (two_m2, two_j2), (two_m3, two_j3))):
        return 0.0
    if any((j - m) % 2 for m, j in ((two_m1, two_j1), (two_m2, two_j2), (two_m3, two_j3))):
        return 0.0
    if (two_j1 + two_j2 + two_j3) % 2 or not abs(two_j1 - two_j2) <= two_j3 <= two_j1 + two_j2:
        return 0.0
    a, b, c = two_j1, two_j2, two_j3
    tri = Fraction(_f((a + b - c) // 2) * _f((a - b + c) // 2) * _f((-a + b + c) // 2),
                   _f((a + b + c) // 2 + 1))
    mfac = 1
    for j, m in ((a, two_m1), (b, two_m2), (c, two_m3)):
        mfac *= _f((j + m) // 2) * _f((j - m) // 2)
    total = Fraction(0)
    # t runs where every factorial argument is non-negative.
    t_lo = max(0, (b - c - two_m1) // 2, (a - c + two_m2) // 2)
    t_hi = min((a + b - c) // 2, (a - two_m1) // 2, (b + two_m2) // 2)
    for t in range(t_lo, t_hi + 1):
        den = (_f(t) * _f((c - b + 2 * t + two_m1) // 2)
               * _f((c - a + 2 * t - two_m2) // 2) * _f((a + b - c - 2 * t) // 2)
               * _f((a - 2 * t - two_m1) // 2) * _f((b - 2 * t + two_m2) // 2))
        total += Fraction((-1) ** t, den)
    if total == 0:
        return 0.0
    phase = -1 if ((a - b - two_m3) // 2) % 2 else 1
    sign = phase * (1 if total > 0 else -1)
    return sign * sqrt_fraction_to_float(tri * mfac * total * total)


def fourjm(two_j, two_m, two_i):
    """4jm(j1 j2 j3 j4; m1 m2 m3 m4)^(i): (j1 j2) coupled to i, then i with (j3 j4)."""
    two_mi = -(two_m[0] + two_m[1])
    if two_mi - two_m[2] - two_m[3] != 0:
        return 0.0
    phase = -1 if ((two_i - two_mi) // 2) % 2 else 1
    return phase * (threejm(two_j[0], two_j[1], two_i, two_m[0], two_m[1], two_mi)
                    * threejm(two_i, two_j[2], two_j[3], -two_mi, two_m[2], two_m[3]))


@lru_cache(maxsize=None)
def _jy_modes(two_j):
    """Eigenvectors W and eigenvalues mu of J_y (basis m = j, j-1, .., -j)."""
    n = two_j + 1
    jp = np.zeros((n, n))
    for a in range(1, n):          # J+ |m> = sqrt((j-m)(j+m+1)) |m+1>, m = j - a
        two_m = two_j - 2 * a
        jp[a - 1, a] = np.sqrt((two_j - two_m) * (two_j + two_m + 2)) / 2
    jy = (jp - jp.T) / 2j          # J_y = (J+ - J-) / (2i)
    mu, w = np.linalg.eigh(jy)
    return mu, w


def su2_d(two_j, two_mp, two_m, beta):
    """d^j_{m' m}(beta) = <j m'| exp(-i beta J_y) |j m> on an array of angles."""
    mu, w = _jy_modes(two_j)
    a, b = (two_j - two_mp) // 2, (two_j - two_m) // 2
    coef = w[a, :] * np.conj(w[b, :])
    val = np.exp(-1j * np.multiply.outer(beta, mu)) @ coef
    return val.real


@lru_cache(maxsize=None)
def _gauss(n):
    return np.polynomial.legendre.leggauss(n)


def boost_d(rho, two_k, two_j, two_l, two_m, r, n_s=256):
    """SL(2,C) boost matrix element d^{(rho,k)}_{j l m}(r) (see the module docstring) on an
    array of rapidities r > 0, by n_s-point Gauss-Legendre quadrature in s."""
    r = np.asarray(r, dtype=float)
    x, w = _gauss(n_s)
    s = np.multiply.outer(r, x)                       # (n_r, n_s) nodes on [-r, r]
    rc = r[:, None]
    sh2 = 2 * np.sinh(rc)
    # e^s - e^-r = e^-r expm1(r (1 + x)) and e^r - e^s = e^s expm1(r (1 - x)): no cancellation
    # at small r.
    ep = np.expm1(np.multiply.outer(r, 1 + x))
    em = np.expm1(np.multiply.outer(r, 1 - x))
    c2 = np.exp(-rc) * ep / sh2                       # cos^2(beta/2)
    s2 = np.exp(s) * em / sh2                         # sin^2(beta/2)
    c2p = np.exp(-s) * ep / sh2                       # cos^2(beta'/2) = e^(r-s) cos^2(beta/2)
    s2p = np.exp(-rc) * em / sh2                      # sin^2(beta'/2) = e^(-r-s) sin^2(beta/2)
    beta = 2 * np.arctan2(np.sqrt(s2), np.sqrt(c2))
    betap = 2 * np.arctan2(np.sqrt(s2p), np.sqrt(c2p))
    dj = su2_d(two_j, two_k, two_m, beta)
    dl = su2_d(two_l, two_k, two_m, betap)
    integ = np.exp(1j * rho * s) * dj * dl
    val = (integ @ w) * r / (2 * np.sinh(r))
    # Phase convention.  Relative to this realisation, basis vector l carries the phase
    # arg Gamma(l + 1 + i rho): the factor exp(-i sum_{n=j+1}^{l} arg(n + i rho)) makes the
    # generator's off-diagonal elements purely imaginary (Naimark's canonical basis) and
    # d_{j l -m} = conj(d_{j l m}).  The further factor i^(j - l) = (-1)^((j - l)/2) gives
    # d_{j l -m} = (-1)^(l - j) conj(d_{j l m}), the symmetry of the two sums of the paper's
    # finite-sum formula (Sec. 3.1), under which the boosters come out real.
    phase = sum(np.arctan2(rho, n / 2) for n in range(two_j + 2, two_l + 1, 2))
    phase += np.pi / 2 * ((two_l - two_j) // 2)
    return np.sqrt((two_j + 1) * (two_l + 1)) * val * np.exp(-1j * phase)


def _r_nodes(n):
    """Nodes and weights (in r, including the 1/u of dr = -du/u) of the two rules on the n
    linearly growing subintervals of u in (0, 1]; returns (r30, w30, r61, w61)."""
    dx = 2.0 / (n * (n + 1))
    out = []
    for npts in (30, 61):
        x, w = _gauss(npts)
        rs, ws = [], []
        lo = 0.0
        for k in range(1, n + 1):
            hi = lo + k * dx if k < n else 1.0
            u = lo + (hi - lo) * (x + 1) / 2
            rs.append(-np.log(u))
            ws.append(w * (hi - lo) / 2 / u)
            lo = hi
        out += [np.concatenate(rs), np.concatenate(ws)]
    return out


def _edge_spins(two_j, dl, e, triple):
    """(boundary spins, virtual spins) of the four links of edge e for an offset triple."""
    two_l = list(two_j)
    for name, o in zip(R.EDGE_TRIPLE[e], triple):
        two_l[R.LINK[name]] += 2 * o
    links = R.EDGE_LINKS[e]
    return [two_j[R.LINK[n]] for n in links], [two_l[R.LINK[n]] for n in links]


def _block_from_d(jb, lb, dfun, weights, two_i_range, two_k_range):
    """One booster block from tabulated d functions: dfun[(two_j, two_l, two_m)] -> values on
    the r nodes, weights including sinh^2 r / (4 pi)."""
    ilo, idim = two_i_range
    klo, kdim = two_k_range
    out = np.zeros((idim, kdim), dtype=complex)
    for ms in product(*(range(-j, j + 1, 2) for j in jb)):
        if sum(ms) != 0:
            continue
        ci = [fourjm(jb, ms, ilo + 2 * a) for a in range(idim)]
        ck = [fourjm(lb, ms, klo + 2 * b) for b in range(kdim)]
        if not any(ci) or not any(ck):
            continue
        f = weights.copy()
        for a in range(4):
            f = f * dfun[(jb[a], lb[a], ms[a])]
        integral = f.sum()
        out += np.multiply.outer(np.array(ci), np.array(ck)) * integral
    return out


def booster_block(two_jb, two_lb, two_i_range, two_k_range, gamma, tol=1e-13, n0=16,
                  n_max=512, n_s=256):
    """B4 block (rows: i of (j1 j2)(j3 j4), columns: k of (l1 l2)(l3 l4)) for one edge.

    Returns (block, error estimate, n); the block is complex (see ``boosters`` for reality)."""
    blocks = boosters_for([(tuple(two_jb), tuple(two_lb), tuple(two_i_range),
                            tuple(two_k_range))], gamma, tol, n0, n_max, n_s)
    return blocks[0]


def boosters_for(edges, gamma, tol=1e-13, n0=16, n_max=512, n_s=256):
    """Blocks for a list of (two_jb, two_lb, i range, k range); one quadrature for all.

    n doubles from n0 until the summed |G61 - G30| of every entry is at most tol times the
    largest |entry| (or n reaches n_max).  Returns [(block, err, n)]."""
    need = set()
    for jb, lb, _, _ in edges:
        for a in range(4):
            for m in range(-jb[a], jb[a] + 1, 2):
                need.add((jb[a], lb[a], m))
    n = n0
    while True:
        r30, w30, r61, w61 = _r_nodes(n)
        res = []
        for rr, ww in ((r30, w30), (r61, w61)):
            dfun = {}
            for (tj, tl, tm) in need:
                rho = gamma * (tj / 2 + 1)
                dfun[(tj, tl, tm)] = boost_d(rho, tj, tj, tl, tm, rr, n_s)
            wt = ww * np.sinh(rr) ** 2 / (4 * np.pi)
            res.append([_block_from_d(jb, lb, dfun, wt, ir, kr) for jb, lb, ir, kr in edges])
        err = [np.abs(b61 - b30) for b30, b61 in zip(*res)]
        scale = max((np.abs(b).max() if b.size else 0.0) for b in res[1])
        worst = max((e.max() if e.size else 0.0) for e in err)
        if worst <= tol * max(scale, 1e-300) or n >= n_max:
            return [(b, e, n) for b, e in zip(res[1], err)]
        n *= 2


def boosters(two_j, dl, gamma, tol=1e-13, n_s=256):
    """Packed boosters of a configuration (layout of ``ranges.booster_layout``).

    Returns (flat real array, max |imaginary part|, max error estimate).  The real parts are
    the boosters; the imaginary parts are reported so that callers can check they vanish."""
    R.check_spins(two_j, dl)
    shapes, offsets = R.booster_layout(two_j, dl)
    bnd = R.boundary_ranges(two_j)
    edges, keys = [], []
    for e in range(2, 6):
        for t, triple in enumerate(product(range(dl + 1), repeat=3)):
            idim, kdim, klo = shapes[(e, t)]
            if idim * kdim == 0:
                continue
            jb, lb = _edge_spins(two_j, dl, e, triple)
            edges.append((tuple(jb), tuple(lb), bnd[e - 1], (klo, kdim)))
            keys.append((e, t))
    flat = np.zeros(offsets[-1])
    imag = 0.0
    errmax = 0.0
    for (e, t), (blk, err, _) in zip(keys, boosters_for(edges, gamma, tol, n_s=n_s)):
        pos = offsets[(e - 2) * (dl + 1) ** 3 + t]
        flat[pos:pos + blk.size] = blk.real.ravel()
        imag = max(imag, float(np.abs(blk.imag).max()))
        errmax = max(errmax, float(err.max()))
    return flat, imag, errmax
