"""Pins of the oracle's FP64 quadrature boosters (eq. (booster)) and their ingredients.

* 3jm against sympy's exact ``wigner_3j``; 4jm orthogonality;
* SU(2) small d against its closed forms for j = 1/2 and 1, the group law;
* SL(2,C) boost matrix elements: the spherical function sin(rho r) / (rho sinh r) of the
  (rho, 0) representation, the identity at r = 0, unitarity (sum over l of |d|^2 = 1), the
  generator at r = 0 against Naimark's matrix elements of the boost generator, and the
  m -> -m symmetry of the paper's finite-sum formula (Sec. 3.1);
* the booster of all spins zero in closed form: with d = sin(gamma r) / (gamma sinh r) the
  integral is (1/(4 pi gamma^4)) int sin^4(gamma r) / sinh^2 r dr, and
  int_0^inf sin^2(b r) / sinh^2 r dr = (pi b coth(pi b) - 1) / 2 with sin^4 = (sin^2 - sin^2(2 .) / 4);
* reality and quadrature convergence of the boosters of the j = 1, dl = 3 configuration.
"""
import math
import random

import numpy as np
import pytest
from sympy import Rational
from sympy.physics.wigner import wigner_3j

from oracle import boosters as Bo


def test_threejm_against_sympy():
    rng = random.Random(11)
    done = 0
    while done < 200:
        a, b = rng.randint(0, 14), rng.randint(0, 14)
        c = rng.randrange(abs(a - b), a + b + 1, 2)
        m1, m2 = rng.randrange(-a, a + 1, 2), rng.randrange(-b, b + 1, 2)
        m3 = -m1 - m2
        if abs(m3) > c:
            continue
        ref = float(wigner_3j(*[Rational(v, 2) for v in (a, b, c, m1, m2, m3)]).evalf(40))
        assert Bo.threejm(a, b, c, m1, m2, m3) == pytest.approx(ref, rel=2e-16, abs=1e-300)
        done += 1
    assert Bo.threejm(2, 2, 2, 2, 0, 0) == 0.0          # m's do not sum to zero
    assert Bo.threejm(2, 2, 6, 0, 0, 0) == 0.0          # triangle violated


@pytest.mark.parametrize("tj", [(2, 2, 2, 2), (1, 3, 2, 2), (4, 2, 3, 3), (6, 6, 6, 6)])
def test_fourjm_orthogonality(tj):
    lo = max(abs(tj[0] - tj[1]), abs(tj[2] - tj[3]))
    hi = min(tj[0] + tj[1], tj[2] + tj[3])
    ivals = list(range(lo, hi + 1, 2))
    import itertools
    ms = [m for m in itertools.product(*(range(-j, j + 1, 2) for j in tj)) if sum(m) == 0]
    for i in ivals:
        for ip in ivals:
            s = sum(Bo.fourjm(tj, m, i) * Bo.fourjm(tj, m, ip) for m in ms)
            assert s == pytest.approx((1.0 / (i + 1)) if i == ip else 0.0, abs=1e-14)


def test_su2_d_closed_forms():
    beta = np.linspace(0.0, math.pi, 7)
    c, s = np.cos(beta / 2), np.sin(beta / 2)
    np.testing.assert_allclose(Bo.su2_d(1, 1, 1, beta), c, atol=1e-15)
    np.testing.assert_allclose(Bo.su2_d(1, 1, -1, beta), -s, atol=1e-15)
    np.testing.assert_allclose(Bo.su2_d(1, -1, 1, beta), s, atol=1e-15)
    np.testing.assert_allclose(Bo.su2_d(2, 2, 2, beta), (1 + np.cos(beta)) / 2, atol=1e-15)
    np.testing.assert_allclose(Bo.su2_d(2, 2, 0, beta), -np.sin(beta) / math.sqrt(2), atol=1e-15)
    np.testing.assert_allclose(Bo.su2_d(2, 0, 0, beta), np.cos(beta), atol=1e-15)
    # group law d(a) d(b) = d(a + b) for j = 5/2
    a, b = 0.4, 1.1
    da = np.array([[Bo.su2_d(5, p, q, np.array([a]))[0] for q in range(5, -6, -2)] for p in range(5, -6, -2)])
    db = np.array([[Bo.su2_d(5, p, q, np.array([b]))[0] for q in range(5, -6, -2)] for p in range(5, -6, -2)])
    dab = np.array([[Bo.su2_d(5, p, q, np.array([a + b]))[0] for q in range(5, -6, -2)] for p in range(5, -6, -2)])
    np.testing.assert_allclose(da @ db, dab, atol=1e-14)


@pytest.mark.parametrize("rho", [0.6, 1.2, 3.7, 9.0])
def test_boost_spherical_function(rho):
    r = np.array([1e-3, 0.2, 1.0, 3.0, 8.0, 20.0])
    got = Bo.boost_d(rho, 0, 0, 0, 0, r)
    np.testing.assert_allclose(got, np.sin(rho * r) / (rho * np.sinh(r)), rtol=0, atol=2e-15)


def test_boost_identity_at_zero():
    # d(r) = delta + O(r): at r = 1e-12 the first-order term is below 1e-11.
    for tk, tj, tl, tm in [(2, 2, 2, 0), (2, 2, 4, 2), (1, 1, 5, -1), (4, 6, 6, 2)]:
        d = Bo.boost_d(3.0, tk, tj, tl, tm, np.array([1e-12]))[0]
        assert abs(d - (1.0 if tj == tl else 0.0)) < 1e-11


@pytest.mark.parametrize("rho,tk,tm", [(1.2, 0, 0), (2.4, 2, 2), (4.8, 6, -2), (3.0, 1, 1)])
def test_boost_unitarity(rho, tk, tm):
    # Row j = k of the unitary boost: sum over l of |d_{k l m}(r)|^2 = 1.
    for r in (0.3, 1.0):
        tot = sum(abs(Bo.boost_d(rho, tk, tk, tl, tm, np.array([r]), n_s=512)[0]) ** 2
                  for tl in range(max(tk, abs(tm)), tk + 120, 2))
        assert tot == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("rho,tk,tj,tm", [(2.4, 2, 2, 2), (2.4, 2, 4, 0), (4.8, 6, 8, -2), (3.0, 1, 3, 1)])
def test_boost_generator_matches_naimark(rho, tk, tj, tm):
    # d/dr at r = 0 is the boost generator: diagonal i k rho m / (j (j+1)); between j and
    # j + 1 a purely imaginary element of modulus |C_{j+1}| sqrt((j+1)^2 - m^2) with
    # |C_J| = sqrt((J^2 - k^2)(J^2 + rho^2) / (4 J^2 - 1)) / J  (Naimark).
    k, j, m = tk / 2, tj / 2, tm / 2
    h = 1e-4

    def deriv(tl):
        d1 = Bo.boost_d(rho, tk, tj, tl, tm, np.array([h]))[0]
        d2 = Bo.boost_d(rho, tk, tj, tl, tm, np.array([2 * h]))[0]
        return (4 * d1 - d2 - 3 * (1.0 if tl == tj else 0.0)) / (2 * h)

    diag = deriv(tj)
    assert diag.real == pytest.approx(0.0, abs=1e-6)
    assert diag.imag == pytest.approx(k * rho * m / (j * (j + 1)), abs=1e-6)
    off = deriv(tj + 2)
    J = j + 1
    mod = math.sqrt((J * J - k * k) * (J * J + rho * rho) / (4 * J * J - 1)) / J * math.sqrt(J * J - m * m)
    assert off.real == pytest.approx(0.0, abs=1e-6)
    assert abs(off.imag) == pytest.approx(mod, rel=1e-6)


@pytest.mark.parametrize("rho,tk,tl,tm", [(2.4, 2, 4, 2), (2.4, 2, 6, 2), (3.0, 1, 5, 1), (3.6, 4, 8, 2)])
def test_boost_m_symmetry(rho, tk, tl, tm):
    r = np.array([0.4, 2.0, 6.0])
    a = Bo.boost_d(rho, tk, tk, tl, tm, r)
    b = Bo.boost_d(rho, tk, tk, tl, -tm, r)
    sign = -1.0 if ((tl - tk) // 2) % 2 else 1.0
    np.testing.assert_allclose(b, sign * np.conj(a), atol=1e-14)


@pytest.mark.parametrize("gamma", [1.2, 0.7])
def test_booster_all_spins_zero_closed_form(gamma):
    blk, err, _ = Bo.booster_block((0, 0, 0, 0), (0, 0, 0, 0), (0, 1), (0, 1), gamma)

    def sin2_over_sinh2(b):  # int_0^inf sin^2(b r) / sinh^2(r) dr
        return (math.pi * b / math.tanh(math.pi * b) - 1) / 2

    ref = (sin2_over_sinh2(gamma) - sin2_over_sinh2(2 * gamma) / 4) / (4 * math.pi * gamma ** 4)
    assert abs(blk[0, 0].imag) < 1e-16
    assert blk[0, 0].real == pytest.approx(ref, rel=1e-13)
    assert err.max() < 1e-13 * ref
    if gamma == 1.2:
        assert ref == pytest.approx(0.0218547155646276, rel=1e-14)


def test_boosters_real_and_converged():
    flat, imag, err = Bo.boosters([2] * 10, 3, 1.2)
    scale = np.abs(flat).max()
    assert imag < 1e-14 * scale
    assert err < 1e-13 * scale
    # The same blocks with twice the subdivision of the converged rule agree to 1e-14.
    from oracle import ranges as R
    two_j, dl = [2] * 10, 3
    shapes, offsets = R.booster_layout(two_j, dl)
    bnd = R.boundary_ranges(two_j)
    for e, triple in [(3, (3, 1, 2)), (5, (2, 3, 3))]:
        t = (triple[0] * (dl + 1) + triple[1]) * (dl + 1) + triple[2]
        idim, kdim, klo = shapes[(e, t)]
        jb, lb = Bo._edge_spins(two_j, dl, e, triple)
        _, _, n = Bo.booster_block(jb, lb, bnd[e - 1], (klo, kdim), 1.2)
        fine, _, _ = Bo.booster_block(jb, lb, bnd[e - 1], (klo, kdim), 1.2, n0=2 * n, n_max=2 * n)
        pos = offsets[(e - 2) * (dl + 1) ** 3 + t]
        np.testing.assert_allclose(flat[pos:pos + idim * kdim].reshape(idim, kdim), fine.real,
                                   rtol=0, atol=1e-14 * scale)


def test_stored_quadrature_boosters_match_the_oracle():
    """The boosters stored beside the j = 1 golden are the oracle's (recomputed here), and the
    j = 3 ones have the packed layout's size, are finite and were taken at gamma = 1.2."""
    import os
    from oracle import ranges as R
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g1 = np.load(os.path.join(here, "vertex_j1_dl3_phys.npz"))
    flat, imag, err = Bo.boosters(list(g1["two_j"]), int(g1["dl"]), float(g1["gamma"]))
    np.testing.assert_allclose(g1["boosters"], flat, rtol=0, atol=1e-15 * np.abs(flat).max())
    g3 = np.load(os.path.join(here, "vertex_j3_dl8_phys.npz"))
    _, offsets = R.booster_layout(list(g3["two_j"]), int(g3["dl"]))
    assert g3["boosters"].size == offsets[-1]
    assert np.all(np.isfinite(g3["boosters"])) and float(g3["gamma"]) == 1.2
    assert int(g3["booster_seed"]) == -1


def test_bench_loads_the_stored_quadrature_boosters():
    import bench
    from oracle import ranges as R
    two_j, dl = [6] * 10, 8
    _, offsets = R.booster_layout(two_j, dl)
    b = bench.quadrature_boosters(two_j, dl, offsets[-1])
    assert b is not None and b.dtype == np.float64 and b.size == offsets[-1]
    assert bench.quadrature_boosters(two_j, dl, offsets[-1] + 1) is None
    assert bench.quadrature_boosters([8] * 10, dl, offsets[-1]) is None


@pytest.mark.parametrize("jb,lb", [((2, 3, 1, 2), (4, 5, 1, 2)),      # edge-2 shape: three links boosted
                                   ((3, 2, 4, 1), (3, 4, 6, 3)),
                                   ((4, 4, 2, 2), (6, 8, 4, 2))])
def test_block_pairing_against_intertwiner_tensors(jb, lb):
    """The m-sum of eq. (booster) in ``_block_from_d`` against the same sum written as a tensor
    contraction of the normalised intertwiners of the spin-network helper (sympy 3jm, written
    independently of the oracle's 3jm/4jm): with D[m1..m4] = sum_r w(r) prod_a d_a(m_a; r),

        B(i, k) = sum_m iota^j_i[m] iota^l_k[m] D[m] / sqrt((2i+1)(2k+1)).

    A mis-paired magnetic index, a wrong 4jm phase or a swapped pair of links in the oracle's
    block would change B for these non-zero spins."""
    from spin_network import intertwiner_stack
    gamma = 1.2
    r30, w30, _, _ = Bo._r_nodes(16)
    wt = w30 * np.sinh(r30) ** 2 / (4 * np.pi)
    dfun = {}
    for tj, tl in zip(jb, lb):
        for tm in range(-tj, tj + 1, 2):
            dfun[(tj, tl, tm)] = Bo.boost_d(gamma * (tj / 2 + 1), tj, tj, tl, tm, r30)
    ilo, iota_j = intertwiner_stack(*jb)
    klo, iota_l = intertwiner_stack(*lb)
    got = Bo._block_from_d(jb, lb, dfun, wt, (ilo, iota_j.shape[0]), (klo, iota_l.shape[0]))
    # Magnetic numbers of link a run over -j_a..j_a: the l-side tensor is cut to those m.
    cut = tuple(slice((tl - tj) // 2, (tl - tj) // 2 + tj + 1) for tj, tl in zip(jb, lb))
    iota_l = iota_l[(slice(None),) + cut]
    mats = [np.stack([dfun[(tj, tl, tm)] for tm in range(-tj, tj + 1, 2)]) for tj, tl in zip(jb, lb)]
    D = np.einsum("ar,br,cr,dr,r->abcd", *mats, wt)
    ref = np.einsum("ipqrs,kpqrs,pqrs->ik", iota_j, iota_l, D)
    ref /= np.sqrt(np.outer(ilo + 2 * np.arange(iota_j.shape[0]) + 1.0,
                            klo + 2 * np.arange(iota_l.shape[0]) + 1.0))
    assert got.shape == ref.shape
    scale = np.abs(ref).max()
    assert scale > 1e-6
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * scale)
