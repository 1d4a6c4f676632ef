"""Pins of the oracle's {15j}, vertex tensor and contraction against independent definitions.

* {15j}: brute-force evaluation of the 4-simplex spin network from sympy 3jm symbols (no 6j
  symbols involved) must equal prod_e sqrt(2 i_e + 1) {15j} of eq. (15j), sign included.
* Vertex tensor: the same brute-force network with booster matrices inserted on edges 2..5,
  summed over shells, against the oracle's shell loop (catches index, ordering and packing
  mistakes); the Delta s = 0 identity-booster limit that reduces to the SU(2) BF vertex;
  the mpmath tier against the FP64 tier; shell additivity; multilinearity in the boosters.
* Contraction and derivatives: central finite differences (exact up to rounding because F
  is multilinear in every input) and numpy's einsum.
"""
import math
import random

import numpy as np
import pytest

import workloads
from oracle import ranges as R
from oracle import vertex as V
from oracle import contract as C
from oracle.fifteenj import fifteenj, fifteenj_block
from spin_network import simplex_evaluation, simplex_tensor, intertwiner_stack


def random_tiny_configs(seed, count, choices=(0, 1, 2, 3)):
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        tj = [rng.choice(choices) for _ in range(10)]
        try:
            R.check_spins(tj, 0)
        except ValueError:
            continue
        out.append(tj)
    return out


def test_15j_all_spins_zero():
    assert fifteenj(0, 0, 0, 0, 0, [0] * 10) == 1.0


def test_15j_against_brute_force_network():
    rng = random.Random(2)
    n_nonzero = 0
    for tj in random_tiny_configs(1, 60):
        bnd = R.boundary_ranges(tj)
        ii = [lo + 2 * rng.randrange(n) for lo, n in bnd]
        ev = simplex_evaluation(dict(zip(R.LINKS, tj)), ii)
        f = fifteenj(*ii, tj) * math.prod(math.sqrt(i + 1.0) for i in ii)
        assert f == pytest.approx(ev, abs=1e-14), (tj, ii)
        n_nonzero += abs(ev) > 1e-12
    assert n_nonzero > 40


def test_15j_block_matches_scalar():
    tj = [3, 3, 4, 4, 4, 2, 1, 2, 1, 4]
    R.check_spins(tj, 1)
    for shell in [(0, 0, 0, 0, 0, 0), (1, 0, 1, 0, 1, 1), (1, 1, 1, 1, 1, 1)]:
        two_l = R.shell_spins(tj, shell)
        kr = [R.virtual_range(two_l, e) for e in range(2, 6)]
        if any(d == 0 for _, d in kr):
            continue
        i1r = R.boundary_ranges(tj)[0]
        w = fifteenj_block(i1r, kr, two_l)
        for idx in np.ndindex(*w.shape):
            args = [i1r[0] + 2 * idx[0]] + [kr[q][0] + 2 * idx[q + 1] for q in range(4)]
            assert w[idx] == pytest.approx(fifteenj(*args, two_l), abs=1e-15)


def test_live_shell_counts():
    assert len(R.all_shells(3)) == 4096
    assert len(R.live_shells([2] * 10, 3)) == 3435
    # Every shell of an integer-spin equilateral vertex with j >= dl/2 is live: k_e ranges
    # contain at least |l - l'| .. l + l' with one spin fixed at j.
    assert len(R.live_shells([4] * 10, 2)) == 3 ** 6


def identity_boosters(two_j):
    """Packed Delta s = 0 boosters with (2k+1) B(i, k) = delta(i, k)."""
    shapes, offsets = R.booster_layout(two_j, 0)
    parts = []
    for e in range(2, 6):
        rows, cols, klo = shapes[(e, 0)]
        assert rows == cols
        parts.append((np.eye(rows) / (klo + 2 * np.arange(cols) + 1.0)[None, :]).ravel())
    return np.concatenate(parts)


@pytest.mark.parametrize("tj", random_tiny_configs(5, 6, choices=(1, 2, 3, 4)))
def test_bf_limit(tj):
    a = V.vertex_tensor(tj, 0, identity_boosters(tj))
    np.testing.assert_allclose(a, V.bf_vertex(tj), rtol=0, atol=1e-14)


def named_booster(e, names_to_two_l, two_i, two_k):
    """A deterministic booster entry that depends on every named virtual spin of the edge."""
    l1, l2, l3 = (names_to_two_l[n] for n in R.EDGE_TRIPLE[e])
    return math.sin(1.3 * e + 0.7 * l1 + 0.31 * l2 * l2 + 0.17 * l3 + 0.9 * two_i - 0.45 * two_k + 0.05 * two_i * two_k)


def pack_named_boosters(tj, dl):
    """Packed buffer in the documented layout: e = 2..5, triple (o1, o2, o3) lexicographic,
    block rows = i_e ascending, cols = k_e ascending."""
    parts = []
    bnd = R.boundary_ranges(tj)
    for e in range(2, 6):
        for o1 in range(dl + 1):
            for o2 in range(dl + 1):
                for o3 in range(dl + 1):
                    two_l = dict(zip(R.LINKS, tj))
                    for name, o in zip(R.EDGE_TRIPLE[e], (o1, o2, o3)):
                        two_l[name] += 2 * o
                    p, q, r, s = (two_l[n] for n in R.EDGE_LINKS[e])
                    klo = max(abs(p - q), abs(r - s))
                    khi = min(p + q, r + s)
                    for ni in range(bnd[e - 1][1]):
                        for two_k in range(klo, khi + 1, 2):
                            parts.append(named_booster(e, two_l, bnd[e - 1][0] + 2 * ni, two_k))
    return np.array(parts)


def brute_force_vertex(tj, dl):
    """Eq. (vertex-ampl) evaluated as boosted spin networks, shell by shell."""
    bnd = R.boundary_ranges(tj)
    dims = [n for _, n in bnd]
    total = np.zeros(dims)
    j = dict(zip(R.LINKS, tj))
    for shell in R.all_shells(dl):
        l = dict(j)
        for name, o in zip(R.VIRTUAL, shell):
            l[name] += 2 * o
        stacks = []
        lo1, st1 = intertwiner_stack(*(j[n] for n in R.EDGE_LINKS[1]))
        stacks.append(st1)
        empty = False
        for e in range(2, 6):
            p, q, r, s = (l[n] for n in R.EDGE_LINKS[e])
            if max(abs(p - q), abs(r - s)) > min(p + q, r + s) or (p + q + r + s) % 2:
                empty = True
                break
            klo, st = intertwiner_stack(p, q, r, s)
            ks = klo + 2 * np.arange(st.shape[0])
            b = np.array([[named_booster(e, l, bnd[e - 1][0] + 2 * ni, k) for k in ks] for ni in range(dims[e - 1])])
            # boosted node: sum_k B(i, k) sqrt(2k+1) iota_k
            stacks.append(np.tensordot(b * np.sqrt(ks + 1.0)[None, :], st, axes=([1], [0])))
        if empty:
            continue
        total += simplex_tensor(l, stacks)
    norms = [np.sqrt(lo + 2 * np.arange(n) + 1.0) for lo, n in bnd]
    # prod_{e>=2} sqrt(2 i_e + 1); node 1's intertwiner is already normalised.
    return total * np.einsum("a,b,c,d,e->abcde", np.ones(dims[0]), *norms[1:])


@pytest.mark.parametrize("tj,dl", [([2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 1), ([1] * 10, 1), ([3, 2, 4, 1, 2, 1, 4, 2, 2, 1], 1)])
def test_vertex_against_brute_force_network(tj, dl):
    R.check_spins(tj, dl)
    a = V.vertex_tensor(tj, dl, pack_named_boosters(tj, dl))
    ref = brute_force_vertex(tj, dl)
    assert np.abs(ref).max() > 1e-3
    np.testing.assert_allclose(a, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_reduced_i1_rows_against_brute_force_network():
    # A reduced set of boundary intertwiners i1 (Sec. 3.1): the rows asked for, in that order.
    tj, dl = [3, 2, 4, 1, 2, 1, 4, 2, 2, 1], 1
    ref = brute_force_vertex(tj, dl)
    rows = [ref.shape[0] - 1, 0]
    a = V.vertex_tensor(tj, dl, pack_named_boosters(tj, dl), i1_rows=rows)
    assert a.shape == (2,) + ref.shape[1:]
    np.testing.assert_allclose(a, ref[rows], rtol=0, atol=1e-13 * np.abs(ref).max())
    with pytest.raises(ValueError):
        V.vertex_tensor(tj, dl, pack_named_boosters(tj, dl), i1_rows=[ref.shape[0]])


def test_fp64_tier_against_mpmath_tier():
    tj, dl = [2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 1
    b = workloads.synthetic_boosters(5, R.block_shapes(tj, dl))
    a = V.vertex_tensor(tj, dl, b)
    ref = V.vertex_tensor_mp(tj, dl, b, dps=30)
    ref = np.vectorize(float)(ref)
    assert np.abs(a - ref).max() <= 1e-14 * np.abs(ref).max()


def test_shell_additivity():
    tj, dl = [2] * 10, 2
    b = workloads.synthetic_boosters(9, R.block_shapes(tj, dl))
    shells = R.all_shells(dl)
    full = V.vertex_tensor(tj, dl, b)
    part = V.vertex_tensor(tj, dl, b, shells=shells[:300]) + V.vertex_tensor(tj, dl, b, shells=shells[300:])
    np.testing.assert_allclose(part, full, rtol=0, atol=1e-13 * np.abs(full).max())


def test_multilinear_in_each_edge():
    tj, dl = [4, 1, 1, 4, 4, 3, 3, 1, 4, 1], 1
    shapes, offsets = R.booster_layout(tj, dl)
    b = workloads.synthetic_boosters(3, R.block_shapes(tj, dl))
    n3 = (dl + 1) ** 3
    edge3 = slice(offsets[n3], offsets[2 * n3])            # all blocks of edge 3
    x, y = b.copy(), b.copy()
    rng = np.random.default_rng(0)
    x[edge3] = rng.standard_normal(edge3.stop - edge3.start)
    y[edge3] = b[edge3] - x[edge3]
    np.testing.assert_allclose(V.vertex_tensor(tj, dl, x) + V.vertex_tensor(tj, dl, y),
                               V.vertex_tensor(tj, dl, b), rtol=0, atol=1e-12)


def test_contract_boundary_matches_einsum():
    tj, dl = [2] * 10, 1
    b = workloads.synthetic_boosters(4, R.block_shapes(tj, dl))
    a = V.vertex_tensor(tj, dl, b)
    psis = workloads.boundary_vectors(4, a.shape)
    f = C.contract_boundary(a, psis)
    ref = np.einsum("abcde,a,b,c,d,e->", a, *psis)
    assert abs(f - ref) <= 1e-14 * np.abs(a).sum()


def test_gradients_against_finite_differences():
    tj, dl = [4, 1, 2, 3, 1, 3, 2, 4, 4, 1], 1
    b = workloads.synthetic_boosters(6, R.block_shapes(tj, dl))
    a = V.vertex_tensor(tj, dl, b)
    psis = workloads.boundary_vectors(6, a.shape)
    h = 1e-6
    # dF/dpsi (holomorphic): perturb the real part of each entry.
    gp = C.grad_psi(a, psis)
    for q in range(5):
        for n in range(a.shape[q]):
            up = [p.copy() for p in psis]
            dn = [p.copy() for p in psis]
            up[q][n] += h
            dn[q][n] -= h
            fd = (C.contract_boundary(a, up) - C.contract_boundary(a, dn)) / (2 * h)
            assert abs(fd - gp[q][n]) <= 2e-8 * max(1.0, abs(gp[q][n]))
    gb = C.grad_boosters(tj, dl, b, psis)
    rng = np.random.default_rng(1)
    for n in rng.choice(b.size, size=25, replace=False):
        up, dn = b.copy(), b.copy()
        up[n] += h
        dn[n] -= h
        fd = (C.contract_boundary(V.vertex_tensor(tj, dl, up), psis)
              - C.contract_boundary(V.vertex_tensor(tj, dl, dn), psis)) / (2 * h)
        assert abs(fd - gb[n]) <= 2e-8 * max(1.0, abs(gb[n])), n
    # directional derivative over all booster entries at once
    d = rng.standard_normal(b.size)
    fd = (C.contract_boundary(V.vertex_tensor(tj, dl, b + h * d), psis)
          - C.contract_boundary(V.vertex_tensor(tj, dl, b - h * d), psis)) / (2 * h)
    assert abs(fd - np.dot(gb, d)) <= 2e-8 * max(1.0, abs(fd))


def test_restricted_booster_gradient_matches_full():
    # Visiting only the shells that use the chosen blocks gives those blocks' full gradient.
    tj, dl = [4, 1, 2, 3, 1, 3, 2, 4, 4, 1], 1
    b = workloads.synthetic_boosters(6, R.block_shapes(tj, dl))
    psis = workloads.boundary_vectors(6, [n for _, n in R.boundary_ranges(tj)])
    full = C.grad_boosters(tj, dl, b, psis)
    shapes, offsets = R.booster_layout(tj, dl)
    n3 = (dl + 1) ** 3
    only = [(2, 0), (3, 5), (5, 7)]
    part = C.grad_boosters(tj, dl, b, psis, only=only)
    assert sorted(part) == sorted(only)
    for e, t in only:
        n = (e - 2) * n3 + t
        ref = full[offsets[n]:offsets[n + 1]].reshape(part[(e, t)].shape)
        np.testing.assert_array_equal(part[(e, t)], ref)
