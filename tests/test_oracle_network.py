"""Pins of the oracle's multi-vertex contractions (oracle/network.py) to definitions checked
another way: brute-force loops on tiny tensors, the boundary contraction of one vertex (itself
pinned against einsum), closed forms of the Delta_3 sum and algebraic identities."""
import itertools
import math

import numpy as np
import pytest

from oracle import contract as C
from oracle import network as N

SHAPE = (2, 3, 2, 3, 2)


def rand_tensor(seed, shape=SHAPE):
    return np.random.default_rng(seed).normal(size=shape)


def rand_vec(rng, n):
    return rng.normal(size=n) + 1j * rng.normal(size=n)


def test_contract_vertices_brute_force_and_identities():
    a, b = rand_tensor(1), rand_tensor(2)
    brute = 0.0
    for idx in itertools.product(*(range(n) for n in SHAPE)):
        brute += a[idx] * b[idx]
    assert abs(N.contract_vertices(a, b) - brute) <= 1e-14 * abs(brute) + 1e-15
    assert N.contract_vertices(a, b) == N.contract_vertices(b, a)
    assert N.contract_vertices(a, a) > 0
    # A one-hot second tensor picks out one entry.
    e = np.zeros(SHAPE)
    e[1, 2, 0, 1, 1] = 1.0
    assert N.contract_vertices(a, e) == a[1, 2, 0, 1, 1]
    # Bilinear.
    c = rand_tensor(3)
    lhs = N.contract_vertices(a, 2.0 * b - 3.0 * c)
    rhs = 2.0 * N.contract_vertices(a, b) - 3.0 * N.contract_vertices(a, c)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1)
    with pytest.raises(ValueError):
        N.contract_vertices(a, rand_tensor(4, (2, 3, 2, 3, 3)))


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_contract_trailing_brute_force(m):
    rng = np.random.default_rng(10 + m)
    a = rand_tensor(5)
    psis = [rand_vec(rng, n) for n in SHAPE[5 - m:]]
    t = N.contract_trailing(a, psis)
    assert t.shape == SHAPE[:5 - m]
    for lead in itertools.product(*(range(n) for n in SHAPE[:5 - m])):
        s = 0.0
        for tail in itertools.product(*(range(n) for n in SHAPE[5 - m:])):
            w = 1.0
            for q, i in enumerate(tail):
                w = w * psis[q][i]
            s += a[lead + tail] * w
        assert abs(t[lead] - s) <= 1e-13 * (abs(s) + 1)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_contract_trailing_then_leading_is_boundary_contraction(m):
    """Contracting the remaining leading indices of the partial result with their vectors gives
    the boundary contraction of the whole tensor (Sec. 3.2)."""
    rng = np.random.default_rng(20 + m)
    a = rand_tensor(6)
    psis = [rand_vec(rng, n) for n in SHAPE]
    t = N.contract_trailing(a, psis[5 - m:])
    for q in reversed(range(5 - m)):
        t = t @ psis[q] if t.ndim == 1 else np.tensordot(t, psis[q], axes=([t.ndim - 1], [0]))
    ref = C.contract_boundary(a, psis)
    assert abs(complex(t) - ref) <= 1e-13 * abs(ref)


def test_contract_trailing_all_five_is_boundary_contraction():
    rng = np.random.default_rng(30)
    a = rand_tensor(7)
    psis = [rand_vec(rng, n) for n in SHAPE]
    ref = C.contract_boundary(a, psis)
    assert abs(complex(N.contract_trailing(a, psis)) - ref) <= 1e-13 * abs(ref)


def test_contract_trailing_one_hot_vectors_pick_slices():
    a = rand_tensor(8)
    e4 = np.zeros(SHAPE[3]); e4[2] = 1.0
    e5 = np.zeros(SHAPE[4]); e5[1] = 1.0
    t = N.contract_trailing(a, [e4, e5])
    np.testing.assert_array_equal(t.real, a[:, :, :, 2, 1])
    assert not t.imag.any()


def trace_form(ta, tb, tc, two_klo, two_x):
    """(-1)^x (2x+1) Tr(S ta S tc S tb), S = diag((-1)^k): the same sum as a matrix product."""
    n = ta.shape[0]
    s = np.diag([(-1.0) ** ((two_klo + 2 * q) // 2) for q in range(n)])
    return (-1) ** (two_x // 2) * (two_x + 1) * np.trace(s @ ta @ s @ tc @ s @ tb)


@pytest.mark.parametrize("n,two_klo,two_x", [(1, 0, 0), (3, 2, 4), (5, 0, 2), (4, 6, 10)])
def test_delta3_against_trace_form(n, two_klo, two_x):
    rng = np.random.default_rng(40 + n)
    ta, tb, tc = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) for _ in range(3))
    v = N.delta3(ta, tb, tc, two_klo, two_x)
    ref = trace_form(ta, tb, tc, two_klo, two_x)
    assert abs(v - ref) <= 1e-13 * (abs(ref) + 1)
    # The sum is a trace of a product: invariant under the cyclic relabelling of the triangle
    # (k1, k2, k3) -> (k2, k3, k1), which maps (ta, tb, tc) to (tc, ta, tb).
    assert abs(N.delta3(tc, ta, tb, two_klo, two_x) - v) <= 1e-13 * (abs(v) + 1)


def test_delta3_identity_matrices():
    """ta = tb = tc = 1: only k1 = k2 = k3 survives, sum_k (-1)^(3k) = sum_k (-1)^k."""
    n, two_klo, two_x = 5, 2, 6
    eye = np.eye(n, dtype=complex)
    expect = sum((-1) ** ((two_klo + 2 * q) // 2) for q in range(n)) * (-1) ** 3 * 7
    assert N.delta3(eye, eye, eye, two_klo, two_x) == expect


def test_delta3_orientation_matters():
    """With non-symmetric matrices the orientation of tb is seen: tb transposed changes the sum
    (so a swapped index would not pass the trace-form pin)."""
    rng = np.random.default_rng(50)
    ta, tb, tc = (rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)) for _ in range(3))
    assert abs(N.delta3(ta, tb, tc, 0, 0) - N.delta3(ta, tb.T, tc, 0, 0)) > 1e-3


def test_delta3_rejects_half_integer_phases():
    eye = np.eye(2, dtype=complex)
    with pytest.raises(ValueError):
        N.delta3(eye, eye, eye, 1, 0)
    with pytest.raises(ValueError):
        N.delta3(eye, eye, eye, 0, 3)
    assert math.isfinite(abs(N.delta3(eye, eye, eye, 0, 0)))
