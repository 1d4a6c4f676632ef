"""Contractions of several vertex tensors (oracle; test infrastructure only).

Spin foam amplitudes with more than one vertex are contractions of vertex tensors over the
intertwiners of their shared (bulk) edges, and with boundary vectors on the others (Sec. 3.1
"Tensor contractions", the contraction of vertex tensors over internal intertwiner indices).
Three patterns of the paper:

* the complete contraction of two vertex tensors, sum over all five intertwiners of A B (the
  left test of Sec. 3.3 "Tensor contractions on CPU and GPU");
* a vertex contracted with boundary vectors on some of its intertwiners, leaving a tensor in
  the others (each vertex of the Delta_3 amplitude of Sec. 4.2 keeps its two bulk
  intertwiners);
* the Delta_3 amplitude from three such matrices: a sum over the three bulk intertwiners with
  the sign (-1)^(k1 + k2 + k3), times (-1)^x (2x + 1) for the spin x of the internal face.

Index conventions are those of the vertex tensor here, A[i1][i2][i3][i4][i5] (row-major, the
bytes of the paper's column-major A^{i5 i4 i3 i2 i1}): a contraction of the paper that pairs its
vectors with the first m column-major indices (i5, i4, ...) pairs them here with the last m
indices (..., i4, i5).  All spins are passed as twice their value.
"""
import math

import numpy as np

__all__ = ["contract_vertices", "contract_trailing", "delta3"]


def contract_vertices(a, b):
    """sum_{i1..i5} A(i1..i5) B(i1..i5) for two real tensors of equal shape, summed with
    ``math.fsum`` (correctly rounded)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("the two tensors must have the same shape")
    return math.fsum((a * b).ravel())


def contract_trailing(a, psis):
    """T(i1..i_{5-m}) = sum over the last m intertwiners of A(i1..i5) psi_1(i_{6-m}) ... psi_m(i5)
    (no complex conjugation), m = len(psis) in 1..5; a complex array over the leading 5 - m
    indices (a 0-d array for m = 5)."""
    a = np.asarray(a, dtype=np.float64)
    m = len(psis)
    if not 1 <= m <= 5:
        raise ValueError("between one and five vectors")
    lead = a.ndim - m
    for q, p in enumerate(psis):
        if np.asarray(p).shape != (a.shape[lead + q],):
            raise ValueError("vector length does not match its intertwiner dimension")
    terms = a.astype(np.complex128)
    for q, p in enumerate(psis):
        shape = [1] * a.ndim
        shape[lead + q] = -1
        terms = terms * np.asarray(p, dtype=np.complex128).reshape(shape)
    return terms.sum(axis=tuple(range(lead, a.ndim)))


def delta3(ta, tb, tc, two_klo, two_x):
    """Delta_3 amplitude (Sec. 4.2) from the three partially contracted vertices.

    ta[k1][k2], tb[k3][k1], tc[k2][k3]: complex n x n matrices over the bulk intertwiner range
    k = (two_klo + 2 n') / 2, n' = 0..n-1 (each vertex keeps the bulk intertwiners of its first
    two nodes, in the orientation of the triangle k1 -> k2 -> k3 -> k1):

        (-1)^x (2x + 1) sum_{k1, k2, k3} (-1)^(k1 + k2 + k3) ta[k1][k2] tb[k3][k1] tc[k2][k3].

    The bulk intertwiners and x must be integer spins (even two_klo and two_x)."""
    ta, tb, tc = (np.asarray(t, dtype=np.complex128) for t in (ta, tb, tc))
    n = ta.shape[0]
    if any(t.shape != (n, n) for t in (ta, tb, tc)):
        raise ValueError("three square matrices of the same size are required")
    if two_klo % 2 or two_x % 2:
        raise ValueError("integer bulk intertwiners and internal spin are required")
    sign = [(-1) ** ((two_klo + 2 * q) // 2) for q in range(n)]
    re, im = [], []
    for k1 in range(n):
        for k2 in range(n):
            for k3 in range(n):
                v = sign[k1] * sign[k2] * sign[k3] * ta[k1, k2] * tb[k3, k1] * tc[k2, k3]
                re.append(v.real)
                im.append(v.imag)
    pre = (-1) ** (two_x // 2) * (two_x + 1)
    return pre * complex(math.fsum(re), math.fsum(im))
