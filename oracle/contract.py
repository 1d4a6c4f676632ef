"""Boundary contraction of the vertex tensor and its derivatives (oracle; test infrastructure).

Sec. 3.2 (``contract(v, cs5, ..., cs1)``) contracts the vertex tensor with one boundary
vector per node.  With vectors psi_a indexed by the boundary intertwiner i_a:

    F = sum_{i1..i5} A(i1..i5) psi_1(i1) psi_2(i2) psi_3(i3) psi_4(i4) psi_5(i5)

(no complex conjugation; the paper's reversed argument order is an artefact of its
column-major storage, so psi_a here always pairs with i_a).

Derivatives (F is multilinear, so these are exact polynomial derivatives):

* dF/dpsi_a(i_a): A contracted with the four other vectors.
* dF/dB_e[l_e](i_e, k_e): by eq. (vertex-ampl), with psi~_a(i) = sqrt(2i+1) psi_a(i),
  M_b = (2k_b+1) B_b and v_b(k_b) = sum_i psi~_b(i) M_b(i, k_b),

      dF/dB_e(i_e, k_e) = psi~_e(i_e) (2k_e+1)
                          * sum_{shells using this block} sum_{i1, k_b, b != e}
                            psi~_1(i1) prod_{b != e} v_b(k_b) W_shell(i1, k2..k5).

  The {15j} tensor W of every shell is recomputed; nothing is stored across shells.
"""
import math

import numpy as np

from . import ranges as R
from .fifteenj import fifteenj_block
from .vertex import unpack_boosters

__all__ = ["contract_boundary", "grad_psi", "grad_boosters"]


def contract_boundary(a, psis):
    """F as a Python complex; real and imaginary parts summed with ``math.fsum``."""
    a = np.asarray(a, dtype=np.float64)
    if len(psis) != 5 or any(np.asarray(p).shape != (n,) for p, n in zip(psis, a.shape)):
        raise ValueError("five vectors matching the tensor dimensions are required")
    terms = a.astype(np.complex128)
    for axis, p in enumerate(psis):
        shape = [1] * 5
        shape[axis] = -1
        terms = terms * np.asarray(p, dtype=np.complex128).reshape(shape)
    return complex(math.fsum(terms.real.ravel()), math.fsum(terms.imag.ravel()))


def grad_psi(a, psis):
    """[dF/dpsi_a] for a = 1..5, each a complex vector of length dim(i_a)."""
    a = np.asarray(a, dtype=np.complex128)
    letters = "abcde"
    out = []
    for q in range(5):
        others = [p for n, p in enumerate(psis) if n != q]
        spec = letters + "," + ",".join(letters[n] for n in range(5) if n != q) + "->" + letters[q]
        out.append(np.einsum(spec, a, *[np.asarray(p, dtype=np.complex128) for p in others]))
    return out


def grad_boosters(two_j, dl, boosters, psis, only=None):
    """dF/dB for every packed booster entry (complex, same packing as the input).

    ``only``: a list of booster blocks (edge e in 2..5, triple index t); then only the shells
    that use one of them are visited and a dict {(e, t): dF/dB block} is returned.
    """
    blocks = unpack_boosters(two_j, dl, boosters)
    wanted = None if only is None else {(int(e), int(t)) for e, t in only}
    bnd = R.boundary_ranges(two_j)
    psit = [np.asarray(p, dtype=np.complex128) * np.sqrt(lo + 2 * np.arange(n) + 1.0)
            for p, (lo, n) in zip(psis, bnd)]
    grads = {key: np.zeros(blk.shape, dtype=np.complex128) for key, blk in blocks.items()}
    for shell in R.all_shells(dl):
        two_l = R.shell_spins(two_j, shell)
        kr = [R.virtual_range(two_l, e) for e in range(2, 6)]
        if any(d == 0 for _, d in kr):
            continue
        keys = {e: (e, R.edge_triple_index(e, shell, dl)) for e in range(2, 6)}
        if wanted is not None and not wanted.intersection(keys.values()):
            continue
        w = fifteenj_block(bnd[0], kr, two_l).astype(np.complex128)   # W[i1, k2, k3, k4, k5]
        weights = {e: (kr[e - 2][0] + 2 * np.arange(kr[e - 2][1]) + 1.0) for e in range(2, 6)}
        v = {e: psit[e - 1] @ (blocks[keys[e]] * weights[e][None, :]) for e in range(2, 6)}
        t = np.einsum("abcde,a->bcde", w, psit[0])                     # [k2, k3, k4, k5]
        g = {
            2: np.einsum("bcde,c,d,e->b", t, v[3], v[4], v[5]),
            3: np.einsum("bcde,b,d,e->c", t, v[2], v[4], v[5]),
            4: np.einsum("bcde,b,c,e->d", t, v[2], v[3], v[5]),
            5: np.einsum("bcde,b,c,d->e", t, v[2], v[3], v[4]),
        }
        for e in range(2, 6):
            grads[keys[e]] += np.outer(psit[e - 1], weights[e] * g[e])
    if wanted is not None:
        return {key: grads[key] for key in sorted(wanted)}
    return np.concatenate([grads[(e, t)].ravel() for e in range(2, 6)
                           for t in range((dl + 1) ** 3)])
