"""The EPRL vertex tensor in the booster decomposition (oracle; test infrastructure only).

Eq. (vertex-ampl):

    A(i1..i5) = prod_{e=1..5} sqrt(2 i_e + 1)
                * sum_{l, k} prod_{e=2..5} (2 k_e + 1) B_e(j, i_e; l, k_e) {15j}(l, i1, k2..k5)

with l12..l15 fixed to the boundary spins and the six other virtual spins cut off at
j_ab + Delta s.  The oracle follows the framed algorithm of Sec. 3.1 step by step:
ranges (step 2), boosters as an input (step 3), then for each shell (steps 5-6) the {15j}
tensor W (6(i)), the four booster sub-matrices of that shell (6(ii)), their contraction
with W over k5, k4, k3, k2 (6(iii), one mode at a time) and the accumulation (6(iv)).
The final normalisation prod_e sqrt(2 i_e + 1) is applied at the end.

The shell sum is accumulated with Neumaier's compensated summation so that the oracle's
own rounding error stays far below the tolerance of the parity tests.

Two tiers:
* ``vertex_tensor``     FP64 products, exactly rounded 6j, compensated shell sum.
* ``vertex_tensor_mp``  everything in mpmath at ``dps`` digits, pure Python loops; tiny
                        inputs only.  Used to bound the error of the FP64 tier.
"""
import numpy as np

from . import ranges as R
from .fifteenj import fifteenj_block, fifteenj
from .wigner import sixj_exact

__all__ = ["vertex_tensor", "vertex_tensor_mp", "unpack_boosters", "shell_contribution"]


def unpack_boosters(two_j, dl, flat):
    """Split the packed booster buffer into {(e, t): 2-D array} blocks."""
    shapes, offsets = R.booster_layout(two_j, dl)
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != offsets[-1]:
        raise ValueError(f"booster buffer holds {flat.size} values, layout needs {offsets[-1]}")
    blocks = {}
    n = 0
    for e in range(2, 6):
        for t in range((dl + 1) ** 3):
            rows, cols, _ = shapes[(e, t)]
            blocks[(e, t)] = flat[offsets[n]:offsets[n + 1]].reshape(rows, cols)
            n += 1
    return blocks


def _weighted(block, two_klo):
    """(2 k_e + 1) B_e(i_e, k_e) for one booster block."""
    ks = two_klo + 2 * np.arange(block.shape[1])
    return block * (ks + 1)[None, :]


def shell_contribution(two_j, dl, blocks, shell, i1_rows=None):
    """The contracted {15j} x booster term of one shell, indexed [i1, i2, i3, i4, i5].

    ``i1_rows`` (indices into the i1 range) restricts the result to those rows of the gauge-fixed
    intertwiner, in the given order.  Returns None for a shell with an empty virtual-intertwiner
    range.
    """
    two_l = R.shell_spins(two_j, shell)
    kr = [R.virtual_range(two_l, e) for e in range(2, 6)]
    if any(d == 0 for _, d in kr):
        return None
    i1r = R.boundary_ranges(two_j)[0]
    if i1_rows is None:
        w = fifteenj_block(i1r, kr, two_l)                        # W[i1, k2, k3, k4, k5]
    else:
        w = np.concatenate([fifteenj_block((i1r[0] + 2 * n, 1), kr, two_l) for n in i1_rows])
    m = {e: _weighted(blocks[(e, R.edge_triple_index(e, shell, dl))], kr[e - 2][0])
         for e in range(2, 6)}
    # Contract one virtual intertwiner at a time: k5, then k4, k3, k2.
    t = np.tensordot(w, m[5], axes=([4], [1]))                    # [i1, k2, k3, k4, i5]
    t = np.tensordot(t, m[4], axes=([3], [1]))                    # [i1, k2, k3, i5, i4]
    t = np.tensordot(t, m[3], axes=([2], [1]))                    # [i1, k2, i5, i4, i3]
    t = np.tensordot(t, m[2], axes=([1], [1]))                    # [i1, i5, i4, i3, i2]
    return np.transpose(t, (0, 4, 3, 2, 1))                       # [i1, i2, i3, i4, i5]


def _normalisation(two_j):
    dims = R.boundary_ranges(two_j)
    vecs = [np.sqrt(lo + 2 * np.arange(n) + 1.0) for lo, n in dims]
    return np.einsum("a,b,c,d,e->abcde", *vecs)


def vertex_tensor(two_j, dl, boosters, shells=None, normalise=True, i1_rows=None):
    """FP64 vertex tensor A[i1, i2, i3, i4, i5] (row-major, i5 fastest).

    ``boosters`` is the packed buffer of raw B4 values (no dimension factors).  ``shells``
    restricts the sum to a subset of shell tuples (default: all of them); the result is
    then the partial sum over those shells.  ``i1_rows`` computes only those rows of the
    gauge-fixed intertwiner i1 (a reduced boundary-intertwiner range, Sec. 3.1 and 3.2); the
    result then has len(i1_rows) rows in that order.
    """
    R.check_spins(two_j, dl)
    blocks = unpack_boosters(two_j, dl, boosters)
    dims = tuple(n for _, n in R.boundary_ranges(two_j))
    if i1_rows is not None:
        i1_rows = [int(n) for n in i1_rows]
        if any(n < 0 or n >= dims[0] for n in i1_rows):
            raise ValueError("i1 row outside the boundary-intertwiner range")
        dims = (len(i1_rows),) + dims[1:]
    s = np.zeros(dims)
    c = np.zeros(dims)
    for shell in (R.all_shells(dl) if shells is None else shells):
        term = shell_contribution(two_j, dl, blocks, shell, i1_rows)
        if term is None:
            continue
        # Neumaier compensated summation, elementwise.
        t = s + term
        c += np.where(np.abs(s) >= np.abs(term), (s - t) + term, (term - t) + s)
        s = t
    a = s + c
    if not normalise:
        return a
    norm = _normalisation(two_j)
    return a * (norm if i1_rows is None else norm[i1_rows])


def vertex_tensor_mp(two_j, dl, boosters, dps=30):
    """Vertex tensor with every operation in mpmath at ``dps`` digits (tiny inputs only).

    Loops directly over shells, intertwiners and x; 6j symbols come from their exact
    rational form.  Returns a numpy array of Python ``mpf`` objects.
    """
    import mpmath

    with mpmath.workdps(dps):
        return _vertex_tensor_mp(two_j, dl, boosters, mpmath.mp)


def _vertex_tensor_mp(two_j, dl, boosters, mp):
    R.check_spins(two_j, dl)
    blocks = unpack_boosters(two_j, dl, boosters)
    bnd = R.boundary_ranges(two_j)
    dims = tuple(n for _, n in bnd)

    def sixj_mp(*args):
        s, p = sixj_exact(*args)
        if s == 0:
            return mp.mpf(0)
        return mp.mpf(s.numerator) / s.denominator * mp.sqrt(mp.mpf(p.numerator) / p.denominator)

    from .fifteenj import x_range, phase15
    acc = np.empty(dims, dtype=object)
    for idx in np.ndindex(*dims):
        acc[idx] = mp.mpf(0)
    for shell in R.all_shells(dl):
        two_l = R.shell_spins(two_j, shell)
        kr = [R.virtual_range(two_l, e) for e in range(2, 6)]
        if any(d == 0 for _, d in kr):
            continue
        l = lambda n: two_l[R.LINK[n]]  # noqa: E731
        ms = {e: blocks[(e, R.edge_triple_index(e, shell, dl))] for e in range(2, 6)}
        for n1 in range(dims[0]):
            i1 = bnd[0][0] + 2 * n1
            for ks in np.ndindex(*(d for _, d in kr)):
                k2, k3, k4, k5 = (kr[q][0] + 2 * ks[q] for q in range(4))
                w = mp.mpf(0)
                for x in x_range(i1, k2, k3, k4, k5, two_l):
                    w += ((x + 1) * sixj_mp(i1, l("25"), x, k5, l("14"), l("15"))
                          * sixj_mp(l("14"), k5, x, l("35"), k4, l("45"))
                          * sixj_mp(k4, l("35"), x, k3, l("24"), l("34"))
                          * sixj_mp(l("24"), k3, x, l("13"), k2, l("23"))
                          * sixj_mp(k2, l("13"), x, i1, l("25"), l("12")))
                if w == 0:
                    continue
                w *= phase15(i1, k2, k3, k4, k5, two_l)
                kk = (k2, k3, k4, k5)
                for rest in np.ndindex(*dims[1:]):
                    prod = w
                    for q in range(4):
                        prod *= mp.mpf(float(ms[q + 2][rest[q], ks[q]])) * (kk[q] + 1)
                    acc[(n1,) + rest] += prod
    for idx in np.ndindex(*dims):
        norm = mp.mpf(1)
        for q in range(5):
            norm *= mp.sqrt(bnd[q][0] + 2 * idx[q] + 1)
        acc[idx] *= norm
    return acc


def bf_vertex(two_j):
    """SU(2) BF vertex prod_e sqrt(2 i_e + 1) {15j}(j; i1..i5): the Delta s = 0 limit of
    eq. (vertex-ampl) with (2 k_e + 1) B_e = delta(i_e, k_e) (the 15j tensor of Sec. 3.2)."""
    R.check_spins(two_j, 0)
    bnd = R.boundary_ranges(two_j)
    dims = tuple(n for _, n in bnd)
    a = np.zeros(dims)
    for idx in np.ndindex(*dims):
        two_i = [bnd[q][0] + 2 * idx[q] for q in range(5)]
        a[idx] = fifteenj(*two_i, list(two_j))
    return a * _normalisation(two_j)
