"""Index ranges of the vertex tensor computation (oracle; test infrastructure only).

Conventions (all spins in two-units):

* Boundary links are ordered (12, 13, 14, 15, 23, 24, 25, 34, 35, 45): the order in which the
  paper lists the ten spins of a 4-simplex (Sec. 4.1, boundary spins j_1a = 5 lambda,
  j_ab = 2 lambda, passed as ``[5 5 5 5 2 2 2 2 2 2]``).
* Edge e carries the four links of the booster tensors of the framed algorithm in Sec. 3.1
  (step 3); its intertwiner couples the first two links and the last two:
      e1: (12 13)(14 15)   e2: (23 24)(25 12)   e3: (34 35)(13 23)
      e4: (45 14)(24 34)   e5: (15 25)(35 45)
  These pairings are also the triads of the 6j symbols in eq. (15j).
* Virtual spins l_ab = j_ab + o_ab, o_ab in 0..dl, on the six links not touching node 1
  (eq. (vertex-ampl): l_12..l_15 are gauge-fixed to the boundary spins; the homogeneous cutoff
  is the "number of shells" Delta s).  A shell is the 6-tuple
  (o23, o24, o25, o34, o35, o45); shells are numbered lexicographically with o45 fastest.
* The virtual intertwiners k_e (e = 2..5) use the same pairings with l in place of j.
* Intertwiner index n <-> value lo + n, ascending (Sec. 3.2: ``v.a[1,1,1,1,1]`` is the
  amplitude with all intertwiners at their lowest value).
* Booster of edge e depends on the three virtual spins of that edge, in the order of the
  superscripts of step 3 of the framed algorithm:
      e2: (l23, l24, l25)  e3: (l34, l35, l23)  e4: (l45, l24, l34)  e5: (l25, l35, l45)
  The packed booster buffer stores, for e = 2..5 and for each offset triple
  t = (o1 * (dl+1) + o2) * (dl+1) + o3 in that order, a dim_i(e) x dim_k(e, t) block,
  row-major (i slow, k fast).  An empty k range gives an empty block.
"""
from itertools import product

LINKS = ("12", "13", "14", "15", "23", "24", "25", "34", "35", "45")
LINK = {name: n for n, name in enumerate(LINKS)}
VIRTUAL = ("23", "24", "25", "34", "35", "45")          # shell coordinates, in shell order

# The four links of each edge: intertwiner couples (first, second) and (third, fourth).
EDGE_LINKS = {
    1: ("12", "13", "14", "15"),
    2: ("23", "24", "25", "12"),
    3: ("34", "35", "13", "23"),
    4: ("45", "14", "24", "34"),
    5: ("15", "25", "35", "45"),
}
# Virtual links of the booster of edge e, in packing order.
EDGE_TRIPLE = {
    2: ("23", "24", "25"),
    3: ("34", "35", "23"),
    4: ("45", "24", "34"),
    5: ("25", "35", "45"),
}


def coupled_range(two_a, two_b, two_c, two_d):
    """Intertwiner range of (a b)(c d): returns (two_lo, dim); dim = 0 when empty."""
    if (two_a + two_b + two_c + two_d) % 2:
        return 0, 0
    lo = max(abs(two_a - two_b), abs(two_c - two_d))
    hi = min(two_a + two_b, two_c + two_d)
    if lo > hi:
        return lo, 0
    return lo, (hi - lo) // 2 + 1


def check_spins(two_j, dl):
    """Raise ValueError for inputs that define no vertex tensor."""
    if len(two_j) != 10:
        raise ValueError("ten boundary spins are required")
    if any(int(t) != t or t < 0 for t in two_j):
        raise ValueError("spins must be non-negative (given in two-units)")
    if int(dl) != dl or dl < 0:
        raise ValueError("the number of shells must be a non-negative integer")
    for e in range(1, 6):
        _, dim = coupled_range(*(two_j[LINK[n]] for n in EDGE_LINKS[e]))
        if dim == 0:
            raise ValueError(f"node {e} admits no intertwiner")


def boundary_ranges(two_j):
    """[(two_lo, dim)] of the boundary intertwiners i1..i5."""
    return [coupled_range(*(two_j[LINK[n]] for n in EDGE_LINKS[e])) for e in range(1, 6)]


def shell_spins(two_j, shell):
    """Virtual spins of all ten links for a shell (o23, o24, o25, o34, o35, o45)."""
    two_l = list(two_j)
    for name, o in zip(VIRTUAL, shell):
        two_l[LINK[name]] = two_j[LINK[name]] + 2 * o
    return two_l


def virtual_range(two_l, e):
    """(two_lo, dim) of the virtual intertwiner k_e given all ten virtual spins."""
    return coupled_range(*(two_l[LINK[n]] for n in EDGE_LINKS[e]))


def all_shells(dl):
    """All (dl+1)^6 shells in lexicographic order (o45 fastest)."""
    return list(product(range(dl + 1), repeat=6))


def shell_is_live(two_j, shell):
    two_l = shell_spins(two_j, shell)
    return all(virtual_range(two_l, e)[1] > 0 for e in range(2, 6))


def live_shells(two_j, dl):
    return [s for s in all_shells(dl) if shell_is_live(two_j, s)]


def edge_triple_index(e, shell, dl):
    """Position of the booster block of edge e used by ``shell`` among the (dl+1)^3 triples."""
    o = dict(zip(VIRTUAL, shell))
    o1, o2, o3 = (o[n] for n in EDGE_TRIPLE[e])
    return (o1 * (dl + 1) + o2) * (dl + 1) + o3


def booster_layout(two_j, dl):
    """Packed booster layout.

    Returns ``(shapes, offsets)``: ``shapes[(e, t)] = (dim_i, dim_k, two_klo)`` and
    ``offsets`` the list of 4 (dl+1)^3 + 1 start offsets (in doubles) in packing order.
    """
    bnd = boundary_ranges(two_j)
    shapes = {}
    offsets = [0]
    for e in range(2, 6):
        for o1, o2, o3 in product(range(dl + 1), repeat=3):
            two_l = list(two_j)
            for name, o in zip(EDGE_TRIPLE[e], (o1, o2, o3)):
                two_l[LINK[name]] += 2 * o
            klo, kdim = virtual_range(two_l, e)
            t = (o1 * (dl + 1) + o2) * (dl + 1) + o3
            shapes[(e, t)] = (bnd[e - 1][1], kdim, klo)
            offsets.append(offsets[-1] + bnd[e - 1][1] * kdim)
    return shapes, offsets


def block_shapes(two_j, dl):
    """List of (rows, cols) of the packed booster blocks, in packing order."""
    shapes, _ = booster_layout(two_j, dl)
    return [shapes[(e, t)][:2] for e in range(2, 6) for t in range((dl + 1) ** 3)]
