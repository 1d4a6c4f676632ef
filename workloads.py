"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and spin labels only; it contains none of the arithmetic
of the vertex tensor.  Shapes (booster block sizes, intertwiner dimensions) are passed in by
the caller, which computes them itself.

Spins are in two-units and follow the link order (12, 13, 14, 15, 23, 24, 25, 34, 35, 45).

Workloads (shaped like the paper's: equilateral 4-simplices with growing spin and shell
count, Sec. 3.3 "Vertex tensor", and irregular boundaries as in Sec. 4):

* ``equilateral``  : all ten spins equal (j = 1, 3, 4 in the single-configuration cases).
* ``random_batch`` : i.i.d. spins from a given set, redrawn until every node admits an
                     intertwiner (even two-j sum and the polygon inequality at each of the
                     five nodes), with a per-configuration shell count.
"""
import numpy as np

# The four links meeting at each node of the 4-simplex boundary graph.
_NODE_LINKS = ((0, 1, 2, 3), (4, 5, 6, 0), (7, 8, 1, 4), (9, 2, 5, 7), (3, 6, 8, 9))


def _node_admissible(two_j):
    for node in _NODE_LINKS:
        s = [two_j[n] for n in node]
        if sum(s) % 2:
            return False
        if 2 * max(s) > sum(s):          # polygon inequality for four spins
            return False
    return True


def equilateral(two_j, dl):
    return [int(two_j)] * 10, int(dl)


def random_batch(seed, count, two_j_choices, dl_range=None, dl_fixed=None):
    """``count`` admissible configurations ``(two_j[10], dl)`` drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    out = []
    choices = np.asarray(two_j_choices)
    while len(out) < count:
        two_j = [int(v) for v in rng.choice(choices, size=10)]
        if not _node_admissible(two_j):
            continue
        if dl_fixed is not None:
            dl = int(dl_fixed)
        else:
            dl = int(rng.integers(dl_range[0], dl_range[1] + 1))
        out.append((two_j, dl))
    return out


def synthetic_boosters(seed, block_shapes):
    """Packed FP64 booster buffer: block (rows, cols) filled with N(0, 1) / cols."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in block_shapes:
        if rows * cols:
            parts.append(rng.standard_normal((rows, cols)).ravel() / cols)
    return np.concatenate(parts) if parts else np.zeros(0)


def boundary_vectors(seed, dims):
    """Five complex FP64 vectors of the given lengths, Gaussian entries, unit 2-norm."""
    rng = np.random.default_rng(seed)
    out = []
    for n in dims:
        v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        out.append(v / np.linalg.norm(v))
    return out


# The five workloads of the benchmark and of the parity tests.
CFG1 = dict(name="j1_dl3", two_j=[2] * 10, dl=3, booster_seed=1001)
CFG2 = dict(name="j3_dl8", two_j=[6] * 10, dl=8, booster_seed=1002)
CFG4 = dict(name="j4_dl8_adjoint", two_j=[8] * 10, dl=8, booster_seed=1004, psi_seed=1004)


def cfg3_batch():
    """64 configurations, j in {1/2 .. 6}, dl uniform in 3..10 (seed 1003)."""
    return random_batch(1003, 64, list(range(1, 13)), dl_range=(3, 10))


def cfg5_batch():
    """16 configurations, j in {5, 5.5, 6, 6.5, 7}, dl = 6 (seed 1005)."""
    return random_batch(1005, 16, [10, 11, 12, 13, 14], dl_fixed=6)


CFG3_SEED, CFG5_SEED = 1003, 1005


def batch_booster_seed(batch_seed, c):
    """Seed of the synthetic boosters of configuration ``c`` of a seeded batch."""
    return batch_seed + 1000 + c
