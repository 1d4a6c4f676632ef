"""Write oracle vertex tensors used by the full-size parity tests.

Calls only the oracle and the seeded input generators.  Output: ``vertex_<name>.npz`` with the
spins, dl, the booster seed, the i1 rows computed (all of them unless a reduced boundary-
intertwiner range is asked for) and A[rows, i2..i5] (float64).  Entries with physical boosters
(the oracle's FP64 quadrature of eq. (booster) at gamma = 1.2) also store those boosters
(booster_seed -1).  The shell sum is split over worker
processes by contiguous shell ranges and the partial tensors are summed in range order.

    python tests/golden/make_golden.py               # every entry (about 35 min, 8 cores)
    python tests/golden/make_golden.py j3_dl8 ...     # the named entries only
    python tests/golden/make_golden.py irr_a irr_b    # the booster-only entries
"""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import boosters as B  # noqa: E402
from oracle import ranges as R  # noqa: E402
from oracle import vertex as V  # noqa: E402

GAMMA = 1.2


def _batch_entry(name, batch, seed, c, rows=None, dl=None):
    tj, d = batch[c]
    return name, dict(two_j=list(tj), dl=d if dl is None else dl,
                      booster_seed=W.batch_booster_seed(seed, c), rows=rows)


def _registry():
    g = {W.CFG2["name"]: dict(two_j=W.CFG2["two_j"], dl=W.CFG2["dl"], booster_seed=W.CFG2["booster_seed"], rows=None),
         "j4_dl8": dict(two_j=W.CFG4["two_j"], dl=W.CFG4["dl"], booster_seed=W.CFG4["booster_seed"], rows=None)}
    b3, b5 = W.cfg3_batch(), W.cfg5_batch()
    # Irregular batch: the eight configurations with the least work in full, and the four with the
    # most work on a reduced i1 range (first and last row, or the middle row).
    for c in (55, 52, 40, 6, 22, 25, 1, 53):
        g.update([_batch_entry(f"b3_c{c:02d}", b3, W.CFG3_SEED, c)])
    for c, rows in ((7, [0, 7]), (41, [0, 8]), (0, [4]), (45, [3])):
        g.update([_batch_entry(f"b3_c{c:02d}_rows", b3, W.CFG3_SEED, c, rows)])
    # Large spins: two configurations on two i1 rows each, and one at dl = 2 in full.
    for c, rows in ((0, [0, 10]), (3, [5, 13])):
        g.update([_batch_entry(f"b5_c{c:02d}_rows", b5, W.CFG5_SEED, c, rows)])
    g.update([_batch_entry("b5_c00_dl2", b5, W.CFG5_SEED, 0, None, dl=2)])
    # The large-spin configuration with the widest intertwiner ranges (13, 13, 13, 13, 12), on its
    # first and last i1 rows.
    g.update([_batch_entry("b5_c05_rows", b5, W.CFG5_SEED, 5, [0, 12])])
    # A configuration whose 8-wide intertwiner tiles need 32-wide virtual windows (dl = 10).
    g["cls1_dl10"] = dict(two_j=[1, 3, 6, 2, 11, 9, 1, 7, 9, 10], dl=10, booster_seed=2010, rows=None)
    # Physical boosters: the j = 1, dl = 3 vertex in full and the j = 3, dl = 8 vertex on its
    # first and last i1 rows.
    g["j1_dl3_phys"] = dict(two_j=W.CFG1["two_j"], dl=W.CFG1["dl"], booster_seed=-1, rows=None)
    g["j3_dl8_phys"] = dict(two_j=W.CFG2["two_j"], dl=W.CFG2["dl"], booster_seed=-1, rows=[0, 6])
    return g


GOLDEN = _registry()

# Boosters alone (the oracle's FP64 quadrature of eq. (booster) at gamma = 1.2), for the parity of
# the device booster builder on irregular spins: ``boosters_<name>.npz`` with the spins, dl,
# gamma and the packed boosters.
BOOSTER_GOLDEN = {"irr_a": ([4, 1, 1, 4, 4, 3, 3, 1, 4, 1], 1),
                  "irr_b": ([2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 1),
                  # configuration 0 of the large-spin batch (spins 5..7) at dl = 0
                  "b5_c00_dl0": (list(W.cfg5_batch()[0][0]), 0)}


def _part(args):
    two_j, dl, b, rows, lo, hi = args
    return V.vertex_tensor(two_j, dl, b, shells=R.all_shells(dl)[lo:hi], i1_rows=rows)


def make(name, procs=8, pieces=64):
    e = GOLDEN[name]
    two_j, dl, seed, rows = e["two_j"], e["dl"], e["booster_seed"], e["rows"]
    n = (dl + 1) ** 6
    pieces = min(pieces, n)
    bounds = [n * q // pieces for q in range(pieces + 1)]
    if seed < 0:
        b, imag, err = B.boosters(two_j, dl, GAMMA)
        assert imag <= 1e-14 * np.abs(b).max() and err <= 1e-13 * np.abs(b).max(), (imag, err)
    else:
        b = W.synthetic_boosters(seed, R.block_shapes(two_j, dl))
    jobs = [(two_j, dl, b, rows, bounds[q], bounds[q + 1]) for q in range(pieces)]
    with Pool(procs) as pool:
        parts = pool.map(_part, jobs)
    a = np.zeros_like(parts[0])
    for p in parts:
        a += p
    nrow = R.boundary_ranges(two_j)[0][1]
    out = os.path.join(HERE, f"vertex_{name}.npz")
    extra = dict(boosters=b, gamma=GAMMA) if seed < 0 else {}
    np.savez_compressed(out, two_j=np.array(two_j), dl=dl, booster_seed=seed,
                        rows=np.arange(nrow) if rows is None else np.array(rows), A=a, **extra)
    return out


def make_boosters(name):
    two_j, dl = BOOSTER_GOLDEN[name]
    b, imag, err = B.boosters(two_j, dl, GAMMA)
    assert imag <= 1e-14 * np.abs(b).max() and err <= 1e-13 * np.abs(b).max(), (imag, err)
    out = os.path.join(HERE, f"boosters_{name}.npz")
    np.savez_compressed(out, two_j=np.array(two_j), dl=dl, gamma=GAMMA, boosters=b)
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or list(GOLDEN) + list(BOOSTER_GOLDEN)
    for nm in names:
        t = time.time()
        path = make_boosters(nm) if nm in BOOSTER_GOLDEN else make(nm)
        print(path, f"{time.time() - t:.0f} s", flush=True)
