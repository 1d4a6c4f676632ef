"""Write oracle vertex tensors used by the full-size parity tests.

Calls only the oracle and the seeded input generators.  Output: ``vertex_<name>.npz`` with the
spins, the shell count, the booster seed and A[i1..i5] (float64).  The shell sum is split over
worker processes by contiguous shell ranges and the partial tensors are summed in range order.

    python tests/golden/make_golden.py            # j = 3, dl = 8 (about 4 minutes on 8 cores)
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import ranges as R  # noqa: E402
from oracle import vertex as V  # noqa: E402


def _part(args):
    two_j, dl, seed, lo, hi = args
    b = workloads.synthetic_boosters(seed, R.block_shapes(two_j, dl))
    return V.vertex_tensor(two_j, dl, b, shells=R.all_shells(dl)[lo:hi])


def make(cfg, procs=8, pieces=64):
    two_j, dl, seed = cfg["two_j"], cfg["dl"], cfg["booster_seed"]
    n = (dl + 1) ** 6
    bounds = [n * q // pieces for q in range(pieces + 1)]
    jobs = [(two_j, dl, seed, bounds[q], bounds[q + 1]) for q in range(pieces)]
    with Pool(procs) as pool:
        parts = pool.map(_part, jobs)
    a = np.zeros_like(parts[0])
    for p in parts:
        a += p
    out = os.path.join(HERE, f"vertex_{cfg['name']}.npz")
    np.savez_compressed(out, two_j=np.array(two_j), dl=dl, booster_seed=seed, A=a)
    return out


if __name__ == "__main__":
    print(make(workloads.CFG2))
