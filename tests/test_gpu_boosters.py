"""The device booster builder (eq. (booster), Sec. 3.1 "Booster coefficients") against the
oracle's FP64 quadrature, through the C ABI.

Bars:
* 3jm symbols: within 4 ulp of the exactly rounded oracle value; exact zeros within 1e-28.
* Boosters: normwise relative error max|GPU - oracle| / max|oracle| <= 1e-10; both sides stop
  refining when their |61-point - 30-point| estimate is below 1e-13 of the largest entry, and
  the imaginary parts must vanish (<= 1e-12 of the largest entry).
* End to end: the vertex tensor built on the device boosters against the stored oracle tensor
  (built on the oracle's boosters) within 1e-10.
"""
import os
import random
import sys

import numpy as np
import pytest

from oracle import boosters as Bo

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-10


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2107_13952_amd as lib
    return lib


def normwise(a, ref):
    ref = np.asarray(ref)
    return np.abs(np.asarray(a) - ref).max() / np.abs(ref).max()


def test_threejm_device_vs_exact(lib):
    rng = random.Random(5)
    args = []
    while len(args) < 3000:
        j1, j2 = rng.randint(0, 30), rng.randint(0, 30)
        j3 = rng.randrange(abs(j1 - j2), j1 + j2 + 1, 2) if rng.random() < 0.9 else rng.randint(0, 30)
        m1 = rng.randrange(-j1, j1 + 1, 2) if j1 or rng.random() < 0.5 else 0
        m2 = rng.randrange(-j2, j2 + 1, 2) if j2 or rng.random() < 0.5 else 0
        m3 = -(m1 + m2) if rng.random() < 0.9 else rng.randint(-j3, j3)
        args.append((j1, j2, j3, m1, m2, m3))
    note("3jm: 3000 symbols")
    got = lib.threejm_batch(args).cpu().numpy()
    for a, g in zip(args, got):
        ref = Bo.threejm(*a)
        if ref == 0.0:
            # An exact zero of a cancelling Racah sum leaves a double-double rounding residue.
            assert abs(g) <= 1e-28, (a, g)
        else:
            assert abs(g - ref) <= 4 * np.spacing(abs(ref)), (a, g, ref)
    with pytest.raises(lib.EprlError):
        lib.threejm_batch([(202, 2, 200, 0, 0, 0)])


def _check(lib, two_j, dl, ref, gamma=1.2):
    b, info = lib.boosters(two_j, dl, gamma)
    b = b.cpu().numpy()
    err = normwise(b, ref)
    note(f"  n={info['n']} error estimate {info['error']:.2e} imag {info['imag']:.2e}; "
         f"normwise vs oracle {err:.2e}")
    scale = np.abs(ref).max()
    assert err <= TOL
    assert info["error"] <= 1e-13 * scale * 1.0001
    assert info["imag"] <= 1e-12 * scale
    return b


@pytest.mark.parametrize("name", ["vertex_j1_dl3_phys", "vertex_j3_dl8_phys", "boosters_irr_a",
                                  "boosters_irr_b", "boosters_b5_c00_dl0"])
def test_boosters_against_stored_oracle(lib, name):
    path = os.path.join(GOLDEN, name + ".npz")
    g = np.load(path)
    two_j, dl = [int(v) for v in g["two_j"]], int(g["dl"])
    note(f"boosters {name}: two_j={two_j} dl={dl}")
    _check(lib, two_j, dl, g["boosters"], float(g["gamma"]))


@pytest.mark.parametrize("two_j,dl", [([1] * 10, 2), ([2] * 10, 0)])
def test_boosters_against_oracle(lib, two_j, dl):
    note(f"boosters {two_j} dl={dl} (oracle computed here)")
    ref, imag, err = Bo.boosters(two_j, dl, 1.2)
    _check(lib, two_j, dl, ref)


def test_all_zero_spin_booster_closed_form(lib):
    """All spins 0: one 1 x 1 block per edge equal to the closed form of the oracle's pin,
    (4 pi gamma^4)^-1 [(pi gamma coth(pi gamma) - 1) / 2 - (2 pi gamma coth(2 pi gamma) - 1) / 8]."""
    gamma = 1.2
    b, info = lib.boosters([0] * 10, 0, gamma)
    x = np.pi * gamma
    closed = ((x / np.tanh(x) - 1) / 2 - (2 * x / np.tanh(2 * x) - 1) / 8) / (4 * np.pi * gamma ** 4)
    assert b.numel() == 4
    assert np.abs(b.cpu().numpy() - closed).max() <= 1e-12 * closed


def test_vertex_on_device_boosters(lib):
    """j = 1, dl = 3: the vertex tensor on the device's boosters against the stored oracle tensor
    on the oracle's boosters."""
    g = np.load(os.path.join(GOLDEN, "vertex_j1_dl3_phys.npz"))
    two_j, dl = [int(v) for v in g["two_j"]], int(g["dl"])
    b, _ = lib.boosters(two_j, dl, float(g["gamma"]))
    a = lib.vertex_tensor(two_j, dl, float(g["gamma"]), b).cpu().numpy()
    err = normwise(a, g["A"])
    note(f"vertex on device boosters: normwise {err:.2e}")
    assert err <= TOL


def test_boosters_invalid_arguments(lib):
    with pytest.raises(lib.EprlError):
        lib.boosters([2] * 10, 1, -1.0)
    with pytest.raises(lib.EprlError):
        lib.boosters([2] * 10, 1, 1.2, tol=0.0)
