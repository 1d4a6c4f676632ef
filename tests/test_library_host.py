"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol the
header declares, and its host-only planner agrees with the oracle on ranges, the packed
booster layout and the shell / term counts."""
import re
import os

import numpy as np
import pytest

from oracle import ranges as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        import paper_2107_13952_amd as lib
    except ImportError as exc:  # pragma: no cover - the build step must run first
        pytest.fail(f"library not built: {exc}")
    return lib


def test_exports_every_declared_symbol():
    lib = _lib()
    header = open(os.path.join(ROOT, "include", "eprl.h")).read()
    declared = sorted(set(re.findall(r"\b(eprl_[a-z0-9_]+)\s*\(", header)))
    assert declared, "no entry points found in the header"
    for name in declared:
        assert hasattr(lib._lib, name), name
    assert sorted(lib.EXPORTED) == declared


CONFIGS = [([2] * 10, 3), ([6] * 10, 2), ([2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 2),
           ([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 1), ([4, 1, 1, 4, 4, 3, 3, 1, 4, 1], 3)]


@pytest.mark.parametrize("two_j,dl", CONFIGS)
def test_layout_matches_oracle(two_j, dl):
    lib = _lib()
    dims, ilo, offs = lib.layout(two_j, dl)
    bnd = R.boundary_ranges(two_j)
    assert dims == [n for _, n in bnd]
    assert ilo == [lo for lo, _ in bnd]
    _, ref = R.booster_layout(two_j, dl)
    np.testing.assert_array_equal(offs, np.array(ref, dtype=np.int64))


@pytest.mark.parametrize("two_j,dl", CONFIGS[:3])
def test_counts_match_oracle(two_j, dl):
    lib = _lib()
    live, terms = lib.count_terms(two_j, dl)
    shells = R.live_shells(two_j, dl)
    assert live == len(shells)
    ref = 0
    n1 = R.boundary_ranges(two_j)[0][1]
    for s in shells:
        two_l = R.shell_spins(two_j, s)
        t = n1
        for e in range(2, 6):
            t *= R.virtual_range(two_l, e)[1]
        ref += t
    assert terms == ref


def test_cfg1_counts():
    lib = _lib()
    live, terms = lib.count_terms([2] * 10, 3)
    assert live == 3435


def test_invalid_inputs_rejected():
    lib = _lib()
    with pytest.raises(lib.EprlError):
        lib.layout([1, 2, 2, 2, 2, 2, 2, 2, 2, 2], 1)       # node 1 has an odd spin sum
    with pytest.raises(lib.EprlError):
        lib.layout([2] * 10, -1)
    with pytest.raises(lib.EprlError):
        lib.layout([20, 2, 2, 2, 2, 2, 2, 2, 2, 2], 0)      # polygon inequality violated


def test_factorised_path_limits():
    # 16 values per virtual spin (dl = 15) is the largest grid of the factorised order; beyond it
    # and for intertwiner dimensions above 16 only the per-shell order applies.
    lib = _lib()
    assert lib.count_work([1] * 10, 15)["ring_class"] >= 0
    assert lib.count_work([1] * 10, 16)["ring_class"] == -1
    assert lib.count_work([6] * 10, 8)["ring_class"] == 0


def test_spin_limit_of_the_6j_tables():
    # Every 6j argument of the tables must stay within two_j = 200, the range of the device
    # evaluation: the largest virtual spin, and intertwiners and x through the boundary spins.
    lib = _lib()
    lib.layout([2] * 10, 97)                                 # x up to i1 + l25 = 4 + 196
    with pytest.raises(lib.EprlError) as exc:
        lib.layout([2] * 10, 98)                             # 4 + 198 = 202
    assert exc.value.code == -4
    lib.layout([50] * 10, 0)                                 # intertwiners up to 100, x up to 150
    with pytest.raises(lib.EprlError) as exc:
        lib.layout([100] * 10, 0)                            # x up to i1 + l25 = 300
    assert exc.value.code == -4
