"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars:
* 6j symbols: every device value within 4 ulp of the exactly rounded oracle value; exact
  zeros of the Racah sum within 1e-28.
* {15j} tensors W of single shells and vertex tensors A: normwise relative error
  max|GPU - oracle| / max|oracle| <= 1e-10 (the parity bar of the method in FP64); typical
  observed values are ~1e-15.
* Contraction and gradients: relative error <= 1e-10 against the oracle's FP64 values;
  adjoint against central finite differences within 2e-8.
Shell-range partial sums must add up to the full tensor and repeated calls must be bitwise
identical (fixed-order reductions).
"""
import os
import random
import sys

import numpy as np
import pytest

import workloads
from oracle import ranges as R
from oracle import vertex as V
from oracle import contract as C
from oracle.fifteenj import fifteenj_block
from oracle.wigner import sixj, triad

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import GOLDEN  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-10


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2107_13952_amd as lib
    return lib


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(params=["shell", "ring", "ring_valu"])
def algo(request, lib):
    """Run a test with one evaluation order of the shell sum, restoring the default after."""
    lib.set_algorithm(request.param)
    yield request.param
    lib.set_algorithm("auto")


def vertex_or_skip(lib, algo, *args, **kw):
    try:
        return lib.vertex_tensor(*args, **kw)
    except lib.EprlError as exc:
        if algo in ("ring", "ring_valu") and exc.code == -4:
            pytest.skip("factorised path not applicable to these dimensions")
        raise


def normwise(a, ref):
    ref = np.asarray(ref)
    scale = np.abs(ref).max()
    return np.abs(np.asarray(a) - ref).max() / (scale if scale > 0 else 1.0)


def boosters_for(torch, two_j, dl, seed):
    b = workloads.synthetic_boosters(seed, R.block_shapes(two_j, dl))
    return b, torch.from_numpy(b).cuda()


# ------------------------------------------------------------------ 6j symbols

def test_sixj_device_vs_exact(lib, torch):
    rng = random.Random(42)
    args = []
    while len(args) < 3000:
        s = [rng.randint(0, 40) for _ in range(6)]
        a, b, c, d, e, f = s
        if triad(a, b, c) and triad(a, e, f) and triad(d, b, f) and triad(d, e, c):
            args.append(s)
    # large spins up to the supported two_j = 200 (where the Racah sum cancels most), and
    # non-admissible ones
    while len(args) < 3300:
        s = [rng.randint(100, 200) for _ in range(6)]
        a, b, c, d, e, f = s
        if triad(a, b, c) and triad(a, e, f) and triad(d, b, f) and triad(d, e, c):
            args.append(s)
    args += [[120, 118, 60, 80, 90, 100], [200, 200, 200, 200, 200, 200], [2, 2, 2, 2, 2, 9]]
    note(f"sixj_batch: {len(args)} symbols")
    out = lib.sixj_batch(np.array(args)).cpu().numpy()
    ref = np.array([sixj(*s) for s in args])
    zero = ref == 0.0
    # non-trivial zeros of the Racah sum come out at the double-double residual level
    assert np.all(np.abs(out[zero]) <= 1e-28)
    ulp = np.abs(out[~zero] - ref[~zero]) / np.spacing(np.abs(ref[~zero]))
    assert ulp.max() <= 4, ulp.max()


# ------------------------------------------------------------------ {15j} of single shells

SHELL_CASES = [([2] * 10, 3), ([2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 2), ([6] * 10, 8),
               ([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 2)]


@pytest.mark.parametrize("two_j,dl", SHELL_CASES)
def test_shell_fifteenj(lib, torch, two_j, dl):
    shells = R.live_shells(two_j, dl) if dl <= 3 else None
    rng = random.Random(7)
    nd = dl + 1
    picks = []
    while len(picks) < 6:
        s = tuple(rng.randrange(nd) for _ in range(6))
        if R.shell_is_live(two_j, s):
            picks.append(s)
    if shells:
        picks += [shells[0], shells[-1]]
    for s in picks:
        idx = 0
        for o in s:
            idx = idx * nd + o
        note(f"shell_fifteenj {two_j} dl={dl} shell={s}")
        w = lib.shell_fifteenj(two_j, dl, idx).cpu().numpy()
        two_l = R.shell_spins(two_j, s)
        kr = [R.virtual_range(two_l, e) for e in range(2, 6)]
        ref = fifteenj_block(R.boundary_ranges(two_j)[0], kr, two_l)
        assert w.shape == ref.shape
        assert normwise(w, ref) <= 1e-13, (s, normwise(w, ref))


# ------------------------------------------------------------------ vertex tensors

SMALL = [([2] * 10, 3, 1001),                                  # j = 1, dl = 3 (cfg1 shape)
         ([2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 2, 11),               # half-integer, irregular
         ([1] * 10, 2, 12),                                     # all spins 1/2
         ([4, 1, 1, 4, 4, 3, 3, 1, 4, 1], 3, 13),               # ragged k ranges
         ([6] * 10, 1, 14),                                     # j = 3 (cfg2 spins), dl = 1
         ([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 1, 15),     # dims 11 (wide tile path)
         ([8] * 10, 0, 16)]                                     # Delta s = 0


@pytest.mark.parametrize("two_j,dl,seed", SMALL)
def test_vertex_tensor_small(lib, torch, algo, two_j, dl, seed):
    b, bd = boosters_for(torch, two_j, dl, seed)
    note(f"vertex_tensor [{algo}] {two_j} dl={dl}")
    a = vertex_or_skip(lib, algo, two_j, dl, 1.2, bd).cpu().numpy()
    ref = V.vertex_tensor(two_j, dl, b)
    err = normwise(a, ref)
    note(f"  normwise error {err:.3e}")
    assert err <= TOL


# Boundary dimensions above 8 with every virtual range at most 8 (only i1 above 8), with and
# without shells: "ring" runs them in the all-matrix-core kernel (class 8), "ring_valu" in the
# 16-wide vector-ALU kernel with 8-wide virtual tiles (class 4), which no workload above reaches.
TILE_CLASS_CASES = [([14, 15, 15, 12, 3, 16, 1, 0, 16, 3], 3, 51, 8),
                    ([14, 8, 13, 11, 12, 8, 2, 5, 7, 6], 0, 52, 8),
                    ([13, 10, 12, 11, 0, 5, 10, 13, 9, 0], 0, 53, 8)]


@pytest.mark.parametrize("two_j,dl,seed,cls", TILE_CLASS_CASES)
def test_tile_class_against_oracle(lib, torch, algo, two_j, dl, seed, cls):
    assert lib.count_work(two_j, dl)["ring_class"] == cls
    b, bd = boosters_for(torch, two_j, dl, seed)
    note(f"tile class {cls} [{algo}] {two_j} dl={dl}")
    a = vertex_or_skip(lib, algo, two_j, dl, 1.2, bd).cpu().numpy()
    err = normwise(a, V.vertex_tensor(two_j, dl, b))
    note(f"  normwise error {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("dl", [0, 2])
def test_all_spins_zero(lib, torch, algo, dl):
    """Degenerate vertex: all ten spins 0, one intertwiner per node (a 1x1x1x1x1 tensor)."""
    b, bd = boosters_for(torch, [0] * 10, dl, 17 + dl)
    note(f"all spins zero [{algo}] dl={dl}")
    a = vertex_or_skip(lib, algo, [0] * 10, dl, 1.2, bd).cpu().numpy()
    ref = V.vertex_tensor([0] * 10, dl, b)
    assert a.shape == (1, 1, 1, 1, 1)
    assert normwise(a, ref) <= TOL


def test_largest_shell_grid(lib, torch):
    """16 values per virtual spin (dl = 15), the largest grid of the factorised path: both orders
    agree on the full tensor and the per-shell order matches the oracle on the last 4000 shells
    (the largest virtual spins); dl = 16 runs in the per-shell order only."""
    two_j, dl = [1] * 10, 15
    b, bd = boosters_for(torch, two_j, dl, 18)
    n = (dl + 1) ** 6
    note("largest shell grid: dl=15 factorised vs per-shell")
    ring = lib.vertex_tensor(two_j, dl, 1.2, bd).cpu().numpy()
    lib.set_algorithm("shell")
    try:
        shell = lib.vertex_tensor(two_j, dl, 1.2, bd).cpu().numpy()
        part = lib.vertex_tensor_range(two_j, dl, 1.2, bd, n - 4000, n).cpu().numpy()
    finally:
        lib.set_algorithm("auto")
    assert normwise(ring, shell) <= 1e-12
    ref = V.vertex_tensor(two_j, dl, b, shells=R.all_shells(dl)[n - 4000:])
    assert normwise(part, ref) <= TOL
    note("dl=16: per-shell order only")
    b16, bd16 = boosters_for(torch, two_j, 16, 19)
    a16 = lib.vertex_tensor(two_j, 16, 1.2, bd16)
    assert torch.isfinite(a16).all()
    lib.set_algorithm("ring")
    try:
        with pytest.raises(lib.EprlError) as exc:
            lib.vertex_tensor(two_j, 16, 1.2, bd16)
        assert exc.value.code == -4
    finally:
        lib.set_algorithm("auto")


def test_bf_limit_identity_boosters(lib, torch, algo):
    two_j = [2, 3, 2, 1, 3, 2, 3, 1, 1, 3]
    shapes, offsets = R.booster_layout(two_j, 0)
    parts = []
    for e in range(2, 6):
        rows, cols, klo = shapes[(e, 0)]
        parts.append((np.eye(rows) / (klo + 2 * np.arange(cols) + 1.0)[None, :]).ravel())
    b = np.concatenate(parts)
    note(f"BF limit [{algo}]")
    a = vertex_or_skip(lib, algo, two_j, 0, 1.0, torch.from_numpy(b).cuda()).cpu().numpy()
    assert normwise(a, V.bf_vertex(two_j)) <= 1e-13


def test_range_additivity_and_determinism(lib, torch):
    two_j, dl = [6] * 10, 2
    b, bd = boosters_for(torch, two_j, dl, 21)
    n = (dl + 1) ** 6
    note("range additivity")
    full = lib.vertex_tensor(two_j, dl, 1.2, bd)
    again = lib.vertex_tensor(two_j, dl, 1.2, bd)
    assert torch.equal(full, again)
    part = lib.vertex_tensor_range(two_j, dl, 1.2, bd, 0, 300)
    lib.vertex_tensor_range(two_j, dl, 1.2, bd, 300, n, accumulate=True, out=part)
    assert normwise(part.cpu().numpy(), full.cpu().numpy()) <= 1e-14
    ref = V.vertex_tensor(two_j, dl, b, shells=R.all_shells(dl)[:300])
    mid = lib.vertex_tensor_range(two_j, dl, 1.2, bd, 0, 300).cpu().numpy()
    assert normwise(mid, ref) <= TOL


def core_index(shell, nd):
    """Core of a shell (o23, o24, o25, o34, o35, o45): ((o24 nd + o25) nd + o34) nd + o35."""
    return ((shell[1] * nd + shell[2]) * nd + shell[3]) * nd + shell[4]


# A 7^5 tensor in the 8-wide factorised kernel and an 11-dimensional one in the all-matrix-core
# kernel.
CORE_CASES = [([6] * 10, 2, 22, 0), ([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 1, 23, 8)]


@pytest.mark.parametrize("two_j,dl,seed,cls", CORE_CASES)
def test_core_ranges(lib, torch, two_j, dl, seed, cls):
    """Partial sums over ranges of cores (l24, l25, l34, l35) in the factorised order: the whole
    range gives the bits of the plain call, two ragged halves add up to the full tensor, a range
    matches the oracle on its shells, an empty range gives zeros, and invalid ranges are refused."""
    assert lib.count_work(two_j, dl)["ring_class"] == cls
    b, bd = boosters_for(torch, two_j, dl, seed)
    nd = dl + 1
    ncore = nd ** 4
    cut = ncore // 3 + 1
    ref_part = V.vertex_tensor(two_j, dl, b,
                               shells=[s for s in R.all_shells(dl) if core_index(s, nd) < cut])
    for algo in ("auto", "ring_valu"):
        lib.set_algorithm(algo)
        try:
            note(f"core ranges [{algo}] {two_j} dl={dl} cut={cut}/{ncore}")
            full = lib.vertex_tensor(two_j, dl, 1.2, bd)
            whole = lib.vertex_tensor_cores(two_j, dl, 1.2, bd, 0, ncore)
            assert torch.equal(full, whole)
            part = lib.vertex_tensor_cores(two_j, dl, 1.2, bd, 0, cut)
            err = normwise(part.cpu().numpy(), ref_part)
            note(f"  first range vs oracle {err:.3e}")
            assert err <= TOL
            lib.vertex_tensor_cores(two_j, dl, 1.2, bd, cut, ncore, accumulate=True, out=part)
            err = normwise(part.cpu().numpy(), full.cpu().numpy())
            note(f"  halves vs full {err:.3e}")
            assert err <= 1e-13
            empty = lib.vertex_tensor_cores(two_j, dl, 1.2, bd, cut, cut)
            assert not empty.any()
            for lo, hi in ((0, ncore + 1), (-1, 3), (5, 4)):
                with pytest.raises(lib.EprlError) as exc:
                    lib.vertex_tensor_cores(two_j, dl, 1.2, bd, lo, hi)
                assert exc.value.code == -1
        finally:
            lib.set_algorithm("auto")
    lib.set_algorithm("shell")
    try:
        with pytest.raises(lib.EprlError) as exc:
            lib.vertex_tensor_cores(two_j, dl, 1.2, bd, 0, ncore)
        assert exc.value.code == -1
    finally:
        lib.set_algorithm("auto")


def sub_boosters(two_j, dl_max, dl, b):
    """The packed boosters of dl taken out of a buffer packed for dl_max (same blocks, found by
    their offsets in the larger layout)."""
    _, offs = R.booster_layout(two_j, dl_max)
    n3 = (dl_max + 1) ** 3
    parts = []
    for e in range(4):
        for o1 in range(dl + 1):
            for o2 in range(dl + 1):
                for o3 in range(dl + 1):
                    q = e * n3 + (o1 * (dl_max + 1) + o2) * (dl_max + 1) + o3
                    parts.append(b[offs[q]:offs[q + 1]])
    return np.concatenate(parts)


@pytest.mark.parametrize("two_j,dl_max,seed", [([2] * 10, 3, 24),
                                               ([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 1, 25),
                                               ([4, 1, 1, 4, 4, 3, 3, 1, 4, 1], 0, 26)])
def test_shell_scan(lib, torch, two_j, dl_max, seed):
    """A(dl) for dl = 0..dl_max from one buffer packed for dl_max: each against the oracle at
    that dl and bitwise against the plain call on its own packed boosters."""
    b, bd = boosters_for(torch, two_j, dl_max, seed)
    note(f"shell scan {two_j} dl_max={dl_max}")
    scan = lib.vertex_tensor_scan(two_j, dl_max, 1.2, bd)
    assert scan.shape[0] == dl_max + 1
    for dl in range(dl_max + 1):
        bs = sub_boosters(two_j, dl_max, dl, b)
        err = normwise(scan[dl].cpu().numpy(), V.vertex_tensor(two_j, dl, bs))
        note(f"  dl={dl}: normwise error {err:.3e}")
        assert err <= TOL
        plain = lib.vertex_tensor(two_j, dl, 1.2, torch.from_numpy(bs).cuda())
        assert torch.equal(plain, scan[dl])
    again = lib.vertex_tensor_scan(two_j, dl_max, 1.2, bd)      # graph replay
    assert torch.equal(again, scan)


def test_shell_scan_full_size(lib, torch):
    """The scan of the j = 3 vertex over dl = 0..8 (its levels read the 6j tables of dl = 8):
    every level bitwise equal to the plain call on its own packed boosters (which builds its own
    tables), and the dl = 8 level equal to the stored oracle tensor when present."""
    import os
    cfg = workloads.CFG2
    two_j, dl_max = cfg["two_j"], cfg["dl"]
    b, bd = boosters_for(torch, two_j, dl_max, cfg["booster_seed"])
    note(f"shell scan {two_j} dl_max={dl_max} (full size)")
    scan = lib.vertex_tensor_scan(two_j, dl_max, 1.2, bd)
    for dl in range(dl_max + 1):
        plain = lib.vertex_tensor(two_j, dl, 1.2, torch.from_numpy(sub_boosters(two_j, dl_max, dl, b)).cuda())
        assert torch.equal(plain, scan[dl]), dl
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"vertex_{cfg['name']}.npz")
    if os.path.exists(path):
        g = np.load(path)
        assert list(g["two_j"]) == two_j and int(g["dl"]) == dl_max
        assert int(g["booster_seed"]) == cfg["booster_seed"]
        assert normwise(scan[dl_max].cpu().numpy(), g["A"]) <= TOL


def test_cfg2_full_size(lib, torch):
    """j = 3, dl = 8 at full size, in the launch configuration of the benchmark: the
    per-shell path on a contiguous block of shells against the oracle; both paths on the full
    tensor against each other, against the stored oracle tensor when present, for bitwise
    repeatability and (per-shell path) additivity of two halves."""
    import os
    cfg = workloads.CFG2
    two_j, dl = cfg["two_j"], cfg["dl"]
    b, bd = boosters_for(torch, two_j, dl, cfg["booster_seed"])
    n = (dl + 1) ** 6
    s0, s1 = 250000, 251500
    note("cfg2 sampled range [shell]")
    part = lib.vertex_tensor_range(two_j, dl, 1.2, bd, s0, s1).cpu().numpy()
    ref = V.vertex_tensor(two_j, dl, b, shells=R.all_shells(dl)[s0:s1])
    err = normwise(part, ref)
    note(f"  normwise error {err:.3e}")
    assert err <= TOL
    full = {}
    for name in ("shell", "ring"):
        lib.set_algorithm(name)
        try:
            note(f"cfg2 full tensor [{name}]")
            full[name] = lib.vertex_tensor(two_j, dl, 1.2, bd)
            again = lib.vertex_tensor(two_j, dl, 1.2, bd)
            assert torch.equal(full[name], again)
        finally:
            lib.set_algorithm("auto")
    halves = lib.vertex_tensor_range(two_j, dl, 1.2, bd, 0, n // 2)
    lib.vertex_tensor_range(two_j, dl, 1.2, bd, n // 2, n, accumulate=True, out=halves)
    shell = full["shell"].cpu().numpy()
    ring = full["ring"].cpu().numpy()
    assert normwise(halves.cpu().numpy(), shell) <= 1e-13
    err = normwise(ring, shell)
    note(f"  ring vs shell normwise {err:.3e}")
    assert err <= TOL
    gold = os.path.join(os.path.dirname(__file__), "golden", f"vertex_{cfg['name']}.npz")
    if os.path.exists(gold):
        g = np.load(gold)
        assert list(g["two_j"]) == two_j and int(g["dl"]) == dl and int(g["booster_seed"]) == cfg["booster_seed"]
        for name, a in (("shell", shell), ("ring", ring)):
            err = normwise(a, g["A"])
            note(f"  {name} vs stored oracle tensor {err:.3e}")
            assert err <= TOL


def load_golden(name, required=True):
    """A stored oracle tensor; a test that needs it is skipped if it has not been written
    (tests/golden/make_golden.py), one that only uses it as an extra check gets None."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"vertex_{name}.npz")
    if not os.path.exists(path):
        if required:
            pytest.skip(f"stored oracle tensor {name} not written")
        return None
    g = np.load(path)
    e = GOLDEN[name]
    assert list(g["two_j"]) == list(e["two_j"]) and int(g["dl"]) == e["dl"]
    assert int(g["booster_seed"]) == e["booster_seed"]
    return g


STORED = [n for n in GOLDEN if n != workloads.CFG2["name"]]


@pytest.mark.parametrize("name", STORED)
def test_stored_oracle_tensor(lib, torch, algo, name):
    """Irregular spins (every tile class), j = 4 and large-spin vertices at full size against
    oracle tensors written offline (all i1 rows, or a reduced i1 range for the largest); the
    j = 1 and j = 3 vertices also with the oracle's quadrature boosters (stored with them)."""
    e = GOLDEN[name]
    g = load_golden(name)
    if e["booster_seed"] < 0:
        bd = torch.from_numpy(np.ascontiguousarray(g["boosters"])).cuda()
    else:
        b, bd = boosters_for(torch, e["two_j"], e["dl"], e["booster_seed"])
    note(f"{name} [{algo}] two_j={e['two_j']} dl={e['dl']}")
    a = vertex_or_skip(lib, algo, e["two_j"], e["dl"], 1.2, bd).cpu().numpy()
    err = normwise(a[g["rows"]], g["A"])
    note(f"  normwise error {err:.3e}")
    assert err <= TOL


def test_batched_full_size(lib, torch):
    """The 64-configuration batch of the benchmark (true dl, 3..10) in one batched call: stored
    oracle tensors, bitwise equality with plain calls and with a replay of the captured graph."""
    configs = workloads.cfg3_batch()
    bds = [boosters_for(torch, tj, dl, workloads.batch_booster_seed(workloads.CFG3_SEED, c))[1]
           for c, (tj, dl) in enumerate(configs)]
    note("batched full size: capture")
    outs = lib.vertex_tensor_batched(configs, 1.2, bds)
    note("batched full size: replay")
    again = [torch.empty_like(a) for a in outs]
    lib.vertex_tensor_batched(configs, 1.2, bds, again)
    torch.cuda.synchronize()
    for a, r in zip(outs, again):
        assert torch.equal(a, r)
    for name in STORED:
        if not name.startswith("b3_"):
            continue
        c = int(name[4:6])
        g = load_golden(name, required=False)
        if g is None:
            continue
        err = normwise(outs[c].cpu().numpy()[g["rows"]], g["A"])
        note(f"  {name} normwise error {err:.3e}")
        assert err <= TOL
    for c in (55, 7, 41, 0):
        tj, dl = configs[c]
        assert torch.equal(outs[c], lib.vertex_tensor(tj, dl, 1.2, bds[c]))


def test_batched_large_spins(lib, torch):
    """The 16-configuration large-spin batch (intertwiner dimensions 11..14, dl = 6) in one batched
    call: stored oracle rows of two configurations and bitwise equality with plain calls."""
    configs = workloads.cfg5_batch()
    bds = [boosters_for(torch, tj, dl, workloads.batch_booster_seed(workloads.CFG5_SEED, c))[1]
           for c, (tj, dl) in enumerate(configs)]
    note("batched large spins")
    outs = lib.vertex_tensor_batched(configs, 1.2, bds)
    for name in ("b5_c00_rows", "b5_c03_rows", "b5_c05_rows"):
        c = int(name[4:6])
        g = load_golden(name, required=False)
        if g is None:
            continue
        err = normwise(outs[c].cpu().numpy()[g["rows"]], g["A"])
        note(f"  {name} normwise error {err:.3e}")
        assert err <= TOL
    for c in (0, 3, 5, 15):
        tj, dl = configs[c]
        assert torch.equal(outs[c], lib.vertex_tensor(tj, dl, 1.2, bds[c]))


def test_batch_graph_survives_factorial_table_growth(lib, torch):
    """A captured batch reads the context's factorial table; a later call that needs a larger
    table (6j arguments up to 200) reallocates it, and the next batched call must capture again
    rather than replay a graph holding the old address."""
    configs = [(tj, min(dl, 2)) for tj, dl in workloads.cfg3_batch()[:4]]
    bds = [boosters_for(torch, tj, dl, 3100 + c)[1] for c, (tj, dl) in enumerate(configs)]
    note("batch graph vs factorial table growth")
    first = [a.clone() for a in lib.vertex_tensor_batched(configs, 1.2, bds)]
    big = lib.sixj_batch(np.array([[200, 200, 200, 200, 200, 200]])).cpu().numpy()
    ref = sixj(200, 200, 200, 200, 200, 200)
    assert abs(big[0] - ref) <= 4 * np.spacing(abs(ref))
    with pytest.raises(lib.EprlError) as exc:
        lib.sixj_batch(np.array([[202, 200, 200, 200, 200, 200]]))
    assert exc.value.code == -4
    again = lib.vertex_tensor_batched(configs, 1.2, bds)
    torch.cuda.synchronize()
    for a, r in zip(first, again):
        assert torch.equal(a, r)


@pytest.mark.parametrize("two_j,dl,seed", [([4, 1, 1, 4, 4, 3, 3, 1, 4, 1], 3, 21),
                                          ([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 1, 22)])
def test_autotune(lib, torch, two_j, dl, seed):
    """The autotuner keeps a valid setting for the configuration's tile class; with it the tensor
    still matches the oracle, repeats bitwise and equals the batched result."""
    b, bd = boosters_for(torch, two_j, dl, seed)
    cls = lib.count_work(two_j, dl)["ring_class"]
    note(f"autotune {two_j} dl={dl} (tile class {cls})")
    res = lib.autotune(two_j, dl, bd)
    try:
        note(f"  chosen {res}")
        assert res["tile_class"] == cls
        assert res["target_workgroups"] in (2048, 4096, 8192, 16384)
        assert res["staging_level"] in ((2,) if cls < 4 else (0, 1, 2))
        a = lib.vertex_tensor(two_j, dl, 1.2, bd)
        assert torch.equal(a, lib.vertex_tensor(two_j, dl, 1.2, bd))
        assert normwise(a.cpu().numpy(), V.vertex_tensor(two_j, dl, b)) <= TOL
        (batched,) = lib.vertex_tensor_batched([(two_j, dl)], 1.2, [bd])
        assert torch.equal(batched, a)
        with pytest.raises(lib.EprlError):
            lib.set_tuning(9, 0, -1)
        with pytest.raises(lib.EprlError):
            lib.set_tuning(cls, 0, 3)
    finally:
        lib.set_tuning(cls, 0, -1)


def test_batched_equals_plain(lib, torch):
    configs = workloads.cfg3_batch()[:6]
    configs = [(tj, min(dl, 2)) for tj, dl in configs]
    bs = [boosters_for(torch, tj, dl, 3000 + c) for c, (tj, dl) in enumerate(configs)]
    note("batched vs plain")
    outs = lib.vertex_tensor_batched(configs, 1.2, [bd for _, bd in bs])
    for (tj, dl), (b, bd), a in zip(configs, bs, outs):
        plain = lib.vertex_tensor(tj, dl, 1.2, bd)
        assert torch.equal(a, plain)
        assert normwise(a.cpu().numpy(), V.vertex_tensor(tj, dl, b)) <= TOL


# ------------------------------------------------------------------ contraction and adjoint

def test_contract_and_adjoint(lib, torch):
    two_j, dl = [4, 1, 2, 3, 1, 3, 2, 4, 4, 1], 2
    b, bd = boosters_for(torch, two_j, dl, 31)
    note("contract + adjoint")
    A = lib.vertex_tensor(two_j, dl, 1.2, bd)
    a = A.cpu().numpy()
    psis = workloads.boundary_vectors(31, a.shape)
    pd = [torch.from_numpy(p).cuda() for p in psis]
    F = complex(lib.contract_boundary(A, pd).cpu().item())
    Fref = C.contract_boundary(V.vertex_tensor(two_j, dl, b), psis)
    assert abs(F - Fref) <= TOL * max(1.0, abs(Fref))
    g = 0.3 - 0.7j
    gpsi, gb = lib.contract_boundary_adjoint(two_j, dl, bd, A, pd, g)
    ref_psi = C.grad_psi(a, psis)
    for q in range(5):
        assert normwise(gpsi[q].cpu().numpy(), g * ref_psi[q]) <= TOL
    ref_b = C.grad_boosters(two_j, dl, b, psis)
    assert normwise(gb.cpu().numpy(), g * ref_b) <= TOL


def test_autograd_against_finite_differences(lib, torch):
    from paper_2107_13952_amd.autograd import vertex_contract
    two_j, dl = [2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 1
    b, _ = boosters_for(torch, two_j, dl, 41)
    dims = [n for _, n in R.boundary_ranges(two_j)]
    psis = workloads.boundary_vectors(41, dims)
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    pts = [torch.from_numpy(p).cuda().requires_grad_(True) for p in psis]
    note("autograd")
    F = vertex_contract(two_j, dl, 1.2, bt, pts)
    loss = (F * (0.4 + 0.9j)).real
    loss.backward()
    h = 1e-6

    def L(bv, pv):
        A = V.vertex_tensor(two_j, dl, bv)
        return (C.contract_boundary(A, pv) * (0.4 + 0.9j)).real

    rng = np.random.default_rng(0)
    gb = bt.grad.cpu().numpy()
    for n in rng.choice(b.size, size=12, replace=False):
        up, dn = b.copy(), b.copy()
        up[n] += h
        dn[n] -= h
        fd = (L(up, psis) - L(dn, psis)) / (2 * h)
        assert abs(fd - gb[n]) <= 2e-8 * max(1.0, abs(fd))
    for q in range(5):
        gq = pts[q].grad.cpu().numpy()
        for n in range(dims[q]):
            for delta in (h, 1j * h):
                up = [p.copy() for p in psis]
                dn = [p.copy() for p in psis]
                up[q][n] += delta
                dn[q][n] -= delta
                fd = (L(b, up) - L(b, dn)) / (2 * h)
                got = gq[n].real if delta == h else gq[n].imag
                assert abs(fd - got) <= 2e-8 * max(1.0, abs(fd))


def _adjoint_full_size(lib, torch, two_j, dl, seed, psi_seed, golden, sample_blocks):
    """Adjoint at full size.  F is linear in each psi_a and in the boosters of each edge, so a
    central difference along a direction confined to one of them is exact up to rounding: the
    psi gradients are checked entry by entry that way, the booster gradient along one random
    direction per edge (forward passes on the GPU), and sampled booster blocks against the
    oracle's gradient (only the shells that use them are visited)."""
    b, bd = boosters_for(torch, two_j, dl, seed)
    dims = [n for _, n in R.boundary_ranges(two_j)]
    psis = workloads.boundary_vectors(psi_seed, dims)
    pd = [torch.from_numpy(p).cuda() for p in psis]
    A = lib.vertex_tensor(two_j, dl, 1.2, bd)
    F = complex(lib.contract_boundary(A, pd).cpu().item())
    g = load_golden(golden, required=False) if golden else None
    if g is not None and len(g["rows"]) == dims[0]:
        Fref = C.contract_boundary(g["A"], psis)
        note(f"  F {F:.6e}, oracle {Fref:.6e}")
        assert abs(F - Fref) <= TOL * abs(Fref)
    gpsi, gb = lib.contract_boundary_adjoint(two_j, dl, bd, A, pd, 1.0)
    gb = gb.cpu().numpy()
    scale = max(abs(F), 1e-300)
    for q in range(5):
        gq = gpsi[q].cpu().numpy()
        for n in range(dims[q]):
            for delta in (1.0, 1.0j):
                up = [p.clone() for p in pd]
                dn = [p.clone() for p in pd]
                up[q][n] += delta
                dn[q][n] -= delta
                fd = (complex(lib.contract_boundary(A, up).cpu().item())
                      - complex(lib.contract_boundary(A, dn).cpu().item())) / 2
                got = gq[n] * delta
                assert abs(fd - got) <= 1e-12 * max(scale, abs(fd)), (q, n, fd, got)
    shapes, offsets = R.booster_layout(two_j, dl)
    n3 = (dl + 1) ** 3
    rng = np.random.default_rng(7)
    for e in range(2, 6):
        lo, hi = offsets[(e - 2) * n3], offsets[(e - 1) * n3]
        d = np.zeros_like(b)
        d[lo:hi] = rng.standard_normal(hi - lo) * np.abs(b[lo:hi]).max()
        dd = torch.from_numpy(d).cuda()
        Fp = complex(lib.contract_boundary(lib.vertex_tensor(two_j, dl, 1.2, bd + dd), pd).cpu().item())
        Fm = complex(lib.contract_boundary(lib.vertex_tensor(two_j, dl, 1.2, bd - dd), pd).cpu().item())
        fd = (Fp - Fm) / 2
        got = complex(np.dot(gb, d))
        note(f"  edge {e}: directional derivative {got:.6e}, central difference {fd:.6e}")
        assert abs(fd - got) <= 1e-10 * max(abs(fd), abs(Fp), abs(Fm))
    ref = C.grad_boosters(two_j, dl, b, psis, only=sample_blocks)
    for (e, t), blk in ref.items():
        n = (e - 2) * n3 + t
        got = gb[offsets[n]:offsets[n + 1]].reshape(blk.shape)
        err = normwise(got, blk)
        note(f"  booster block (e{e}, {t}) vs oracle gradient {err:.3e}")
        assert err <= TOL


def test_adjoint_j4_full_size(lib, torch):
    cfg = workloads.CFG4
    note("adjoint j=4 dl=8")
    dl = cfg["dl"]
    mid = ((dl // 2) * (dl + 1) + dl // 2) * (dl + 1) + dl // 2
    _adjoint_full_size(lib, torch, cfg["two_j"], dl, cfg["booster_seed"], cfg["psi_seed"], "j4_dl8",
                       [(2, 0), (5, mid)])


def test_adjoint_large_spins(lib, torch):
    tj, dl = workloads.cfg5_batch()[0]
    note(f"adjoint large spins two_j={tj} dl={dl}")
    _adjoint_full_size(lib, torch, tj, dl, workloads.batch_booster_seed(workloads.CFG5_SEED, 0),
                       workloads.CFG5_SEED, None, [(3, 0)])


# ------------------------------------------------------------------ BF vertex (no boosters)

BF_CASES = [[2, 3, 2, 1, 3, 2, 3, 1, 1, 3], [2] * 10, [6] * 10, [0] * 10,
            [13, 10, 11, 12, 10, 14, 11, 13, 13, 10]]


@pytest.mark.parametrize("two_j", BF_CASES)
def test_bf_vertex_against_oracle(lib, torch, two_j):
    """The boosterless BF vertex against the oracle's, which is pinned by the brute-force
    spin network (tests/test_oracle_vertex.py)."""
    note(f"bf vertex {two_j}")
    a = lib.bf_vertex_tensor(two_j).cpu().numpy()
    ref = V.bf_vertex(two_j)
    assert a.shape == ref.shape
    err = normwise(a, ref)
    note(f"  normwise error {err:.3e}")
    assert err <= TOL


def test_bf_vertex_wide_intertwiners(lib, torch):
    """Intertwiner dimensions above 16 (all spins 10, dimension 21): sampled entries against the
    oracle's {15j} one by one, and the Delta l = 0 vertex tensor with identity boosters on a case
    both paths take."""
    from oracle.fifteenj import fifteenj
    two_j = [20] * 10
    note("bf vertex dims 21")
    a = lib.bf_vertex_tensor(two_j).cpu().numpy()
    bnd = R.boundary_ranges(two_j)
    assert a.shape == tuple(n for _, n in bnd)
    rng = np.random.default_rng(5)
    idx = [tuple(int(rng.integers(n)) for _, n in bnd) for _ in range(300)]
    ref = np.array([fifteenj(*[bnd[q][0] + 2 * i[q] for q in range(5)], two_j)
                    * np.prod([np.sqrt(bnd[q][0] + 2 * i[q] + 1.0) for q in range(5)]) for i in idx])
    got = np.array([a[i] for i in idx])
    assert np.abs(got - ref).max() <= TOL * np.abs(a).max()
    # identity boosters at dl = 0 reproduce the BF vertex through the EPRL path
    tj = [13, 10, 11, 12, 10, 14, 11, 13, 13, 10]
    shapes, offsets = R.booster_layout(tj, 0)
    parts = []
    for e in range(2, 6):
        rows, cols, klo = shapes[(e, 0)]
        parts.append((np.eye(rows) / (klo + 2 * np.arange(cols) + 1.0)[None, :]).ravel())
    eprl = lib.vertex_tensor(tj, 0, 1.0, torch.from_numpy(np.concatenate(parts)).cuda())
    assert normwise(eprl.cpu().numpy(), lib.bf_vertex_tensor(tj).cpu().numpy()) <= 1e-13
