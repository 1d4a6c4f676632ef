"""Multi-vertex contractions on the GPU (through the C ABI) against the oracle: the complete
contraction of two vertex tensors, boundary vectors on the trailing intertwiners of a vertex,
and the Delta_3 amplitude assembled from three partially contracted BF vertices.

Bar: error relative to the sum of the absolute values of the terms <= 1e-13 (each result is one
sum of products, accumulated in FP64 in a fixed order), and bitwise repeatability."""
import sys

import numpy as np
import pytest

from oracle import network as N
from oracle import vertex as V

pytestmark = pytest.mark.gpu


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


def cvec(rng, n):
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    return v / np.linalg.norm(v)


SHAPES = [(7, 7, 7, 7, 7), (3, 5, 2, 7, 11), (1, 1, 1, 1, 1), (16, 16, 16, 16, 16)]


@pytest.mark.parametrize("shape", SHAPES)
def test_contract_vertices(lib, torch, shape):
    rng = np.random.default_rng(sum(shape))
    a, b = rng.normal(size=shape), rng.normal(size=shape)
    note(f"contract_vertices {shape}")
    ad, bd = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    f = lib.contract_vertices(ad, bd)
    ref = N.contract_vertices(a, b)
    bound = 1e-13 * float(np.abs(a * b).sum())
    assert abs(float(f) - ref) <= bound
    assert torch.equal(f, lib.contract_vertices(ad, bd))


@pytest.mark.parametrize("shape", SHAPES[:3] + [(16, 16, 16, 16, 16)])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_contract_trailing(lib, torch, shape, m):
    rng = np.random.default_rng(100 * m + sum(shape))
    a = rng.normal(size=shape)
    psis = [cvec(rng, n) for n in shape[5 - m:]]
    note(f"contract_trailing {shape} m={m}")
    ad = torch.from_numpy(a).cuda()
    pd = [torch.from_numpy(p).cuda() for p in psis]
    t = lib.contract_trailing(ad, pd)
    assert tuple(t.shape) == shape[:5 - m]
    ref = N.contract_trailing(a, psis)
    absterms = np.abs(a)
    for q, p in enumerate(psis):
        sh = [1] * 5
        sh[5 - m + q] = -1
        absterms = absterms * np.abs(p).reshape(sh)
    bound = 1e-13 * absterms.sum(axis=tuple(range(5 - m, 5)))
    assert np.all(np.abs(t.cpu().numpy() - ref) <= bound + 1e-300)
    assert torch.equal(t, lib.contract_trailing(ad, pd))


def test_contract_delta3_random(lib, torch):
    rng = np.random.default_rng(7)
    for n, two_klo, two_x in [(1, 0, 0), (5, 2, 4), (33, 0, 8), (64, 4, 2), (128, 0, 2)]:
        ts = [rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) for _ in range(3)]
        note(f"delta3 n={n} two_klo={two_klo} two_x={two_x}")
        f = complex(lib.contract_delta3(*[torch.from_numpy(t).cuda() for t in ts], two_klo, two_x))
        ref = N.delta3(*ts, two_klo, two_x)
        bound = 1e-13 * (two_x + 1) * float(np.einsum("ab,ca,bc->", *[np.abs(t) for t in ts]))
        assert abs(f - ref) <= bound
    eye = torch.eye(3, dtype=torch.complex128, device="cuda")
    big = torch.zeros((257, 257), dtype=torch.complex128, device="cuda")
    with pytest.raises(lib.EprlError) as exc:
        lib.contract_delta3(big, big, big, 0, 0)
    assert exc.value.code == -1
    for two_klo, two_x in [(1, 0), (0, 3)]:
        with pytest.raises(lib.EprlError) as exc:
            lib.contract_delta3(eye, eye, eye, two_klo, two_x)
        assert exc.value.code == -1


@pytest.mark.parametrize("two_J,two_x", [(2, 2), (4, 4), (6, 2)])
def test_delta3_of_bf_vertices(lib, torch, two_J, two_x):
    """The Delta_3 pattern of Sec. 4.2: three equal BF vertices with boundary spins (x, J, ..., J),
    each contracted with three seeded boundary vectors on its last three intertwiners, leaving the
    two bulk intertwiners; then the sum over the triangle of bulk intertwiners."""
    two_j = [two_x] + [two_J] * 9
    dims, ilo, _ = lib.layout(two_j, 0)
    assert dims[0] == dims[1] and ilo[0] == ilo[1]
    rng = np.random.default_rng(two_J * 10 + two_x)
    a_ref = V.bf_vertex(two_j)
    ad = lib.bf_vertex_tensor(two_j)
    assert np.abs(ad.cpu().numpy() - a_ref).max() <= 1e-13 * np.abs(a_ref).max()
    mats, refs = [], []
    for v in range(3):
        psis = [cvec(rng, n) for n in dims[2:]]
        mats.append(lib.contract_trailing(ad, [torch.from_numpy(p).cuda() for p in psis]))
        refs.append(N.contract_trailing(a_ref, psis))
    note(f"delta3 of BF vertices two_j={two_j}")
    f = complex(lib.contract_delta3(mats[0], mats[1], mats[2], ilo[0], two_x))
    ref = N.delta3(refs[0], refs[1], refs[2], ilo[0], two_x)
    assert abs(f - ref) <= 1e-10 * max(abs(ref), 1e-300)
