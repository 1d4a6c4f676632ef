"""The allocation-free contraction entry point against the allocating one, through the C ABI:
two calls in a row, the second on a smaller vertex tensor, each compared with
eprl_contract_boundary on the same inputs (same kernels and partial-sum count: bitwise equal)."""
import ctypes

import numpy as np
import pytest

import workloads
from oracle import ranges as R
from oracle import vertex as V
from oracle import contract as C

pytestmark = pytest.mark.gpu


def _call(lib, name, A, psis, F):
    h = lib._ctx(A.device).bind()
    dims = (ctypes.c_int * 5)(*A.shape)
    ptrs = (ctypes.c_void_p * 5)(*[p.data_ptr() for p in psis])
    rc = getattr(lib._lib, name)(h, dims, ctypes.c_void_p(A.data_ptr()), ptrs,
                                 ctypes.c_void_p(F.data_ptr()))
    assert rc == 0, lib._lib.eprl_last_error(h).decode()


def test_noalloc_contraction_matches_allocating_call():
    import torch
    import paper_2107_13952_amd as lib
    cases = [([13, 10, 11, 12, 10, 14, 11, 13, 13, 10], 1, 61),   # dims 11^5
             ([2, 3, 2, 1, 3, 2, 3, 1, 1, 3], 1, 62)]             # dims 2 x 3 x 2 x 2 x 2
    for two_j, dl, seed in cases:
        print(f"no-alloc contraction {two_j} dl={dl}", flush=True)
        b = workloads.synthetic_boosters(seed, R.block_shapes(two_j, dl))
        A = lib.vertex_tensor(two_j, dl, 1.2, torch.from_numpy(b).cuda())
        psis = [torch.from_numpy(p).cuda() for p in workloads.boundary_vectors(seed, list(A.shape))]
        F0 = torch.zeros(2, dtype=torch.float64, device="cuda")
        F1 = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        _call(lib, "eprl_contract_boundary", A, psis, F0)
        _call(lib, "eprl_contract_boundary_noalloc", A, psis, F1)
        torch.cuda.synchronize()
        assert torch.equal(F0, F1), (F0, F1)
        if A.numel() < 1000:
            ref = C.contract_boundary(V.vertex_tensor(two_j, dl, b), [p.cpu().numpy() for p in psis])
            got = complex(F1[0].item(), F1[1].item())
            assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref))
