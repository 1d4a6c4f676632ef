"""Python binding of the MI355X vertex-tensor library (``libeprl.so``, C ABI in include/eprl.h).

Argument marshalling only: every step of the computation runs in the HIP kernels of the
library.  PyTorch provides device memory and the current stream; all device tensors are
float64 (complex vectors complex128) on a ROCm device.  If the library has not been built
the import of this package fails: there is no CPU fallback.

Functions mirror the C entry points:

* ``layout(two_j, dl)`` and ``count_terms(two_j, dl)``  (host only)
* ``vertex_tensor(two_j, dl, gamma, boosters)``          eq. (vertex-ampl)
* ``bf_vertex_tensor(two_j)``                              the BF (15j) vertex, no boosters
* ``vertex_tensor_range(...)``                            partial shell sums (resume unit)
* ``vertex_tensor_cores(...)``                            partial sums over cores (l24, l25, l34, l35)
* ``vertex_tensor_batched(configs, gamma, boosters)``     many configurations, one launch
* ``vertex_tensor_scan(two_j, dl_max, gamma, boosters)``  A(dl) for dl = 0..dl_max, one batch
* ``contract_boundary(A, psis)``                          contraction with five vectors
* ``contract_boundary_adjoint(...)``                      its derivatives
* ``contract_vertices(A, B)``, ``contract_trailing(A, psis)``, ``contract_delta3(...)``
                                                          multi-vertex contractions
* ``boosters(two_j, dl, gamma)``                          eq. (booster) by quadrature on the GPU
* ``VertexContract``                                      torch.autograd.Function of F(psi, B)
"""
import ctypes
import functools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeprl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with paper_2107_13952_amd.build.build() "
        "(hipcc --offload-arch=gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

_i32p = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.c_void_p

_SIGS = {
    "eprl_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    "eprl_destroy": (None, [ctypes.c_void_p]),
    "eprl_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "eprl_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "eprl_set_algorithm": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "eprl_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "eprl_autotune": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, _dp, _dp, _i32p]),
    "eprl_layout": (ctypes.c_int, [_i32p, ctypes.c_int, _i32p, _i32p, _i64p]),
    "eprl_count_terms": (ctypes.c_int, [_i32p, ctypes.c_int, _i64p, ctypes.POINTER(ctypes.c_double)]),
    "eprl_count_work": (ctypes.c_int, [_i32p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "eprl_vertex_tensor": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, ctypes.c_double, _dp, _dp]),
    "eprl_bf_vertex_tensor": (ctypes.c_int, [ctypes.c_void_p, _i32p, _dp]),
    "eprl_vertex_tensor_range": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, ctypes.c_double, _dp,
                                                ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _dp]),
    "eprl_vertex_tensor_cores": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, ctypes.c_double, _dp,
                                                ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _dp]),
    "eprl_vertex_tensor_scan": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, ctypes.c_double, _dp, _dp]),
    "eprl_vertex_tensor_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, _i32p, ctypes.c_double,
                                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "eprl_contract_boundary": (ctypes.c_int, [ctypes.c_void_p, _i32p, _dp, ctypes.POINTER(ctypes.c_void_p), _dp]),
    "eprl_boosters": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     _dp, ctypes.POINTER(ctypes.c_double)]),
    "eprl_threejm_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, _dp]),
    "eprl_contract_vertices": (ctypes.c_int, [ctypes.c_void_p, _i32p, _dp, _dp, _dp]),
    "eprl_contract_trailing": (ctypes.c_int, [ctypes.c_void_p, _i32p, _dp, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_void_p), _dp]),
    "eprl_contract_delta3": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            _dp, _dp, _dp, _dp]),
    "eprl_contract_boundary_noalloc": (ctypes.c_int, [ctypes.c_void_p, _i32p, _dp, ctypes.POINTER(ctypes.c_void_p), _dp]),
    "eprl_contract_boundary_adjoint": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, _dp, _dp,
                                                      ctypes.POINTER(ctypes.c_void_p),
                                                      ctypes.POINTER(ctypes.c_double),
                                                      ctypes.POINTER(ctypes.c_void_p), _dp]),
    "eprl_sixj_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _i32p, _dp]),
    "eprl_shell_fifteenj": (ctypes.c_int, [ctypes.c_void_p, _i32p, ctypes.c_int, ctypes.c_int64, _i32p, _dp,
                                           ctypes.c_int64]),
    "eprl_timing_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "eprl_timing_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _i64p]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)
ERRORS = {-1: "EPRL_EINVAL", -2: "EPRL_ENOMEM", -3: "EPRL_EHIP", -4: "EPRL_ERANGE"}


class EprlError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


def _ints(vals, n=None):
    arr = (ctypes.c_int * len(vals))(*[int(v) for v in vals])
    if n is not None and len(vals) != n:
        raise ValueError(f"expected {n} values, got {len(vals)}")
    return arr


# ---------------------------------------------------------------- host-only calls

_PLAN_ERRORS = {-4: "a 6j argument of the configuration exceeds two_j = 200 (j + dl, the "
                    "intertwiners and x must stay within j = 100)"}

def layout(two_j, dl):
    """(dims_i[5], two_ilo[5], booster_offsets int64 array of 4 (dl+1)^3 + 1)."""
    dims, ilo, offs = _layout(tuple(int(v) for v in two_j), int(dl))
    return list(dims), list(ilo), offs.copy()


@functools.lru_cache(maxsize=64)
def _layout(two_j, dl):
    """layout() of a configuration, computed once per process (host-only planning)."""
    dims = (ctypes.c_int * 5)()
    ilo = (ctypes.c_int * 5)()
    offs = np.zeros(4 * (int(dl) + 1) ** 3 + 1, dtype=np.int64)
    rc = _lib.eprl_layout(_ints(two_j, 10), int(dl), dims, ilo,
                          offs.ctypes.data_as(_i64p))
    if rc:
        raise EprlError(rc, _PLAN_ERRORS.get(rc, "inadmissible spins or shell count"))
    offs.setflags(write=False)
    return tuple(dims), tuple(ilo), offs


def count_terms(two_j, dl):
    """(live shells, {15j} x booster terms)."""
    live = ctypes.c_int64()
    terms = ctypes.c_double()
    rc = _lib.eprl_count_terms(_ints(two_j, 10), int(dl), ctypes.byref(live), ctypes.byref(terms))
    if rc:
        raise EprlError(rc, "inadmissible spins or shell count")
    return live.value, terms.value


def count_work(two_j, dl):
    """dict: terms, shell_flops, ring_useful_flops, ring_mfma_flops (exact host counts) and
    ring_class (tile class of the factorised kernel, -1 when it does not apply)."""
    out = (ctypes.c_double * 5)()
    rc = _lib.eprl_count_work(_ints(two_j, 10), int(dl), out)
    if rc:
        raise EprlError(rc, "inadmissible spins or shell count")
    return {"terms": out[0], "shell_flops": out[1], "ring_useful_flops": out[2],
            "ring_mfma_flops": out[3], "ring_class": int(out[4])}


# ---------------------------------------------------------------- device calls

def _torch():
    import torch
    return torch


class _Context:
    """One library context per device, re-bound to torch's current stream at every call."""

    def __init__(self, device):
        self.device = device
        self.handle = ctypes.c_void_p()
        rc = _lib.eprl_create(ctypes.byref(self.handle), int(device), None)
        if rc:
            raise EprlError(rc, "cannot create a context on device %d" % device)

    def bind(self):
        torch = _torch()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.eprl_set_stream(self.handle, ctypes.c_void_p(stream))
        return self.handle

    def check(self, rc):
        if rc:
            raise EprlError(rc, _lib.eprl_last_error(self.handle).decode())

    def __del__(self):
        try:
            if self.handle:
                _lib.eprl_destroy(self.handle)
        except Exception:
            pass


_CONTEXTS = {}


def _ctx(device):
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("no ROCm GPU visible: the vertex-tensor library runs only on the GPU")
    dev = torch.device(device).index if torch.device(device).index is not None else torch.cuda.current_device()
    if dev not in _CONTEXTS:
        _CONTEXTS[dev] = _Context(dev)
    return _CONTEXTS[dev]


def _check_dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def vertex_tensor(two_j, dl, gamma, boosters, out=None):
    """A[i1, i2, i3, i4, i5] (float64, on the boosters' device), eq. (vertex-ampl)."""
    return vertex_tensor_range(two_j, dl, gamma, boosters, 0, (int(dl) + 1) ** 6, False, out)


def bf_vertex_tensor(two_j, device="cuda", out=None):
    """SU(2) BF vertex prod_e sqrt(2 i_e + 1) {15j}(j; i1..i5) (float64 [i1..i5], no boosters)."""
    torch = _torch()
    dims = list(_layout(tuple(int(v) for v in two_j), 0)[0])
    if out is None:
        out = torch.empty(dims, dtype=torch.float64, device=device)
    ap = _check_dev(out, torch.float64, "out")
    if list(out.shape) != dims:
        raise ValueError(f"output shape {list(out.shape)} != {dims}")
    ctx = _ctx(out.device)
    ctx.check(_lib.eprl_bf_vertex_tensor(ctx.bind(), _ints(two_j, 10), ap))
    return out


def _partial_call(fn, two_j, dl, gamma, boosters, begin, end, accumulate, out):
    torch = _torch()
    dims, _, offs = _layout(tuple(int(v) for v in two_j), int(dl))
    dims = list(dims)
    if boosters.numel() != int(offs[-1]):
        raise ValueError(f"booster buffer holds {boosters.numel()} values, layout needs {int(offs[-1])}")
    bp = _check_dev(boosters, torch.float64, "boosters")
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an output tensor")
        out = torch.empty(dims, dtype=torch.float64, device=boosters.device)
    ap = _check_dev(out, torch.float64, "out")
    if list(out.shape) != dims:
        raise ValueError(f"output shape {list(out.shape)} != {dims}")
    ctx = _ctx(boosters.device)
    ctx.check(fn(ctx.bind(), _ints(two_j, 10), int(dl), float(gamma), bp, int(begin), int(end),
                 1 if accumulate else 0, ap))
    return out


def vertex_tensor_range(two_j, dl, gamma, boosters, shell_begin, shell_end, accumulate=False, out=None):
    """Partial sum of A over shells [shell_begin, shell_end) of the (dl+1)^6 enumeration."""
    return _partial_call(_lib.eprl_vertex_tensor_range, two_j, dl, gamma, boosters, shell_begin,
                         shell_end, accumulate, out)


def vertex_tensor_cores(two_j, dl, gamma, boosters, core_begin, core_end, accumulate=False, out=None):
    """Partial sum of A over the cores [core_begin, core_end) of the factorised order, core
    ((o24 (dl+1) + o25) (dl+1) + o34) (dl+1) + o35, every l23 and l45 included."""
    return _partial_call(_lib.eprl_vertex_tensor_cores, two_j, dl, gamma, boosters, core_begin,
                         core_end, accumulate, out)


def vertex_tensor_scan(two_j, dl_max, gamma, boosters, out=None):
    """A(dl) for dl = 0..dl_max as one float64 tensor [dl_max + 1, i1, .., i5]; boosters packed
    for dl_max (layout(two_j, dl_max))."""
    torch = _torch()
    dims, _, offs = _layout(tuple(int(v) for v in two_j), int(dl_max))
    shape = [int(dl_max) + 1] + list(dims)
    if boosters.numel() != int(offs[-1]):
        raise ValueError(f"booster buffer holds {boosters.numel()} values, layout needs {int(offs[-1])}")
    bp = _check_dev(boosters, torch.float64, "boosters")
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=boosters.device)
    ap = _check_dev(out, torch.float64, "out")
    if list(out.shape) != shape:
        raise ValueError(f"output shape {list(out.shape)} != {shape}")
    ctx = _ctx(boosters.device)
    ctx.check(_lib.eprl_vertex_tensor_scan(ctx.bind(), _ints(two_j, 10), int(dl_max), float(gamma), bp, ap))
    return out


def vertex_tensor_batched(configs, gamma, boosters, outs=None):
    """configs: list of (two_j[10], dl); boosters: list of device tensors.  Returns list of A."""
    torch = _torch()
    n = len(configs)
    if len(boosters) != n:
        raise ValueError("one booster buffer per configuration is required")
    if outs is None:
        outs = [torch.empty(layout(tj, dl)[0], dtype=torch.float64, device=b.device)
                for (tj, dl), b in zip(configs, boosters)]
    flat_j = [v for tj, _ in configs for v in tj]
    dls = [dl for _, dl in configs]
    bptr = (ctypes.c_void_p * n)(*[_check_dev(b, torch.float64, "boosters").value for b in boosters])
    aptr = (ctypes.c_void_p * n)(*[_check_dev(a, torch.float64, "out").value for a in outs])
    for (tj, dl), b in zip(configs, boosters):
        if b.numel() != int(layout(tj, dl)[2][-1]):
            raise ValueError("booster buffer size does not match its configuration")
    ctx = _ctx(boosters[0].device if n else "cuda")
    ctx.check(_lib.eprl_vertex_tensor_batched(ctx.bind(), n, _ints(flat_j), _ints(dls), float(gamma), bptr, aptr))
    return outs


def _psi_ptrs(psis, dims):
    torch = _torch()
    if len(psis) != 5:
        raise ValueError("five boundary vectors are required")
    ptrs = []
    for a, (p, n) in enumerate(zip(psis, dims)):
        if p.shape != (n,):
            raise ValueError(f"psi{a + 1} must have length {n}")
        ptrs.append(_check_dev(p, torch.complex128, f"psi{a + 1}").value)
    return (ctypes.c_void_p * 5)(*ptrs)


def contract_boundary(A, psis):
    """F = sum A psi1 psi2 psi3 psi4 psi5 as a complex128 0-d device tensor."""
    torch = _torch()
    ap = _check_dev(A, torch.float64, "A")
    dims = list(A.shape)
    if len(dims) != 5:
        raise ValueError("A must have five indices")
    F = torch.empty(2, dtype=torch.float64, device=A.device)
    ctx = _ctx(A.device)
    ctx.check(_lib.eprl_contract_boundary(ctx.bind(), _ints(dims, 5), ap, _psi_ptrs(psis, dims),
                                          ctypes.c_void_p(F.data_ptr())))
    return torch.view_as_complex(F)


def contract_vertices(A, B):
    """sum_i A(i) B(i) of two float64 vertex tensors of the same shape (0-d device tensor)."""
    torch = _torch()
    ap = _check_dev(A, torch.float64, "A")
    bp = _check_dev(B, torch.float64, "B")
    dims = list(A.shape)
    if len(dims) != 5 or list(B.shape) != dims:
        raise ValueError("A and B must be five-index tensors of the same shape")
    F = torch.empty((), dtype=torch.float64, device=A.device)
    ctx = _ctx(A.device)
    ctx.check(_lib.eprl_contract_vertices(ctx.bind(), _ints(dims, 5), ap, bp, ctypes.c_void_p(F.data_ptr())))
    return F


def contract_trailing(A, psis):
    """A contracted with len(psis) = m vectors on its last m intertwiners (psis[0] pairs with
    i_{6-m}, psis[-1] with i5): complex128 tensor over the first 5 - m intertwiners."""
    torch = _torch()
    ap = _check_dev(A, torch.float64, "A")
    dims = list(A.shape)
    m = len(psis)
    if len(dims) != 5 or not 1 <= m <= 5:
        raise ValueError("A must have five indices and between one and five vectors are given")
    ptrs = []
    for q, p in enumerate(psis):
        n = dims[5 - m + q]
        if p.shape != (n,):
            raise ValueError(f"vector {q} must have length {n}")
        ptrs.append(_check_dev(p, torch.complex128, f"psi[{q}]").value)
    T = torch.empty(dims[:5 - m] + [2], dtype=torch.float64, device=A.device)
    ctx = _ctx(A.device)
    ctx.check(_lib.eprl_contract_trailing(ctx.bind(), _ints(dims, 5), ap, m, (ctypes.c_void_p * m)(*ptrs),
                                          ctypes.c_void_p(T.data_ptr())))
    return torch.view_as_complex(T)


def contract_delta3(TA, TB, TC, two_klo, two_x):
    """Delta_3 amplitude (-1)^x (2x+1) sum (-1)^(k1+k2+k3) TA[k1,k2] TB[k3,k1] TC[k2,k3] from three
    complex128 n x n device matrices (0-d complex device tensor)."""
    torch = _torch()
    n = TA.shape[0]
    ptrs = []
    for name, t in (("TA", TA), ("TB", TB), ("TC", TC)):
        if tuple(t.shape) != (n, n):
            raise ValueError(f"{name} must be {n} x {n}")
        ptrs.append(_check_dev(t, torch.complex128, name))
    F = torch.empty(2, dtype=torch.float64, device=TA.device)
    ctx = _ctx(TA.device)
    ctx.check(_lib.eprl_contract_delta3(ctx.bind(), int(n), int(two_klo), int(two_x), *ptrs,
                                        ctypes.c_void_p(F.data_ptr())))
    return torch.view_as_complex(F)


def contract_boundary_noalloc(A, psis, F):
    """contract_boundary into a caller-given float64 device tensor F of 2 entries (re, im); the
    library allocates nothing (its partial sums use a fixed device array)."""
    torch = _torch()
    ap = _check_dev(A, torch.float64, "A")
    fp = _check_dev(F, torch.float64, "F")
    if F.numel() != 2:
        raise ValueError("F must hold two float64 values (re, im)")
    dims = list(A.shape)
    if len(dims) != 5:
        raise ValueError("A must have five indices")
    ctx = _ctx(A.device)
    ctx.check(_lib.eprl_contract_boundary_noalloc(ctx.bind(), _ints(dims, 5), ap, _psi_ptrs(psis, dims), fp))
    return F


def contract_boundary_adjoint(two_j, dl, boosters, A, psis, grad_F=1.0, want_psi=True, want_boosters=True):
    """(g dF/dpsi_a for a = 1..5, g dF/dB) as complex128 device tensors (holomorphic derivatives)."""
    torch = _torch()
    dims, _, offs = layout(two_j, dl)
    if want_boosters and boosters.numel() != int(offs[-1]):
        raise ValueError(f"booster buffer holds {boosters.numel()} values, layout needs {int(offs[-1])}")
    if want_psi and list(A.shape) != dims:
        raise ValueError(f"vertex tensor shape {list(A.shape)} != {dims}")
    dev = psis[0].device
    g = complex(grad_F)
    gbuf = (ctypes.c_double * 2)(g.real, g.imag)
    gpsi = [torch.empty(n, dtype=torch.complex128, device=dev) for n in dims] if want_psi else None
    gb = torch.empty(int(offs[-1]), dtype=torch.complex128, device=dev) if want_boosters else None
    gpsi_ptrs = (ctypes.c_void_p * 5)(*[t.data_ptr() for t in gpsi]) if want_psi else None
    bp = _check_dev(boosters, torch.float64, "boosters") if want_boosters else None
    ap = _check_dev(A, torch.float64, "A") if want_psi else None
    ctx = _ctx(dev)
    ctx.check(_lib.eprl_contract_boundary_adjoint(
        ctx.bind(), _ints(two_j, 10), int(dl), bp, ap, _psi_ptrs(psis, dims), gbuf,
        gpsi_ptrs, ctypes.c_void_p(gb.data_ptr()) if want_boosters else None))
    return gpsi, gb


def boosters(two_j, dl, gamma, tol=1e-13, device="cuda", out=None):
    """Packed boosters of eq. (booster) (layout(two_j, dl)) computed on the GPU.  Returns the
    float64 device tensor and a dict with the largest quadrature error estimate, the largest
    imaginary part and the number n of subintervals used."""
    torch = _torch()
    _, _, offs = _layout(tuple(int(v) for v in two_j), int(dl))
    if out is None:
        out = torch.empty(int(offs[-1]), dtype=torch.float64, device=device)
    bp = _check_dev(out, torch.float64, "out")
    if out.numel() != int(offs[-1]):
        raise ValueError(f"output holds {out.numel()} values, layout needs {int(offs[-1])}")
    info = (ctypes.c_double * 3)()
    ctx = _ctx(out.device)
    ctx.check(_lib.eprl_boosters(ctx.bind(), _ints(two_j, 10), int(dl), float(gamma), float(tol), bp, info))
    return out, {"error": info[0], "imag": info[1], "n": int(info[2])}


def threejm_batch(args, device="cuda"):
    """Evaluate 3jm symbols on the GPU; args is an (n, 6) integer array (two_j1..3, two_m1..3)."""
    torch = _torch()
    a = np.ascontiguousarray(np.asarray(args, dtype=np.int32).reshape(-1, 6))
    out = torch.empty(a.shape[0], dtype=torch.float64, device=device)
    ctx = _ctx(out.device)
    ctx.check(_lib.eprl_threejm_batch(ctx.bind(), a.shape[0], a.ctypes.data_as(_i32p),
                                      ctypes.c_void_p(out.data_ptr())))
    return out


def sixj_batch(args, device="cuda"):
    """Evaluate 6j symbols on the GPU; args is an (n, 6) integer array of two_j values."""
    torch = _torch()
    a = np.ascontiguousarray(np.asarray(args, dtype=np.int32).reshape(-1, 6))
    out = torch.empty(a.shape[0], dtype=torch.float64, device=device)
    ctx = _ctx(out.device)
    ctx.check(_lib.eprl_sixj_batch(ctx.bind(), a.shape[0], a.ctypes.data_as(_i32p),
                                   ctypes.c_void_p(out.data_ptr())))
    return out


def shell_fifteenj(two_j, dl, shell, device="cuda"):
    """The {15j} tensor W(i1, k2, k3, k4, k5) of one shell (diagnostic)."""
    torch = _torch()
    dims, _, _ = layout(two_j, dl)
    cap = dims[0] * 16 ** 4
    W = torch.zeros(cap, dtype=torch.float64, device=device)
    kd = (ctypes.c_int * 4)()
    ctx = _ctx(W.device)
    ctx.check(_lib.eprl_shell_fifteenj(ctx.bind(), _ints(two_j, 10), int(dl), int(shell), kd,
                                       ctypes.c_void_p(W.data_ptr()), cap))
    shape = [dims[0]] + list(kd)
    n = int(np.prod(shape))
    return W[:n].reshape(shape)


KERNELS = {"sixj_tables": 0, "assemble": 1, "reduce": 2, "adjoint_shells": 3, "ring": 4, "bf_vertex": 5,
           "ring_batch": 6}
ALGORITHMS = {"auto": 0, "shell": 1, "ring": 2, "ring_valu": 3}


def set_algorithm(name, device="cuda"):
    """Select how vertex tensors are evaluated: "auto" (default), "shell", "ring" or "ring_valu"."""
    ctx = _ctx(device)
    ctx.check(_lib.eprl_set_algorithm(ctx.handle, ALGORITHMS[name]))


def set_tuning(tile_class, target_workgroups=0, staging_level=-1, device="cuda"):
    """Work split of the factorised order for one tile class (0 / -1 restore the defaults)."""
    ctx = _ctx(device)
    ctx.check(_lib.eprl_set_tuning(ctx.handle, int(tile_class), int(target_workgroups),
                                   int(staging_level)))


def autotune(two_j, dl, boosters, out=None):
    """Time the factorised order on this configuration over workgroup targets and staging
    levels and keep the fastest for its tile class; returns the chosen setting."""
    torch = _torch()
    dims, _, _ = layout(two_j, dl)
    if out is None:
        out = torch.empty(dims, dtype=torch.float64, device=boosters.device)
    res = (ctypes.c_int * 3)()
    ctx = _ctx(boosters.device)
    ctx.check(_lib.eprl_autotune(ctx.bind(), _ints(two_j, 10), int(dl),
                                 _check_dev(boosters, torch.float64, "boosters"),
                                 _check_dev(out, torch.float64, "A"), res))
    return {"tile_class": res[0], "target_workgroups": res[1], "staging_level": res[2]}


def timing_enable(enable=True, device="cuda"):
    """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
    ctx = _ctx(device)
    ctx.check(_lib.eprl_timing_enable(ctx.bind(), 1 if enable else 0))


def timing_read(kernel, device="cuda"):
    """(total milliseconds, launches) recorded for ``kernel`` (a name of ``KERNELS``)."""
    ctx = _ctx(device)
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    ctx.check(_lib.eprl_timing_read(ctx.bind(), KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


from .autograd import VertexContract  # noqa: E402,F401
