"""Benchmark of the EPRL vertex-tensor hot path on one MI355X.

One step = one full vertex tensor of the equilateral j = 3 (two_j = 6), dl = 8 workload
(7^5 FP64 output, 531441 shells of which 498955 live): 6j tables, the shell sum of
{15j} x booster terms, reduction and normalisation, with the library's default evaluation
order (the factorised shell sum).  The per-shell order of the paper's framed algorithm is timed
beside it.  Inputs (seeded synthetic boosters of the right ragged shape) are resident in HBM
before the timed region.

Prints one JSON line:
  value        {15j} x booster terms per second (terms = sum over live shells of
               dim(i1) prod_e dim(k_e), independent of the algorithm)
  roofline     the factorised kernel's useful FP64 rate (exact count of the flops its active
               index ranges need) against the FP64 matrix peak, with its average duration
               measured by HIP events on the library's stream
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
  batched      64 seeded irregular configurations (dl 3..10): batched call vs per-config calls
  differentiation  j=4, dl=8 forward, contraction and adjoint, adjoint vs central differences
  large_batch  16 seeded large-spin configurations (dl 6): batched vs per-config calls
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector and matrix) peak
METRIC = "{15j}×booster terms/s (FP64) & FP64-MFMA util; batched vs plain, 1 GPU @1e-10"


def cpu_baseline(two_j, dl, boosters_np, nshell_sample):
    """The oracle on a contiguous block of shells, single thread."""
    from threadpoolctl import threadpool_limits
    from oracle import ranges as R
    from oracle import vertex as V
    shells = R.all_shells(dl)
    mid = len(shells) // 2
    block = shells[mid:mid + nshell_sample]
    n1 = R.boundary_ranges(two_j)[0][1]
    terms = 0.0
    for s in block:
        two_l = R.shell_spins(two_j, s)
        kd = [R.virtual_range(two_l, e)[1] for e in range(2, 6)]
        terms += n1 * float(np.prod(kd))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        V.vertex_tensor(two_j, dl, boosters_np, shells=block)
        dt = time.perf_counter() - t0
    return {"value": terms / dt, "unit": "terms/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(block)} consecutive shells (from index {mid}) of the same workload, "
                      f"{terms:.3g} terms in {dt:.1f} s, one thread"}


def quadrature_boosters(two_j, dl, size):
    """The FP64 quadrature boosters of eq. (booster) at gamma = 1.2 stored beside the oracle's
    j = 3, dl = 8 vertex rows (written offline by tests/golden/make_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", "vertex_j3_dl8_phys.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    if list(g["two_j"]) != list(two_j) or int(g["dl"]) != dl or g["boosters"].size != size:
        return None
    return np.ascontiguousarray(g["boosters"], dtype=np.float64)


def measured_traffic(split=None):
    """HBM bytes per ring_kernel launch from the committed counter summary, when it was taken on
    the current kernel source (same sha256 prefix) with the work split timed here (default:
    8192 workgroups, all booster blocks staged); otherwise None."""
    target, stg = (8192, 2) if split is None else (split["target_workgroups"], split["staging_level"])
    path = os.path.join(ROOT, "profiles", "ring_kernel_j3_dl8_counters.md")
    src = os.path.join(ROOT, "paper_2107_13952_amd", "csrc", "ring.hip")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m = re.search(r"kernel source sha256 ([0-9a-f]{16})", text)
    t = re.search(r"traffic bytes per launch, split %d %d: ([0-9.eE+]+)" % (target, stg), text)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


def counter_workload(lib, torch, two_j, dl, b, split):
    """The dominant kernel three times (with the given work split) and a plain 256 MiB device copy
    three times (the copy calibrates what FETCH_SIZE and WRITE_SIZE read for a known number of
    bytes)."""
    cls = lib.count_work(two_j, dl)["ring_class"]
    lib.set_tuning(cls, split[0], split[1])
    for _ in range(3):
        lib.vertex_tensor(two_j, dl, 1.2, b)
    torch.cuda.synchronize()
    x = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("counter workload done", flush=True)


def timed(torch, fn, reps):
    """Average wall time of fn() over reps calls after one untimed call, synchronised."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def block_shapes(lib, two_j, dl):
    """(rows, cols) of every packed booster block, from the library's layout."""
    dims, _, offs = lib.layout(two_j, dl)
    n3 = (dl + 1) ** 3
    return [(dims[e + 1], int((offs[e * n3 + t + 1] - offs[e * n3 + t]) // dims[e + 1]))
            for e in range(4) for t in range(n3)]


def differentiation(lib, torch, dev):
    """j=4, dl=8 vertex contracted with five seeded boundary vectors: forward, contraction and
    adjoint times, and the adjoint's booster gradient against central differences along one random
    direction per edge (F is linear in each edge's boosters, so the difference is exact up to
    rounding)."""
    cfg = workloads.CFG4
    two_j, dl = cfg["two_j"], cfg["dl"]
    b_np = workloads.synthetic_boosters(cfg["booster_seed"], block_shapes(lib, two_j, dl))
    b = torch.from_numpy(b_np).to(dev)
    dims, _, offsets = lib.layout(two_j, dl)
    psis = [torch.from_numpy(p).to(dev) for p in workloads.boundary_vectors(cfg["psi_seed"], dims)]
    A = lib.vertex_tensor(two_j, dl, 1.2, b)
    t_fwd = timed(torch, lambda: lib.vertex_tensor(two_j, dl, 1.2, b, out=A), 3)
    t_con = timed(torch, lambda: lib.contract_boundary(A, psis), 10)
    t_adj = timed(torch, lambda: lib.contract_boundary_adjoint(two_j, dl, b, A, psis, 1.0), 2)
    _, gb = lib.contract_boundary_adjoint(two_j, dl, b, A, psis, 1.0)
    gb = gb.cpu().numpy()
    n3 = (dl + 1) ** 3
    rng = np.random.default_rng(7)
    worst = 0.0
    for e in range(4):
        lo, hi = offsets[e * n3], offsets[(e + 1) * n3]
        d = np.zeros_like(b_np)
        d[lo:hi] = rng.standard_normal(hi - lo) * np.abs(b_np[lo:hi]).max()
        dd = torch.from_numpy(d).to(dev)
        fp = complex(lib.contract_boundary(lib.vertex_tensor(two_j, dl, 1.2, b + dd), psis).cpu().item())
        fm = complex(lib.contract_boundary(lib.vertex_tensor(two_j, dl, 1.2, b - dd), psis).cpu().item())
        fd = (fp - fm) / 2
        worst = max(worst, abs(fd - complex(np.dot(gb, d))) / max(abs(fd), abs(fp), abs(fm)))
    terms = lib.count_terms(two_j, dl)[1]
    return {"workload": "equilateral j=4 (two_j=8), dl=8, five seeded unit complex boundary vectors",
            "forward_ms": t_fwd * 1e3, "forward_terms_per_s": terms / t_fwd,
            "contract_us": t_con * 1e6, "adjoint_ms": t_adj * 1e3,
            "adjoint_vs_central_difference_max_rel_err": worst}


def large_batch(lib, torch, dev):
    """16 seeded configurations with spins 5..7 and dl = 6: batched graph vs per-configuration calls."""
    configs = workloads.cfg5_batch()
    bl = [torch.from_numpy(workloads.synthetic_boosters(
        workloads.batch_booster_seed(workloads.CFG5_SEED, c), block_shapes(lib, tj, d))).to(dev)
        for c, (tj, d) in enumerate(configs)]
    terms = sum(lib.count_terms(tj, d)[1] for tj, d in configs)
    outs = lib.vertex_tensor_batched(configs, 1.2, bl)
    t_b = timed(torch, lambda: lib.vertex_tensor_batched(configs, 1.2, bl, outs), 1)
    t_p = timed(torch, lambda: [lib.vertex_tensor(tj, d, 1.2, bb, out=a)
                                for (tj, d), bb, a in zip(configs, bl, outs)], 1)
    # Boundary contraction and its adjoint (psi and booster gradients) of every configuration,
    # with seeded unit complex boundary vectors.
    psis = [[torch.from_numpy(p).to(dev) for p in workloads.boundary_vectors(
        workloads.CFG5_SEED * 10 + c, list(a.shape))] for c, a in enumerate(outs)]

    def adjoint_all():
        for (tj, d), bb, a, ps in zip(configs, bl, outs, psis):
            lib.contract_boundary(a, ps)
            lib.contract_boundary_adjoint(tj, d, bb, a, ps, 1.0)

    t_a = timed(torch, adjoint_all, 1)
    return {"workload": "16 seeded configurations, j in 5..7, dl = 6, intertwiner dims 11..14",
            "terms": terms, "batched_terms_per_s": terms / t_b, "plain_terms_per_s": terms / t_p,
            "contraction_and_adjoint_s": t_a}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(lib, torch, two_j, dl, b, out, steps, warmup, kernel):
    """Warm up, then time `steps` vertex tensors between two events on the current stream; then
    the same steps again with the library's per-launch events on, for the kernel breakdown
    (kept out of the first pass: creating and recording events per launch costs host time)."""
    for _ in range(warmup):
        lib.vertex_tensor(two_j, dl, 1.2, b, out=out)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    t0 = time.perf_counter()
    for _ in range(steps):
        lib.vertex_tensor(two_j, dl, 1.2, b, out=out)
    host_ms = (time.perf_counter() - t0) * 1e3 / steps
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    progress(f"host time per call (enqueue) {host_ms:.3f} ms")
    lib.timing_enable(True)
    for _ in range(steps):
        lib.vertex_tensor(two_j, dl, 1.2, b, out=out)
    torch.cuda.synchronize()
    kms, kn = lib.timing_read(kernel)
    tab_ms, tab_n = lib.timing_read("sixj_tables")
    red_ms, red_n = lib.timing_read("reduce")
    lib.timing_enable(False)
    return ms, kms / max(kn, 1), {"sixj_tables": tab_ms / max(tab_n, 1), kernel: kms / max(kn, 1),
                                 "reduce": red_ms / max(red_n, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-shells", type=int, default=3000, help="oracle sample size (0 = skip)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--synthetic-boosters", action="store_true",
                    help="seeded random boosters instead of the stored quadrature boosters")
    ap.add_argument("--no-paper-order", action="store_true", help="skip timing the per-shell order")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default work split instead of the autotuned one")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the j=4 forward/adjoint block")
    ap.add_argument("--no-large", action="store_true", help="skip the large-spin batch block")
    ap.add_argument("--counter-workload", action="store_true",
                    help="run the dominant kernel and a calibration copy for rocprofv3 --pmc, then exit")
    ap.add_argument("--counter-split", type=int, nargs=2, default=[8192, 2],
                    metavar=("WORKGROUPS", "STAGING"), help="work split for --counter-workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the vertex tensor runs on a single MI355X "
              "(several GPUs would split the shell sum by ranges of cores); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2107_13952_amd as lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = workloads.CFG2
    two_j, dl = cfg["two_j"], cfg["dl"]
    dims, ilo, offs = lib.layout(two_j, dl)
    shapes = [(dims[e + 1], int((offs[e * (dl + 1) ** 3 + t + 1] - offs[e * (dl + 1) ** 3 + t]) // dims[e + 1]))
              for e in range(4) for t in range((dl + 1) ** 3)]
    b_np = None if args.synthetic_boosters else quadrature_boosters(two_j, dl, int(offs[-1]))
    physical = b_np is not None
    if not physical:
        b_np = workloads.synthetic_boosters(cfg["booster_seed"], shapes)
    b = torch.from_numpy(b_np).to(dev)
    live, terms = lib.count_terms(two_j, dl)
    work = lib.count_work(two_j, dl)
    progress(f"workload two_j={two_j} dl={dl}: {live} live shells, {terms:.3g} terms")
    out = torch.empty(dims, dtype=torch.float64, device=dev)
    if args.counter_workload:
        counter_workload(lib, torch, two_j, dl, b, args.counter_split)
        return

    lib.set_algorithm("auto")
    tuned = None
    if not args.no_autotune:
        tuned = lib.autotune(two_j, dl, b, out)
        progress(f"autotuned: {tuned}")
    ms, ring_ms, kernels = time_steps(lib, torch, two_j, dl, b, out, args.steps, args.warmup, "ring")
    progress(f"factorised order: {ms:.3f} ms/step, ring kernel {ring_ms:.3f} ms")
    useful = work["ring_useful_flops"] / (ring_ms * 1e-3) / 1e12
    executed = work["ring_mfma_flops"] / (ring_ms * 1e-3) / 1e12

    result = {
        "metric": METRIC,
        "value": terms / (ms * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": ("synthetic spins; boosters from the FP64 quadrature of eq. (booster) at "
                 "gamma=1.2 (stored oracle output)" if physical else
                 "synthetic: seeded N(0,1)/dim(k) boosters of the exact packed shape (A is "
                 "multilinear in them; the work does not depend on their values)"),
        "config": {"workload": "plain EPRL vertex tensor, equilateral j=3 (two_j=6), dl=8, "
                               "gamma=1.2, intertwiners 0..6 (7^5 FP64 tensor)",
                   "two_j": two_j, "dl": dl, "live_shells": live, "terms": terms,
                   "algorithm": "factorised shell sum (ring), FP64 matrix-core contractions",
                   "work_split": tuned or "default"},
        "roofline": {"bound": "mfma", "achieved": useful, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": useful / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(tuned),
                     "kernel": "ring_kernel", "avg_ms": ring_ms,
                     "alg_flops_per_launch": work["ring_useful_flops"],
                     "alg_flops_per_term": work["ring_useful_flops"] / terms,
                     "mfma_executed_tflops": executed,
                     "per_shell_order_flops_over_time_tflops":
                         work["shell_flops"] / (ring_ms * 1e-3) / 1e12},
        "kernels_ms": kernels,
    }
    if not args.no_paper_order:
        lib.set_algorithm("shell")
        steps = max(2, args.steps // 3)
        pms, asm_ms, pk = time_steps(lib, torch, two_j, dl, b, out, steps, 1, "assemble")
        lib.set_algorithm("auto")
        progress(f"per-shell order: {pms:.3f} ms/step, assembly kernel {asm_ms:.3f} ms")
        result["paper_order"] = {
            "ms_per_step": pms, "terms_per_s": terms / (pms * 1e-3), "kernels_ms": pk,
            "kernel_tflops": work["shell_flops"] / (asm_ms * 1e-3) / 1e12,
            "alg_flops_per_term": work["shell_flops"] / terms}
    if not args.no_batched:
        configs = workloads.cfg3_batch()
        bl = []
        for c, (tj, d) in enumerate(configs):
            dd, _, oo = lib.layout(tj, d)
            sh = [(dd[e + 1], int((oo[e * (d + 1) ** 3 + t + 1] - oo[e * (d + 1) ** 3 + t]) // dd[e + 1]))
                  for e in range(4) for t in range((d + 1) ** 3)]
            bl.append(torch.from_numpy(workloads.synthetic_boosters(
            workloads.batch_booster_seed(workloads.CFG3_SEED, c), sh)).to(dev))
        bterms = sum(lib.count_terms(tj, d)[1] for tj, d in configs)
        progress(f"batched workload: {len(configs)} configurations, {bterms:.3g} terms")
        outs = lib.vertex_tensor_batched(configs, 1.2, bl)
        torch.cuda.synchronize()
        progress("batched warm-up done")
        t0 = time.perf_counter()
        lib.vertex_tensor_batched(configs, 1.2, bl, outs)
        torch.cuda.synchronize()
        t_batched = time.perf_counter() - t0
        t0 = time.perf_counter()
        for (tj, d), bb, a in zip(configs, bl, outs):
            lib.vertex_tensor(tj, d, 1.2, bb, out=a)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        progress(f"batched {t_batched:.2f} s, plain {t_plain:.2f} s")
        result["batched"] = {"workload": "64 seeded configurations, j in 1/2..6, dl in 3..10",
                             "terms": bterms, "batched_terms_per_s": bterms / t_batched,
                             "plain_terms_per_s": bterms / t_plain}
    if not args.no_adjoint:
        progress("differentiation: j=4 dl=8 forward, contraction, adjoint")
        result["differentiation"] = differentiation(lib, torch, dev)
    if not args.no_large:
        progress("large-spin batch: 16 configurations")
        result["large_batch"] = large_batch(lib, torch, dev)
    if args.cpu_shells > 0:
        progress(f"cpu baseline: oracle on {args.cpu_shells} shells")
        result["cpu_baseline"] = cpu_baseline(two_j, dl, b_np, args.cpu_shells)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
