"""Benchmark of the EPRL vertex-tensor hot path on one MI355X.

One step = the whole hot path over the large-spin batch: 16 seeded irregular 4-simplices with
spins j in {5, 5.5, 6, 6.5, 7}, dl = 6 (intertwiner dimensions 10..14, 4.9e11 {15j} x booster
terms), gamma = 1.2: the 16 vertex tensors in one batched call (6j tables, the factorised shell
sum in one persistent launch, reductions and normalisation, replayed from a captured graph),
then for every configuration the boundary contraction with five seeded unit complex vectors and
its adjoint (gradients with respect to the vectors and to every booster entry).  Inputs
(seeded synthetic boosters of the exact packed shape) are resident in HBM before the timed
region.

Prints one JSON line:
  value        {15j} x booster terms of the 16 vertex tensors per second of step
  roofline     the persistent factorised kernel: its useful FP64 flops (exact count of the
               multiply-adds its active index ranges need) per launch divided by its average
               launch duration (HIP events on the library's stream, from a second pass that
               enqueues the batch's launches directly), against the MI355X FP64 peak
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload, on every host core
  batched_vs_plain  forward only: the batched call against 16 plain calls (median of replays)
  Extra blocks: the equilateral j = 3, dl = 8 plain vertex (``plain_j3_dl8``), the 64-configuration
  irregular batch (``irregular_batch``), the j = 3 shell scan dl = 0..8 (``shell_scan_j3``), the
  device booster builder on the j = 3, dl = 8 vertex (``booster_builder_j3_dl8``) and the j = 4,
  dl = 8 differentiation check (``differentiation``).
"""
import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector and matrix) peak
METRIC = "{15j}×booster terms/s (FP64) & FP64-MFMA util; batched vs plain, 1 GPU @1e-10"


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_block(args):
    """Oracle partial vertex tensor over one block of shells (worker process, one thread)."""
    two_j, dl, boosters, lo, hi = args
    from threadpoolctl import threadpool_limits
    from oracle import ranges as R
    from oracle import vertex as V
    with threadpool_limits(limits=1):
        V.vertex_tensor(two_j, dl, boosters, shells=R.all_shells(dl)[lo:hi])
    return hi - lo


def cpu_baseline(two_j, dl, boosters_np, shells_per_worker):
    """The oracle on a contiguous block of shells of one configuration, split over a pool of
    worker processes (one per host core, one thread each)."""
    from multiprocessing import get_context
    from oracle import ranges as R
    # One worker per host core available to this process, at most 16 (the host share of one GPU).
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(16, avail))
    shells = R.all_shells(dl)
    mid = len(shells) // 2
    n = shells_per_worker * cores
    block = shells[mid:mid + n]
    n1 = R.boundary_ranges(two_j)[0][1]
    terms = 0.0
    for s in block:
        two_l = R.shell_spins(two_j, s)
        kd = [R.virtual_range(two_l, e)[1] for e in range(2, 6)]
        terms += n1 * float(np.prod(kd))
    jobs = [(two_j, dl, boosters_np, mid + w * shells_per_worker, mid + (w + 1) * shells_per_worker)
            for w in range(cores)]
    # Forked before this process touches the GPU (the baseline runs first), so no child ever
    # holds a GPU context.
    with get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_block, jobs[:1])          # import cost outside the timed region
        t0 = time.perf_counter()
        pool.map(_oracle_block, jobs)
        dt = time.perf_counter() - t0
    return {"value": terms / dt, "unit": "terms/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} consecutive shells (from index {mid}) of configuration 0 of the batch "
                      f"(two_j={two_j}, dl={dl}), {terms:.3g} terms in {dt:.1f} s on {cores} "
                      f"worker processes, one thread each (os.cpu_count() = {os.cpu_count()}, "
                      f"{avail} in this process's affinity mask)"}


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


def measured_traffic(name, key, source):
    """HBM bytes per launch of a kernel from a committed counter summary, when it was taken on
    the current kernel source file `source` (same sha256 prefix) and names `key`; else None."""
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2107_13952_amd", "csrc", source)
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m = re.search(r"kernel source sha256 ([0-9a-f]{16})", text)
    t = re.search(re.escape(key) + r": ([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


def block_shapes(lib, two_j, dl):
    """(rows, cols) of every packed booster block, from the library's layout."""
    dims, _, offs = lib.layout(two_j, dl)
    n3 = (dl + 1) ** 3
    return [(dims[e + 1], int((offs[e * n3 + t + 1] - offs[e * n3 + t]) // dims[e + 1]))
            for e in range(4) for t in range(n3)]


def event_times(torch, fn, reps, warmup=1):
    """Per-call durations (ms) of fn() between HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for r in range(reps):
        fn()
        ev[r + 1].record()
    torch.cuda.synchronize()
    return [ev[r].elapsed_time(ev[r + 1]) for r in range(reps)]


def spread(ms):
    return {"median_ms": statistics.median(ms), "min_ms": min(ms), "max_ms": max(ms), "reps": len(ms)}


class LargeBatch:
    """The 16-configuration large-spin batch with its boundary vectors and output buffers."""

    def __init__(self, lib, torch, dev):
        self.lib, self.torch = lib, torch
        self.configs = workloads.cfg5_batch()
        self.b_np = [workloads.synthetic_boosters(workloads.batch_booster_seed(workloads.CFG5_SEED, c),
                                                  block_shapes(lib, tj, d))
                     for c, (tj, d) in enumerate(self.configs)]
        self.b = [torch.from_numpy(x).to(dev) for x in self.b_np]
        self.terms = sum(lib.count_terms(tj, d)[1] for tj, d in self.configs)
        self.outs = [torch.empty(lib.layout(tj, d)[0], dtype=torch.float64, device=dev)
                     for tj, d in self.configs]
        self.psis = [[torch.from_numpy(p).to(dev) for p in workloads.boundary_vectors(
            workloads.CFG5_SEED * 10 + c, lib.layout(tj, d)[0])] for c, (tj, d) in enumerate(self.configs)]
        self.F = []
        self.grads = []

    def forward_batched(self):
        self.lib.vertex_tensor_batched(self.configs, 1.2, self.b, self.outs)

    def forward_plain(self):
        for (tj, d), bb, a in zip(self.configs, self.b, self.outs):
            self.lib.vertex_tensor(tj, d, 1.2, bb, out=a)

    def adjoint(self):
        self.F, self.grads = [], []
        for (tj, d), bb, a, ps in zip(self.configs, self.b, self.outs, self.psis):
            self.F.append(self.lib.contract_boundary(a, ps))
            self.grads.append(self.lib.contract_boundary_adjoint(tj, d, bb, a, ps, 1.0))

    def step(self):
        self.forward_batched()
        self.adjoint()


def plain_j3(lib, torch, dev, synthetic, autotune, steps):
    """The equilateral j = 3, dl = 8 vertex, plain calls (the tensor of the paper's Sec. 3.3
    scaling with all spins equal), with the roofline of its factorised kernel."""
    cfg = workloads.CFG2
    two_j, dl = cfg["two_j"], cfg["dl"]
    dims, _, offs = lib.layout(two_j, dl)
    b_np = None if synthetic else quadrature_boosters(two_j, dl, int(offs[-1]))
    physical = b_np is not None
    if not physical:
        b_np = workloads.synthetic_boosters(cfg["booster_seed"], block_shapes(lib, two_j, dl))
    b = torch.from_numpy(b_np).to(dev)
    out = torch.empty(dims, dtype=torch.float64, device=dev)
    terms = lib.count_terms(two_j, dl)[1]
    work = lib.count_work(two_j, dl)
    tuned = lib.autotune(two_j, dl, b, out) if autotune else None
    # (target workgroups, staging level) of the work split the timed calls use
    split = (tuned["target_workgroups"], tuned["staging_level"]) if tuned else (8192, 2)
    ms = event_times(torch, lambda: lib.vertex_tensor(two_j, dl, 1.2, b, out=out), steps, 3)
    lib.timing_enable(True)
    for _ in range(steps):
        lib.vertex_tensor(two_j, dl, 1.2, b, out=out)
    torch.cuda.synchronize()
    kms, kn = lib.timing_read("ring")
    lib.timing_enable(False)
    ring_ms = kms / max(kn, 1)
    med = statistics.median(ms)
    return {"workload": "plain EPRL vertex tensor, equilateral j=3 (two_j=6), dl=8, 7^5 FP64 tensor, "
                        + ("quadrature boosters" if physical else "seeded boosters"),
            "terms": terms, "terms_per_s": terms / (med * 1e-3), "step": spread(ms),
            "work_split": tuned or "default",
            "ring_kernel": {"avg_ms": ring_ms, "alg_flops_per_launch": work["ring_useful_flops"],
                            "achieved_tflops": work["ring_useful_flops"] / (ring_ms * 1e-3) / 1e12,
                            "frac": work["ring_useful_flops"] / (ring_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                            "mfma_executed_tflops": work["ring_mfma_flops"] / (ring_ms * 1e-3) / 1e12,
                            "traffic": measured_traffic("ring_kernel_j3_dl8_counters.md",
                                                        "traffic bytes per launch, split "
                                                        f"{split[0]} {split[1]}", "ring.hip")}}


def irregular_batch(lib, torch, dev, reps):
    """64 seeded irregular configurations (j in 1/2..6, dl in 3..10): batched vs plain calls."""
    configs = workloads.cfg3_batch()
    bl = [torch.from_numpy(workloads.synthetic_boosters(
        workloads.batch_booster_seed(workloads.CFG3_SEED, c), block_shapes(lib, tj, d))).to(dev)
        for c, (tj, d) in enumerate(configs)]
    terms = sum(lib.count_terms(tj, d)[1] for tj, d in configs)
    outs = [torch.empty(lib.layout(tj, d)[0], dtype=torch.float64, device=dev) for tj, d in configs]
    # First call of a new batch shape: planning, schedules, metadata upload, graph capture and
    # the run itself (host wall clock).
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lib.vertex_tensor_batched(configs, 1.2, bl, outs)
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    tb = event_times(torch, lambda: lib.vertex_tensor_batched(configs, 1.2, bl, outs), reps)
    tp = event_times(torch, lambda: [lib.vertex_tensor(tj, d, 1.2, bb, out=a)
                                     for (tj, d), bb, a in zip(configs, bl, outs)], reps)
    return {"workload": "64 seeded configurations, j in 1/2..6, dl in 3..10", "terms": terms,
            "batched_terms_per_s": terms / (statistics.median(tb) * 1e-3),
            "plain_terms_per_s": terms / (statistics.median(tp) * 1e-3),
            "batched": spread(tb), "plain": spread(tp),
            "first_call_ms": first_ms,
            "first_call_host_ms_estimate": first_ms - statistics.median(tb)}


def shell_scan(lib, torch, dev, reps):
    """A(dl) for dl = 0..8 of the equilateral j = 3 vertex from one booster buffer packed for
    dl = 8 (one batched call) against the nine plain calls on their own packed boosters."""
    cfg = workloads.CFG2
    two_j, dl_max = cfg["two_j"], cfg["dl"]
    b = torch.from_numpy(workloads.synthetic_boosters(cfg["booster_seed"],
                                                      block_shapes(lib, two_j, dl_max))).to(dev)
    out = lib.vertex_tensor_scan(two_j, dl_max, 1.2, b)
    # Per-dl buffers for the plain calls: the blocks of each dl taken out of the dl_max buffer.
    _, _, offs = lib.layout(two_j, dl_max)
    n3 = (dl_max + 1) ** 3
    sub = []
    for d in range(dl_max + 1):
        idx = [e * n3 + (o1 * (dl_max + 1) + o2) * (dl_max + 1) + o3 for e in range(4)
               for o1 in range(d + 1) for o2 in range(d + 1) for o3 in range(d + 1)]
        sub.append(torch.cat([b[int(offs[q]):int(offs[q + 1])] for q in idx]))
    terms = sum(lib.count_terms(two_j, d)[1] for d in range(dl_max + 1))
    ts = event_times(torch, lambda: lib.vertex_tensor_scan(two_j, dl_max, 1.2, b, out=out), reps)
    tp = event_times(torch, lambda: [lib.vertex_tensor(two_j, d, 1.2, sub[d], out=out[d])
                                     for d in range(dl_max + 1)], reps)
    return {"workload": "shell scan A(dl), dl = 0..8, equilateral j=3 (two_j=6), seeded boosters",
            "terms": terms, "scan": spread(ts), "plain_calls": spread(tp),
            "scan_terms_per_s": terms / (statistics.median(ts) * 1e-3),
            "plain_terms_per_s": terms / (statistics.median(tp) * 1e-3),
            "single_dl8_terms": lib.count_terms(two_j, dl_max)[1]}


def booster_builder(lib, torch, dev, reps):
    """The boosters of the equilateral j = 3, dl = 8 vertex (eq. (booster), 2916 blocks) by the
    device quadrature, against the oracle's quadrature stored beside the j = 3 parity tensor."""
    cfg = workloads.CFG2
    two_j, dl = cfg["two_j"], cfg["dl"]
    _, _, offs = lib.layout(two_j, dl)
    out = torch.empty(int(offs[-1]), dtype=torch.float64, device=dev)
    _, info = lib.boosters(two_j, dl, 1.2, out=out)
    ms = event_times(torch, lambda: lib.boosters(two_j, dl, 1.2, out=out), reps)
    ref = quadrature_boosters(two_j, dl, int(offs[-1]))
    err = None
    if ref is not None:
        err = float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max())
    # The boosters of configuration 0 of the large-spin batch (spins 5..7, dl = 6): timing and the
    # quadrature's own error estimate (the oracle would take hours for this one).
    tj5, d5 = workloads.cfg5_batch()[0]
    _, _, offs5 = lib.layout(tj5, d5)
    out5 = torch.empty(int(offs5[-1]), dtype=torch.float64, device=dev)
    _, info5 = lib.boosters(tj5, d5, 1.2, out=out5)
    ms5 = event_times(torch, lambda: lib.boosters(tj5, d5, 1.2, out=out5), 2)
    return {"workload": "boosters of the equilateral j=3 (two_j=6), dl=8 vertex, gamma=1.2, "
                        f"{int(offs[-1])} values", "time": spread(ms), "subintervals": info["n"],
            "error_estimate": info["error"], "max_imag": info["imag"],
            "normwise_vs_oracle_quadrature": err,
            "large_spin_config0": {"two_j": list(tj5), "dl": d5, "values": int(offs5[-1]),
                                   "time": spread(ms5), "subintervals": info5["n"],
                                   "error_estimate_rel": info5["error"] / float(out5.abs().max()),
                                   "max_imag": info5["imag"]}}


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
    t_fwd = statistics.median(event_times(torch, lambda: lib.vertex_tensor(two_j, dl, 1.2, b, out=A), 5))
    t_con = statistics.median(event_times(torch, lambda: lib.contract_boundary(A, psis), 10))
    t_adj = statistics.median(event_times(
        torch, lambda: lib.contract_boundary_adjoint(two_j, dl, b, A, psis, 1.0), 5))
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
            "forward_ms": t_fwd, "forward_terms_per_s": terms / (t_fwd * 1e-3),
            "contract_us": t_con * 1e3, "adjoint_ms": t_adj,
            "adjoint_vs_central_difference_max_rel_err": worst}


def counter_workload(lib, torch, dev, which):
    """The kernel named by `which` three times (the large-spin batch, the j = 3, dl = 8 vertex, or
    that vertex in the per-shell order), then a plain 256 MiB device copy three times (the copy
    calibrates what FETCH_SIZE and WRITE_SIZE read for a known number of bytes)."""
    if which == "batch":
        lb = LargeBatch(lib, torch, dev)
        for _ in range(3):
            lb.forward_batched()
    else:
        cfg = workloads.CFG2
        two_j, dl = cfg["two_j"], cfg["dl"]
        b = torch.from_numpy(workloads.synthetic_boosters(cfg["booster_seed"],
                                                          block_shapes(lib, two_j, dl))).to(dev)
        # "j3shell": the per-shell order of the framed algorithm on the same vertex.
        lib.set_algorithm("shell" if which == "j3shell" else "auto")
        for _ in range(3):
            lib.vertex_tensor(two_j, dl, 1.2, b)
        lib.set_algorithm("auto")
    torch.cuda.synchronize()
    x = torch.ones(32 << 20, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("counter workload done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-shells", type=int, default=400,
                    help="oracle shells per host core for the CPU baseline (0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline step (no j=3 plain, irregular batch or j=4 blocks)")
    ap.add_argument("--synthetic-boosters", action="store_true",
                    help="seeded boosters for the j=3 block instead of the stored quadrature ones")
    ap.add_argument("--no-autotune", action="store_true", help="default work split for the j=3 block")
    ap.add_argument("--counter-workload", choices=["batch", "j3", "j3shell"],
                    help="run one kernel three times and a calibration copy for rocprofv3 --pmc, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the vertex tensors run on a single MI355X "
              "(several GPUs would split a batch by configuration, or one vertex by ranges of "
              "cores, with one sum of the partial tensors at the end); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    cpu = None
    if args.cpu_shells > 0 and not args.counter_workload:
        # The oracle's leg runs first, on the host only, before anything initialises the GPU.
        from oracle import ranges as R
        tj, d = workloads.cfg5_batch()[0]
        b0 = workloads.synthetic_boosters(workloads.batch_booster_seed(workloads.CFG5_SEED, 0),
                                          R.block_shapes(tj, d))
        progress(f"cpu baseline: oracle on {args.cpu_shells} shells per host core")
        cpu = cpu_baseline(tj, d, b0, args.cpu_shells)
        progress(f"cpu baseline: {cpu['value']:.3g} terms/s")

    import torch
    import paper_2107_13952_amd as lib

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.counter_workload:
        counter_workload(lib, torch, dev, args.counter_workload)
        return

    lb = LargeBatch(lib, torch, dev)
    works = [lib.count_work(tj, d) for tj, d in lb.configs]
    useful = sum(w["ring_useful_flops"] for w in works)
    executed = sum(w["ring_mfma_flops"] for w in works)
    classes = sorted({w["ring_class"] for w in works})
    progress(f"large-spin batch: {len(lb.configs)} configurations, {lb.terms:.3g} terms, tile classes {classes}")
    lib.set_algorithm("auto")
    lb.forward_batched()                       # capture
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        lb.step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        lb.step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    progress(f"step {ms:.1f} ms (median {statistics.median(step_ms):.1f})")
    # Forward only, batched graph vs plain calls.
    fb = event_times(torch, lb.forward_batched, 5)
    fp = event_times(torch, lb.forward_plain, 5)
    fa = event_times(torch, lb.adjoint, 3)
    progress(f"forward batched {statistics.median(fb):.1f} ms, plain {statistics.median(fp):.1f} ms, "
             f"contraction + adjoint {statistics.median(fa):.1f} ms")
    # Second pass with the library's per-launch events on (the batch then enqueues its launches
    # directly instead of replaying the graph).
    lib.timing_enable(True)
    for _ in range(3):
        lb.forward_batched()
    torch.cuda.synchronize()
    kms, kn = lib.timing_read("ring_batch")
    tab_ms, tab_n = lib.timing_read("sixj_tables")
    red_ms, red_n = lib.timing_read("reduce")
    lib.timing_enable(False)
    lib.timing_enable(True)
    for _ in range(2):
        lb.adjoint()
    torch.cuda.synchronize()
    adj_ms, adj_n = lib.timing_read("adjoint_shells")
    lib.timing_enable(False)
    launches = kn / 3.0
    kernel_ms = kms / max(kn, 1)
    alg_per_launch = useful / max(launches, 1.0)
    achieved = alg_per_launch / (kernel_ms * 1e-3) / 1e12
    # Every configuration of this batch takes the all-matrix-core factorised kernel (class 8)
    # unless the planner picked otherwise; the roofline names the kernel that ran.
    kname, ksrc = ("wide_batch_kernel", "wide.hip") if classes == [8] else ("ring_batch_kernel", "ring.hip")
    progress(f"{kname} {kernel_ms:.2f} ms per launch ({launches:g} launches per step): "
             f"{achieved:.2f} TFLOP/s useful")

    result = {
        "metric": METRIC,
        "value": lb.terms / (ms * 1e-3),
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded spins, N(0,1)/dim(k) boosters of the exact packed shape (A is "
                "multilinear in them; the work does not depend on their values) and unit complex "
                "Gaussian boundary vectors",
        "config": {"workload": "large-spin batch: 16 seeded irregular 4-simplices, j in 5..7, dl=6, "
                               "gamma=1.2, intertwiner dims 10..14; step = batched vertex tensors + "
                               "boundary contraction and adjoint of each",
                   "configs": [{"two_j": tj, "dl": d} for tj, d in lb.configs],
                   "terms": lb.terms, "tile_classes": classes,
                   "algorithm": "factorised shell sum (ring), FP64 matrix-core contractions, one "
                                "persistent launch per tile class in a captured graph"},
        "step_spread": spread(step_ms),
        "batched_vs_plain": {"forward_batched": spread(fb), "forward_plain": spread(fp),
                             "batched_terms_per_s": lb.terms / (statistics.median(fb) * 1e-3),
                             "plain_terms_per_s": lb.terms / (statistics.median(fp) * 1e-3),
                             "contraction_and_adjoint": spread(fa)},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(f"{kname}_large_batch_counters.md",
                                                 "traffic bytes per launch", ksrc),
                     "kernel": kname, "avg_ms": kernel_ms,
                     "launches_per_step": launches,
                     "alg_flops_per_launch": alg_per_launch,
                     "alg_flops_per_term": useful / lb.terms,
                     "mfma_executed_tflops": executed / max(launches, 1.0) / (kernel_ms * 1e-3) / 1e12},
        "kernels_ms_per_step": {"sixj_tables": tab_ms / 3, "ring_batch": kms / 3, "reduce": red_ms / 3,
                                "adjoint_shells": adj_ms / 2},
    }
    if not args.no_extras:
        progress("plain j=3 dl=8")
        result["plain_j3_dl8"] = plain_j3(lib, torch, dev, args.synthetic_boosters,
                                          not args.no_autotune, 10)
        progress("irregular batch")
        result["irregular_batch"] = irregular_batch(lib, torch, dev, 5)
        progress("shell scan j=3 dl=0..8")
        result["shell_scan_j3"] = shell_scan(lib, torch, dev, 5)
        progress("booster builder j=3 dl=8")
        result["booster_builder_j3_dl8"] = booster_builder(lib, torch, dev, 3)
        progress("differentiation j=4 dl=8")
        result["differentiation"] = differentiation(lib, torch, dev)
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
