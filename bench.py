"""Benchmark of the EPRL vertex-tensor hot path on one MI355X.

One step = one full vertex tensor of the equilateral j = 3 (two_j = 6), dl = 8 workload
(7^5 FP64 output, 531441 shells of which 498955 live): 6j tables, {15j} assembly with the
four booster mode products, shell-sum reduction and normalisation.  Inputs (seeded synthetic
boosters of the right ragged shape) are resident in HBM before the timed region.

Prints one JSON line:
  value        {15j} x booster terms per second (terms = sum over live shells of
               dim(i1) prod_e dim(k_e), independent of the algorithm)
  roofline     the assembly kernel's algorithmic FP64 rate against the chip's FP64 peak,
               with its average duration measured by HIP events on the library's stream
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
  batched      cfg3-shaped batch (64 seeded configurations): batched call vs per-config calls
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 (vector and matrix) peak
METRIC = "{15j}×booster terms/s (FP64) & FP64-MFMA util; batched vs plain, 1 GPU @1e-10"


def shell_grid_dims(dims, offs, dl):
    """Per-shell k dimensions (dk2..dk5) over the (dl+1)^6 grid from the packed layout."""
    nd = dl + 1
    nd3 = nd ** 3
    sizes = np.diff(offs).reshape(4, nd3)
    kd = [sizes[e] // dims[e + 1] for e in range(4)]
    o = np.indices((nd,) * 6).reshape(6, -1)
    t = [(o[0] * nd + o[1]) * nd + o[2], (o[3] * nd + o[4]) * nd + o[0],
         (o[5] * nd + o[1]) * nd + o[3], (o[2] * nd + o[4]) * nd + o[5]]
    return [kd[e][t[e]].astype(np.int64) for e in range(4)]


def mode_macs(dims, kdims):
    d1, d2, d3, d4, d5 = dims
    k2, k3, k4, k5 = kdims
    live = (k2 > 0) & (k3 > 0) & (k4 > 0) & (k5 > 0)
    m5 = d1 * k2 * k3 * k4 * k5 * d5
    m4 = d1 * k2 * k3 * k4 * d5 * d4
    m3 = d1 * k2 * k3 * d4 * d5 * d3
    m2 = d1 * k2 * d3 * d4 * d5 * d2
    return float(np.sum(np.where(live, m5 + m4 + m3 + m2, 0)))


def sampled_xterms(two_j, dl, dims, ilo, kdims, nsample=1500, seed=0):
    """Estimate of sum over live shells and (i1, k2..k5) of the number of allowed x values."""
    nd = dl + 1
    k2, k3, k4, k5 = kdims
    live = np.nonzero((k2 > 0) & (k3 > 0) & (k4 > 0) & (k5 > 0))[0]
    rng = np.random.default_rng(seed)
    pick = rng.choice(live, size=min(nsample, live.size), replace=False)
    j = list(two_j)
    total = 0.0
    for s in pick:
        o = [(s // nd ** (5 - q)) % nd for q in range(6)]
        l23, l24, l25, l34, l35, l45 = (j[4 + q] + 2 * o[q] for q in range(6))
        # lowest k of each edge: max(|p-q|, |r-s|) of its pairing
        klo = [max(abs(l23 - l24), abs(l25 - j[0])), max(abs(l34 - l35), abs(j[1] - l23)),
               max(abs(l45 - j[2]), abs(l24 - l34)), max(abs(j[3] - l25), abs(l35 - l45))]
        ks = [klo[e] + 2 * np.arange(kdims[e][s]) for e in range(4)]
        i1 = ilo[0] + 2 * np.arange(dims[0])
        I1, K2, K3, K4, K5 = np.meshgrid(i1, *ks, indexing="ij")
        lo = np.maximum.reduce([abs(I1 - l25), abs(K5 - j[2]), abs(l35 - K4), abs(l24 - K3), abs(j[1] - K2)])
        hi = np.minimum.reduce([I1 + l25, K5 + j[2], l35 + K4, l24 + K3, j[1] + K2])
        total += np.maximum(0, (hi - lo) // 2 + 1).sum()
    return total * live.size / pick.size


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


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-shells", type=int, default=3000, help="oracle sample size (0 = skip)")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the vertex tensor on a single "
              "MI355X (see the sharding notes in DESIGN.md); use --gpus 1", file=sys.stderr)
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
    b_np = workloads.synthetic_boosters(cfg["booster_seed"], shapes)
    b = torch.from_numpy(b_np).to(dev)
    live, terms = lib.count_terms(two_j, dl)
    kd = shell_grid_dims(dims, offs, dl)
    macs = mode_macs(dims, kd)
    xterms = sampled_xterms(two_j, dl, dims, ilo, kd)
    alg_flops = 2.0 * macs + 6.0 * xterms

    progress(f"workload two_j={two_j} dl={dl}: {live} live shells, {terms:.3g} terms")
    out = torch.empty(dims, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        lib.vertex_tensor(two_j, dl, 1.2, b, out=out)
    torch.cuda.synchronize()
    lib.timing_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        lib.vertex_tensor(two_j, dl, 1.2, b, out=out)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    asm_ms, asm_n = lib.timing_read("assemble")
    tab_ms, tab_n = lib.timing_read("sixj_tables")
    red_ms, red_n = lib.timing_read("reduce")
    lib.timing_enable(False)
    asm_avg = asm_ms / max(asm_n, 1)
    progress(f"timed {args.steps} steps: {ms:.3f} ms/step, assembly kernel {asm_avg:.3f} ms")
    achieved = alg_flops / (asm_avg * 1e-3) / 1e12

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
        "data": "synthetic: seeded N(0,1)/dim(k) boosters of the exact packed shape (A is "
                "multilinear in them; the work does not depend on their values)",
        "config": {"workload": "plain EPRL vertex tensor, equilateral j=3 (two_j=6), dl=8, "
                               "gamma=1.2, intertwiners 0..6 (7^5 FP64 tensor)",
                   "two_j": two_j, "dl": dl, "live_shells": live, "terms": terms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "assemble_kernel", "avg_ms": asm_avg,
                     "alg_flops_per_launch": alg_flops,
                     "alg_flops_per_term": alg_flops / terms},
        "kernels_ms": {"sixj_tables": tab_ms / max(tab_n, 1), "assemble": asm_avg,
                       "reduce": red_ms / max(red_n, 1)},
    }
    if not args.no_batched:
        configs = workloads.cfg3_batch()
        bl = []
        for c, (tj, d) in enumerate(configs):
            dd, _, oo = lib.layout(tj, d)
            sh = [(dd[e + 1], int((oo[e * (d + 1) ** 3 + t + 1] - oo[e * (d + 1) ** 3 + t]) // dd[e + 1]))
                  for e in range(4) for t in range((d + 1) ** 3)]
            bl.append(torch.from_numpy(workloads.synthetic_boosters(1003 + 1000 + c, sh)).to(dev))
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
    if args.cpu_shells > 0:
        progress(f"cpu baseline: oracle on {args.cpu_shells} shells")
        result["cpu_baseline"] = cpu_baseline(two_j, dl, b_np, args.cpu_shells)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
