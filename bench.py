"""Benchmark: cell x cluster log-likelihood evaluations per second of the
sub-cluster split/merge sampler on one MI355X.

A step is one pass of the whole hot path over the synthetic matrix: a sweep
(parameter redraw, log-likelihoods against every cluster and the two
sub-clusters of the chosen one, Gumbel-max assignment, sufficient statistics)
followed by a split/merge move; every 10th step also takes the empirical-Bayes
step of the per-gene concentration.  Evaluations per sweep are N (K + 2).

Prints one JSON line.  Timing: W untimed steps, then K steps between two
stream synchronisations; after that, K more steps with HIP events around every
stage (recorded by the library on its stream) give the per-stage times and
the assignment kernel's own duration.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell×cluster loglik evals/s per sweep, split-BF16 vs plain FP32, same accuracy"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (recipe, description)
    "c5": ("c5", "1,300,000 cells x 2,000 genes, 40 power-law clusters (exponent 1.5), profiles Dir(0.03), "
                 "library LogNormal(mean 3,000, sigma 0.7); start from the true partition, K = 40"),
    "c2": ("c2", "68,000 cells x 1,000 genes, 10 clusters with Dir(1) sizes, profiles Dir(0.05), "
                 "library LogNormal(mean 2,000, sigma 0.6); start from the true partition, K = 10"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(n_cells: int, nnz: int, sub_dd: bool = False) -> int:
    # packed (gene | count) entries 4 B each, padded row offsets 8 B, labels
    # read and written (int32 cluster + uint8 sub-cluster each way); with the
    # sub-cluster draw in the same kernel and the split proposal term, the FP64
    # score difference of each cell's draw written too
    return 4 * nnz + 8 * (n_cells + 1) + 10 * n_cells + (8 * n_cells if sub_dd else 0)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_assign_bf16_c5_hbm_traffic.txt")


def measured_traffic():
    """HBM bytes per launch of the matrix-core kernel from the committed
    FETCH_SIZE / WRITE_SIZE summaries (copy-calibrated), or None when they are
    missing or the kernel's sources changed since the counters were taken."""
    from paper_1812_10048_amd.profsum import source_digest
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    digests = set(re.findall(r"^source digest: (\w+)", text, re.M))
    got = {}
    for c, v in re.findall(r"^traffic (FETCH_SIZE|WRITE_SIZE) dpmm::k_assign_bf16[^:]*: ([0-9.eE+-]+) bytes per dispatch",
                           text, re.M):
        got[c] = float(v)
    if digests != {source_digest()} or set(got) != {"FETCH_SIZE", "WRITE_SIZE"}:
        return None
    return got["FETCH_SIZE"] + got["WRITE_SIZE"]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_steps(o, n_steps, budget_s=None):
    """(evaluations, seconds) of full steps (sweep + split/merge) of the
    oracle; evaluations N (K + 2) per sweep, K taken before the sweep."""
    evals = 0
    steps = 0
    t0 = time.perf_counter()
    while steps < n_steps:
        K = o.K
        o.sweep()
        o.split_merge()
        evals += o.N * (K + 2)
        steps += 1
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            break
    return evals, time.perf_counter() - t0, steps


def cpu_baseline(d, K_true, seed: int, cs0):
    """The FP64 oracle timed on the host's cores, as planned beside the GPU
    run: (i) three full steps on the whole matrix from the GPU's start state
    (all threads), (ii) a 20,000-cell sample on one thread, (iii) the
    2,000 x 500 recipe from one cluster, 100 steps (all threads)."""
    import numpy as np
    import oracle

    threads = oracle.num_threads()
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, d.n_genes, alpha=1.0, beta=1.0, seed=seed, k_max=128, init=False)
    o.set_state(0, K_true, d.z, cs0, np.ones(K_true))
    ev, dt, steps = _oracle_steps(o, 3)
    log(f"cpu oracle: {steps} steps on {d.n_cells} cells in {dt:.2f}s on {threads} threads")
    del o
    n = min(d.n_cells, 20_000)
    rp1, col1, val1 = d.host_arrays(n)
    o1 = oracle.Oracle(rp1, col1, val1, d.n_genes, alpha=1.0, beta=1.0, seed=seed, k_max=128, init=False)
    o1.set_state(0, K_true, d.z[:n], cs0[:n], np.ones(K_true))
    oracle.set_num_threads(1)
    ev1, dt1, steps1 = _oracle_steps(o1, 10 ** 9, budget_s=5.0)
    oracle.set_num_threads(threads)
    del o1
    from paper_1812_10048_amd import synth
    c1 = synth.generate("c1", seed=0)
    rpc, colc, valc = c1.host_arrays()
    oc = oracle.Oracle(rpc, colc, valc, c1.n_genes, alpha=1.0, beta=1.0, seed=0, k_max=64, k_init=1)
    evc, dtc, stepsc = _oracle_steps(oc, 100)
    return {"value": ev / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"all {d.n_cells} cells of the same matrix, {steps} full steps (sweep + split/merge, "
                      f"paper-literal moves) from the GPU run's start state, {dt:.2f} s",
            "cpu_model": cpu_model(),
            "one_thread": {"value": ev1 / dt1, "sample": f"first {n} cells, {steps1} steps in {dt1:.1f} s"},
            "c1_full_run": {"value": evc / dtc, "seconds": dtc, "steps": stepsc, "K_end": int(oc.K),
                            "sample": "2,000 x 500 recipe from one cluster, 100 steps"}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="split_bf16", choices=["fp32", "fp64", "split_bf16"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain FP32 reference run")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="copy a buffer of this many MiB once before the run, to calibrate memory counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is described "
              "in DESIGN.md but not built", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1812_10048_amd import synth
    from paper_1812_10048_amd.sampler import Sampler

    recipe, desc = WORKLOADS[args.workload]
    t0 = time.time()
    d = synth.generate(recipe, seed=args.seed, device="cuda")
    torch.cuda.synchronize()
    log(f"generated {recipe}: N={d.n_cells} G={d.n_genes} nnz={d.nnz} zeros={d.zero_fraction():.3f} "
        f"in {time.time() - t0:.1f}s")
    K_true = d.n_true
    rng = np.random.default_rng(args.seed)
    c0 = torch.from_numpy(d.z)
    cs0 = torch.from_numpy(rng.integers(0, 2, size=d.n_cells))

    def make(precision):
        smp = Sampler(d.row_ptr, d.col, d.val, d.n_genes, alpha=1.0, beta=1.0, seed=args.seed, k_init=1,
                      k_max=128, precision=precision)
        smp.set_state(0, K_true, c0, cs0, np.ones(K_true, dtype=np.uint8))
        return smp

    def step(smp, i):
        smp.sweep(1)
        smp.split_merge()
        if (i + 1) % 10 == 0:
            smp.eb_update()

    def run(precision):
        smp = make(precision)
        for i in range(args.warmup):
            step(smp, i)
        torch.cuda.synchronize()
        st0 = smp.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(smp, args.warmup + i)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st1 = smp.stats()
        # after the timed region: the same number of steps again with an event
        # pair around every stage, for the per-stage times and the average
        # duration of the assignment kernel (events on the library's stream)
        smp.timing(True)
        smp.timing_stages()
        t1 = time.perf_counter()
        for i in range(args.steps):
            step(smp, args.warmup + args.steps + i)
        torch.cuda.synchronize()
        dt_events = time.perf_counter() - t1
        stages = smp.timing_stages()
        smp.timing(False)
        kms, launches = stages["assign"]
        c, cs = smp.labels()
        res = dict(dt=dt, evals=st1["evals"] - st0["evals"], kms=kms, launches=launches, K0=st0["K"],
                   K1=st1["K"], refined=st1["refined"] - st0["refined"], near_tie=st1["near_tie"] - st0["near_tie"],
                   c=c, cs=cs, stages={k: v[0] / max(1, args.steps) for k, v in stages.items()},
                   dt_with_events=dt_events)
        log(f"{precision}: {args.steps} steps in {dt:.4f}s ({dt_events:.4f}s with stage events), K {res['K0']} -> "
            f"{res['K1']}, assign kernel {kms / max(1, launches):.4f} ms x {launches}, refined {res['refined']}, "
            f"stages ms/step " + ", ".join(f"{k} {v:.4f}" for k, v in res["stages"].items()))
        smp.close()
        return res

    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mb} MiB read + {args.copy_probe_mb} MiB written")
        del src, dst
    main_run = run(args.precision)
    cmp = None
    if args.precision != "fp32" and not args.no_compare:
        ref = run("fp32")
        same = bool(torch.equal(ref["c"], main_run["c"]) and torch.equal(ref["cs"], main_run["cs"]))
        fp32_kernel_s = ref["kms"] / 1e3 / max(1, ref["launches"])
        cmp = {"fp32_value": ref["evals"] / ref["dt"], "fp32_ms_per_step": ref["dt"] / args.steps * 1e3,
               "fp32_assign_kernel_ms": ref["kms"] / max(1, ref["launches"]),
               "fp32_assign_frac_hbm": alg_bytes(d.n_cells, d.nnz) / fp32_kernel_s / 1e9 / HBM_PEAK_GBS,
               "fp32_stages_ms_per_step": ref["stages"],
               "speedup_vs_fp32": (main_run["evals"] / main_run["dt"]) / (ref["evals"] / ref["dt"]),
               "kernel_speedup_vs_fp32": (ref["kms"] / max(1, ref["launches"])) /
                                         max(1e-12, main_run["kms"] / max(1, main_run["launches"])),
               "labels_identical_to_fp32": same}
    dt, kms, launches = main_run["dt"], main_run["kms"], main_run["launches"]
    evals = main_run["evals"]
    value = evals / dt
    st0 = {"K": main_run["K0"]}
    st1 = {"K": main_run["K1"]}

    kernel_s = kms / 1e3 / max(1, launches)
    fused = args.precision == "split_bf16"
    nbytes = alg_bytes(d.n_cells, d.nnz, sub_dd=fused)   # (paper-literal moves: the split proposal term is on)
    achieved = nbytes / kernel_s / 1e9
    kname = {"split_bf16": "k_assign_bf16 (cluster draw with the sub-cluster draw and statistics fused)",
             "fp32": "k_assign_valu<float>", "fp64": "k_assign_valu<double>"}
    traffic = measured_traffic() if args.precision == "split_bf16" and args.workload == "c5" else None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": kname[args.precision], "alg_bytes_per_launch": nbytes,
                "avg_launch_ms": kms / max(1, launches)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d, K_true, args.seed, cs0.numpy())
        log(f"cpu baseline {cpu['value']:.3e} evals/s on {cpu['cores']} threads, one thread "
            f"{cpu['one_thread']['value']:.3e}, c1 100 steps in {cpu['c1_full_run']['seconds']:.2f}s")

    dtype = {"fp32": "fp32", "fp64": "fp64", "split_bf16": "bf16"}[args.precision]
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n_cells": d.n_cells, "n_genes": d.n_genes,
                   "nnz": d.nnz, "precision": args.precision, "K_start": st0["K"], "K_end": st1["K"],
                   "step": "sweep + split/merge (+ empirical-Bayes beta step every 10th)",
                   "moves": "paper-literal: split proposal term, Gibbs over K + 1, random splits",
                   "stages_ms_per_step": main_run["stages"], "refined": main_run["refined"],
                   "near_tie": main_run["near_tie"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "comparison": cmp,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
