"""Per-sweep precision report of the split-BF16 sweep against the FP64 oracle
(a script run on a GPU machine, not a test).

The GPU chain runs on its own (sweep + split/merge, paper-literal moves) from
one cluster.  Before every sweep the oracle takes the GPU's state (labels,
reset flags, step), appends the new cluster and redraws the parameters, which
are then those the GPU draws (same Philox stream, same statistics), and forms
every cell's FP64 log-likelihood against every cluster (eq. 26).  The GPU sweep
dumps the scores its matrix-core kernel computed.  Recorded per sweep:
  * max, median and 99.9th percentile of |S_gpu - S_fp64| / max(1, |S_fp64|)
    over all cells and clusters;
  * cells re-scored in FP64 by the GPU (decisions within the certified
    rounding bound) and the GPU's count of near-tie decisions;
  * label differences from the oracle's own sweep from the same state, split
    into those whose oracle Gumbel-max margin is below 1e-6 (near ties) and
    the others (which must not occur).

With --fused the GPU sweeps run without the dump, i.e. with the sub-cluster
pass fused into the cluster draw (the benchmarked form); then only the labels,
re-scores and near ties are recorded.

usage: python tests/precision_report.py [--recipe c2] [--sweeps 200] [--seed 0] [--fused]
           [--out gpurun_out/precision_c2_split_bf16.jsonl]
           [--summary gpurun_out/split_bf16_c2_precision.txt]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1812_10048_amd import synth  # noqa: E402
from paper_1812_10048_amd.sampler import Sampler  # noqa: E402

MARGIN = 1e-6


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--recipe", default="c2")
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--k-max", type=int, default=128)
    ap.add_argument("--fused", action="store_true", help="no score dump: the fused sweep, labels only")
    ap.add_argument("--out", default=os.path.join(ROOT, "gpurun_out", "precision_c2_split_bf16.jsonl"))
    ap.add_argument("--summary", default=os.path.join(ROOT, "gpurun_out", "split_bf16_c2_precision.txt"))
    args = ap.parse_args(argv)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)

    d = synth.generate(args.recipe, seed=args.seed, device="cuda")
    rp, col, val = d.host_arrays()
    kw = dict(alpha=1.0, beta=1.0, seed=args.seed, k_max=args.k_max)
    s = Sampler(d.row_ptr, d.col, d.val, d.n_genes, k_init=1, precision="split_bf16", **kw)
    o = oracle.Oracle(rp, col, val, d.n_genes, init=False, **kw)
    new_cluster = bool(o._st.flags & oracle.NEW_CLUSTER)
    print(f"{args.recipe}: {d.n_cells} cells x {d.n_genes} genes, nnz {d.nnz}, {args.sweeps} sweeps", flush=True)
    all_cells = np.arange(d.n_cells, dtype=np.int64)
    recs = []
    t0 = time.time()
    with open(args.out, "w") as f:
        for sweep in range(args.sweeps):
            snap = s.snapshot()
            c0, cs0 = snap["c"].cpu().numpy(), snap["cs"].cpu().numpy()
            reset = np.asarray(snap["reset"])
            # this sweep's parameters on the oracle, and the FP64 scores
            o.set_state(snap["step"], snap["K"], c0, cs0, reset)
            if new_cluster:
                o.extend()
            o.redraw()
            Ks = o.K
            st0 = s.stats()
            if args.fused:
                s.sweep(1)
                rel = np.full(1, np.nan)
            else:
                # the GPU sweep with its matrix-core scores dumped
                ref = o.cell_logliks(all_cells)[:, :Ks]
                dbg = s.debug_scores(Ks, fp64=False)
                s.sweep(1)
                s.debug_scores(None)
                got = dbg[:, :Ks].double().cpu().numpy()
                del dbg
                rel = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
            st1 = s.stats()
            # the oracle's own sweep from the same state: labels and margins
            o.set_state(snap["step"], snap["K"], c0, cs0, reset)
            o.sweep()
            c1, cs1 = s.labels()
            c1, cs1 = c1.cpu().numpy(), cs1.cpu().numpy()
            bad_c = np.nonzero(c1 != o.c)[0]
            bad_s = np.nonzero((c1 == o.c) & (cs1 != o.cs))[0]
            near = int(np.sum(o.margin_c[bad_c] < MARGIN) + np.sum(o.margin_s[bad_s] < MARGIN))
            rec = dict(sweep=sweep, K=int(Ks), max_rel_err=float(rel.max()), median_rel_err=float(np.median(rel)),
                       p999_rel_err=float(np.quantile(rel, 0.999)),
                       refined=int(st1["refined"] - st0["refined"]), gpu_near_tie=int(st1["near_tie"] - st0["near_tie"]),
                       oracle_near_tie=int(np.sum(o.margin_c < MARGIN)),
                       label_mismatch=int(len(bad_c) + len(bad_s)), near_tie_mismatch=near,
                       other_mismatch=int(len(bad_c) + len(bad_s)) - near)
            f.write(json.dumps(rec) + "\n")
            f.flush()
            recs.append(rec)
            if sweep % 20 == 0 or rec["other_mismatch"]:
                print(json.dumps(rec), flush=True)
            s.split_merge()
    dt = time.time() - t0
    mx = np.array([r["max_rel_err"] for r in recs])
    md = np.array([r["median_rel_err"] for r in recs])
    form = ("the fused sweep (no score dump; labels only)" if args.fused
            else "the sweep with its matrix-core scores dumped")
    lines = [
        f"split-BF16 sweep against the FP64 oracle, per sweep: recipe {args.recipe} "
        f"({d.n_cells} cells x {d.n_genes} genes, nnz {d.nnz}), {len(recs)} sweeps from one cluster, seed {args.seed}, "
        f"paper-literal moves, k_max {args.k_max}; {form}",
        f"command: python tests/precision_report.py --recipe {args.recipe} --sweeps {args.sweeps} --seed {args.seed}"
        + (" --fused" if args.fused else ""),
        f"run time {dt:.1f} s; K after the last sweep {recs[-1]['K'] if recs else 0}",
    ]
    if not args.fused:
        lines += [
            f"max relative log-likelihood error: worst sweep {mx.max():.3e}, median over sweeps {np.median(mx):.3e}",
            f"median relative error: worst sweep {md.max():.3e}, median over sweeps {np.median(md):.3e}",
        ]
    lines += [
        f"cells re-scored in FP64: {sum(r['refined'] for r in recs)} in all; GPU near-tie decisions "
        f"{sum(r['gpu_near_tie'] for r in recs)}, oracle near-tie decisions {sum(r['oracle_near_tie'] for r in recs)}",
        f"label differences from the oracle: {sum(r['label_mismatch'] for r in recs)} "
        f"(near ties, margin < 1e-6: {sum(r['near_tie_mismatch'] for r in recs)}; others: "
        f"{sum(r['other_mismatch'] for r in recs)})",
        "",
        "sweep   K   max_rel_err  median_rel_err  p99.9_rel_err  refined  near_tie  mismatch(near/other)",
    ]
    for r in recs:
        lines.append(f"{r['sweep']:5d} {r['K']:3d}   {r['max_rel_err']:.3e}   {r['median_rel_err']:.3e}      "
                     f"{r['p999_rel_err']:.3e}    {r['refined']:6d}  {r['gpu_near_tie']:7d}   "
                     f"{r['near_tie_mismatch']}/{r['other_mismatch']}")
    with open(args.summary, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:8]), flush=True)
    return 0 if all(r["other_mismatch"] == 0 for r in recs) else 1


if __name__ == "__main__":
    sys.exit(main())
