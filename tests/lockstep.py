"""Lockstep comparison of the GPU sampler (through the C ABI) with the FP64
oracle, for the GPU tests (test helper, not collected).

Both sides start from the same state and draw the same Philox numbers.  After
every step:
  * log pi and log theta: |gpu - oracle| <= 1e-9 max(1, |oracle|);
  * labels equal, except cells whose oracle Gumbel-max margin is below 1e-6
    (near ties, which a different rounding may decide the other way); after
    such a step both sides are re-synchronised from the GPU state, so the
    comparison goes on instead of stopping;
  * statistics bit-exact, the log joint within 1e-9 relative;
  * split/merge log R within 1e-9 of the sum of its terms' magnitudes, the
    same accept decisions and pass;
  * the GPU's near-tie counter equal to the oracle's count of cluster
    decisions with margin below 1e-6.
Each run appends one JSON line (steps compared, near-tie cells, re-syncs,
largest errors) to gpurun_out/parity_report.jsonl when that folder exists.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import torch

MARGIN = 1e-6
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def report(record: dict) -> None:
    d = os.path.join(os.environ.get("GRAFT_REPO_ROOT", ROOT), "gpurun_out")
    if os.path.isdir(d):
        with open(os.path.join(d, "parity_report.jsonl"), "a") as f:
            f.write(json.dumps(record) + "\n")


class Lockstep:
    def __init__(self, name: str, o, s):
        self.name, self.o, self.s = name, o, s
        self.sweeps = self.sm_calls = 0
        self.near_tie_cells = 0          # cells decided differently at a near tie
        self.resyncs = 0
        self.oracle_near_ties = 0        # oracle cluster decisions with margin < 1e-6
        self.gpu_near_ties = 0           # the GPU counter, summed over re-syncs
        self.passes = {0: 0, 1: 0, 2: 0}
        self.accepted = 0
        self.err = {"params": 0.0, "logr": 0.0, "log_joint": 0.0}

    # -- comparisons ---------------------------------------------------------
    def labels(self):
        c, cs = self.s.labels()
        return c.cpu().numpy(), cs.cpu().numpy()

    def compare_labels(self, what: str) -> int:
        o = self.o
        c, cs = self.labels()
        bad_c = np.nonzero(c != o.c)[0]
        bad_s = np.nonzero((c == o.c) & (cs != o.cs))[0]
        assert np.all(o.margin_c[bad_c] < MARGIN), (self.name, what, bad_c[:10], o.margin_c[bad_c][:10])
        assert np.all(o.margin_s[bad_s] < MARGIN), (self.name, what, bad_s[:10], o.margin_s[bad_s][:10])
        return len(bad_c) + len(bad_s)

    def compare_stats(self):
        o, s = self.o, self.s
        st = s.stats(with_tables=True)
        K = st["K"]
        assert K == o.K, (self.name, K, o.K)
        assert np.array_equal(st["nsub"], o.nsub[: 2 * K])
        assert np.array_equal(st["ssub"].cpu().numpy(), o.ssub[: 2 * K])
        ref = o.log_joint()
        e = abs(st["log_joint"] - ref) / max(1.0, abs(ref))
        assert e <= 1e-9, (self.name, st["log_joint"], ref)
        self.err["log_joint"] = max(self.err["log_joint"], e)
        return st

    def compare_params(self):
        o = self.o
        K = o.K
        lp, lt = self.s.params()
        lp = lp.cpu().numpy()[:K]
        lt = lt.cpu().numpy()
        ref_lp = o.logpi[:K]
        assert np.all(np.abs(lp - ref_lp) <= 1e-9 * np.maximum(1.0, np.abs(ref_lp)))
        gc, rc = lt[:K], o.logtheta[:K]
        gs, rs = lt[o.k_max: o.k_max + 2 * K], o.logtheta[o.k_max: o.k_max + 2 * K]
        e = max(np.max(np.abs(gc - rc) / np.maximum(1.0, np.abs(rc)), initial=0.0),
                np.max(np.abs(gs - rs) / np.maximum(1.0, np.abs(rs)), initial=0.0))
        assert e <= 1e-9, (self.name, e)
        self.err["params"] = max(self.err["params"], float(e))

    def compare_hastings(self):
        o = self.o
        p, logr, acc = self.s.hastings()
        assert p == o.sm_pass
        n = o.sm_n
        assert len(logr) == n
        ref, scale = o.sm_logr[:n], o.sm_scale[:n]
        assert np.array_equal(np.isnan(logr), np.isnan(ref))
        ok = ~np.isnan(ref)
        err = np.abs(logr[ok] - ref[ok]) / np.maximum(1.0, scale[ok])
        assert np.all(err <= 1e-9), (self.name, err.max())
        assert np.array_equal(acc, o.sm_accept[:n])
        if err.size:
            self.err["logr"] = max(self.err["logr"], float(err.max()))
        self.passes[p] = self.passes.get(p, 0) + 1
        self.accepted += int(acc.sum())

    # -- steps ----------------------------------------------------------------
    def resync(self):
        """Both sides take the GPU's state (labels, reset flags, step)."""
        o, s = self.o, self.s
        self.gpu_near_ties += s.stats()["near_tie"]
        snap = s.snapshot()
        c, cs = snap["c"].cpu().numpy(), snap["cs"].cpu().numpy()
        o.set_state(snap["step"], snap["K"], c, cs, np.asarray(snap["reset"]))
        s.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
        self.resyncs += 1

    def sweep(self):
        o, s = self.o, self.s
        o.sweep()
        s.sweep(1)
        self.sweeps += 1
        self.oracle_near_ties += int(np.sum(o.margin_c < MARGIN))
        self.compare_params()
        m = self.compare_labels(f"sweep {self.sweeps}")
        if m:
            self.near_tie_cells += m
            self.resync()
        self.compare_stats()
        return m

    def split_merge(self):
        o, s = self.o, self.s
        o.split_merge()
        s.split_merge()
        self.sm_calls += 1
        self.compare_hastings()
        # the decisions are equal, so are the labels
        assert self.compare_labels(f"split/merge {self.sm_calls}") == 0
        self.compare_stats()

    def iterate(self, n: int):
        for _ in range(n):
            self.sweep()
            self.split_merge()

    def finish(self, **extra) -> dict:
        gpu_nt = self.gpu_near_ties + self.s.stats()["near_tie"]
        assert gpu_nt == self.oracle_near_ties, (self.name, gpu_nt, self.oracle_near_ties)
        rec = dict(test=self.name, sweeps=self.sweeps, sm_calls=self.sm_calls,
                   near_tie_mismatch_cells=self.near_tie_cells, resyncs=self.resyncs,
                   near_tie_decisions=gpu_nt, passes=self.passes, accepted=self.accepted,
                   K=int(self.o.K), max_err=self.err, **extra)
        report(rec)
        say(json.dumps(rec))
        return rec
