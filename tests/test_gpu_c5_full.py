"""Parity at the benchmark's full size and launch configuration: 1,300,000
cells x 2,000 genes, 40 power-law clusters, split-BF16, k_max 128, started
from the true partition as bench.py does.

Two steps (sweep + split/merge) run in lockstep with the FP64 oracle on the
whole matrix:
  * log pi and log theta within 1e-9 (relative, floor 1);
  * every label equal, except cells whose oracle Gumbel-max margin is below
    1e-6; the statistics (int64, 2K x G) equal whenever the labels are;
  * the Hastings ratios within 1e-9 of the sum of their terms' magnitudes and
    the accept decisions equal;
  * in the first sweep, the split-BF16 log-likelihoods of 3,000 sampled cells
    against every cluster within 3e-5 relative of FP64, and the FP64
    sub-cluster scores within 1e-6.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu

MARGIN = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check_labels(o, s, what):
    c, cs = s.labels()
    c, cs = c.cpu().numpy(), cs.cpu().numpy()
    bad_c = np.nonzero(c != o.c)[0]
    bad_s = np.nonzero((c == o.c) & (cs != o.cs))[0]
    assert np.all(o.margin_c[bad_c] < MARGIN), (what, bad_c[:10], o.margin_c[bad_c][:10])
    assert np.all(o.margin_s[bad_s] < MARGIN), (what, bad_s[:10], o.margin_s[bad_s][:10])
    return len(bad_c) + len(bad_s)


def _check_stats(o, s):
    st = s.stats(with_tables=True)
    K = st["K"]
    assert K == o.K
    assert np.array_equal(st["nsub"], o.nsub[: 2 * K])
    assert np.array_equal(st["ssub"].cpu().numpy(), o.ssub[: 2 * K])


def _check_params(o, s):
    K = o.K
    lp, lt = s.params()
    lp, lt = lp.cpu().numpy()[:K], lt.cpu().numpy()
    assert np.all(np.abs(lp - o.logpi[:K]) <= 1e-9 * np.maximum(1.0, np.abs(o.logpi[:K])))
    for g, r in ((lt[:K], o.logtheta[:K]), (lt[o.k_max: o.k_max + 2 * K], o.logtheta[o.k_max: o.k_max + 2 * K])):
        assert np.max(np.abs(g - r) / np.maximum(1.0, np.abs(r))) <= 1e-9


def _check_hastings(o, s):
    p, logr, acc = s.hastings()
    assert p == o.sm_pass
    n = o.sm_n
    ref, scale = o.sm_logr[:n], o.sm_scale[:n]
    assert np.array_equal(np.isnan(logr), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.all(np.abs(logr[ok] - ref[ok]) <= 1e-9 * np.maximum(1.0, scale[ok]))
    assert np.array_equal(acc, o.sm_accept[:n])


def test_benchmark_configuration_in_lockstep_with_the_oracle():
    seed = 0
    _say("c5 full size: generate")
    d = synth.generate("c5", seed=seed, device="cuda")
    K0 = d.n_true
    rng = np.random.default_rng(seed)
    cs0 = rng.integers(0, 2, size=d.n_cells)
    reset = np.ones(K0, dtype=np.uint8)
    kw = dict(alpha=1.0, beta=1.0, seed=seed, k_max=128)
    s = Sampler(d.row_ptr, d.col, d.val, d.n_genes, k_init=1, precision="split_bf16", **kw)
    s.set_state(0, K0, torch.from_numpy(d.z), torch.from_numpy(cs0), reset)
    _say("c5 full size: oracle state")
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, d.n_genes, init=False, **kw)
    o.set_state(0, K0, d.z, cs0, reset)
    _check_stats(o, s)
    for step in range(2):
        _say(f"c5 full size: sweep {step}")
        K = o.K
        dbg = s.debug_scores(K) if step == 0 else None
        o.sweep()
        s.sweep(1)
        _check_params(o, s)
        mism = _check_labels(o, s, f"sweep {step}")
        _say(f"c5 full size: sweep {step}: {mism} near-tie mismatches, refined {s.stats()['refined']}")
        if dbg is not None:
            cells = np.sort(np.random.default_rng(1).choice(d.n_cells, size=3000, replace=False))
            ref = o.cell_logliks(cells)
            got = dbg[torch.from_numpy(cells).cuda()].cpu().numpy()
            s.debug_scores(None)
            rel = np.abs(got[:, :K] - ref[:, :K]) / np.maximum(1.0, np.abs(ref[:, :K]))
            _say(f"c5 full size: max relative log-likelihood error {rel.max():.3g}")
            assert np.all(np.abs(got[:, :K] - ref[:, :K]) <= 3e-5 * np.abs(ref[:, :K]) + 1e-3)
            live = ~np.isnan(got[:, K])
            assert np.all(np.abs(got[live, K:K + 2] - ref[live, K:K + 2]) <=
                          1e-6 * np.abs(ref[live, K:K + 2]) + 1e-3)
        if mism:
            return    # the chains part at a near-tie; what followed is compared above
        _check_stats(o, s)
        o.split_merge()
        s.split_merge()
        _check_hastings(o, s)
        if _check_labels(o, s, f"split/merge {step}"):
            return
        _check_stats(o, s)
