"""Split and merge Hastings ratios at the 100,000 x 2,000 scale (12 power-law
clusters), through the C ABI, against the FP64 oracle.

The ratio kernels reduce each candidate over tiles of 512 genes and combine
the tiles in order; at G = 2,000 that is four tiles, the last one ragged.
The GPU chain runs a few sweeps from the true partition (random sub-labels);
the oracle takes its state, and both then take four split/merge passes:

  * every log R within 1e-9 of the sum of its terms' magnitudes;
  * the same accept flags, labels and statistics after every pass.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_c4_hastings_match_oracle():
    _say("c4 hastings: generate")
    d = synth.generate("c4", seed=1, device="cuda")
    G, K0 = d.n_genes, d.n_true
    rp, col, val = d.host_arrays()
    kw = dict(alpha=1.0, beta=0.5, seed=13, k_max=64)
    s = Sampler(d.row_ptr, d.col, d.val, G, k_init=1, precision="split_bf16", **kw)
    rng = np.random.default_rng(7)
    s.set_state(0, K0, torch.from_numpy(d.z), torch.from_numpy(rng.integers(0, 2, size=d.n_cells)),
                np.ones(K0, dtype=np.uint8))
    for _ in range(6):
        s.sweep(1)
    snap = s.snapshot()
    _say("c4 hastings: oracle from step", snap["step"], "K", snap["K"])
    o = oracle.Oracle(rp, col, val, G, init=False, **kw)
    o.set_state(snap["step"], snap["K"], snap["c"].cpu().numpy(), snap["cs"].cpu().numpy(),
                np.asarray(snap["reset"]))
    # both sides from the same state (set_state also clears the per-cell eq. 8
    # probabilities of the split proposal term on both)
    s.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    passes = []
    for it in range(4):
        o.split_merge()
        s.split_merge()
        p, logr, acc = s.hastings()
        assert p == o.sm_pass
        n = o.sm_n
        ref, scale = o.sm_logr[:n], o.sm_scale[:n]
        assert len(logr) == n
        assert np.array_equal(np.isnan(logr), np.isnan(ref))
        ok = ~np.isnan(ref)
        err = np.abs(logr[ok] - ref[ok]) / np.maximum(1.0, scale[ok])
        _say(f"c4 hastings: pass {p}, {n} candidates, max scaled error {err.max() if err.size else 0.0:.3g}")
        assert np.all(err <= 1e-9), err.max()
        assert np.array_equal(acc, o.sm_accept[:n])
        c, cs = s.labels()
        assert np.array_equal(c.cpu().numpy(), o.c) and np.array_equal(cs.cpu().numpy(), o.cs)
        st = s.stats(with_tables=True)
        assert st["K"] == o.K
        assert np.array_equal(st["ssub"].cpu().numpy()[:2 * o.K], o.ssub[:2 * o.K])
        passes.append(p)
    _say("c4 hastings: passes", passes)
