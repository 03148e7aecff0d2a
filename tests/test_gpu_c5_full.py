"""Parity at the benchmark's full size and launch configuration: 1,300,000
cells x 2,000 genes, 40 power-law clusters, split-BF16, k_max 128, the default
(paper-literal) moves, started from the true partition as bench.py does.

Three iterations (sweep + split/merge) run in lockstep with the FP64 oracle
on the whole matrix (tests/lockstep.py: parameters, labels up to near ties,
statistics, log joint, Hastings ratios, near-tie counts).  In every sweep the
sweep's own log-likelihoods of one random cell per block of 256 (5,079 cells)
and of the last cell are checked: the split-BF16 cluster scores within
3e-5 relative of FP64, and from the second sweep on (no cluster re-draws its
sub-labels at random any more) the FP64 sub-cluster scores within 1e-9; the
FP64 listed-cell dump of the same cells within 1e-9.
"""
import numpy as np
import pytest
import torch

import oracle
from lockstep import Lockstep, say
from paper_1812_10048_amd import synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu


def test_benchmark_configuration_in_lockstep_with_the_oracle():
    seed = 0
    say("c5 full size: generate")
    d = synth.generate("c5", seed=seed, device="cuda")
    K0 = d.n_true
    rng = np.random.default_rng(seed)
    cs0 = rng.integers(0, 2, size=d.n_cells)
    reset = np.ones(K0, dtype=np.uint8)
    kw = dict(alpha=1.0, beta=1.0, seed=seed, k_max=128)
    s = Sampler(d.row_ptr, d.col, d.val, d.n_genes, k_init=1, precision="split_bf16", **kw)
    s.set_state(0, K0, torch.from_numpy(d.z), torch.from_numpy(cs0), reset)
    say("c5 full size: oracle state")
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, d.n_genes, init=False, **kw)
    o.set_state(0, K0, d.z, cs0, reset)
    ls = Lockstep("c5", o, s)
    ls.compare_stats()
    nblk = (d.n_cells + 255) // 256
    pick_rng = np.random.default_rng(1)
    worst = {}
    sub_checked = 0
    for step in range(3):
        say(f"c5 full size: sweep {step}")
        K = o.K
        Ks = K + 1 if K < o.k_max else K        # the Gibbs step runs over a new cluster (eq. 4)
        dbg = s.debug_scores(Ks, fp64=True)
        ls.sweep()
        s.debug_scores(None)
        cells = np.minimum(np.arange(nblk) * 256 + pick_rng.integers(0, 256, size=nblk), d.n_cells - 1)
        cells = np.unique(np.r_[cells, d.n_cells - 1]).astype(np.int64)
        got = dbg[torch.from_numpy(cells).cuda()].cpu().numpy()
        del dbg
        ref = o.cell_logliks(cells)
        K2 = o.K
        Kc = min(Ks, K2)
        rel = np.abs(got[:, :Kc] - ref[:, :Kc]) / np.maximum(1.0, np.abs(ref[:, :Kc]))
        worst[f"cluster_rel_err_sweep{step}"] = float(rel.max())
        say(f"c5 full size: sweep {step}: max relative log-likelihood error {rel.max():.3g}, "
            f"refined {s.stats()['refined']}")
        assert np.all(np.abs(got[:, :Kc] - ref[:, :Kc]) <= 3e-5 * np.abs(ref[:, :Kc]) + 1e-3)
        if step >= 1 and K2 >= K:
            live = ~np.isnan(got[:, Ks])
            assert live.mean() > 0.99
            sub = np.abs(got[live, Ks:Ks + 2] - ref[live, K2:K2 + 2]) / np.maximum(1.0, np.abs(ref[live, K2:K2 + 2]))
            worst[f"sub_rel_err_sweep{step}"] = float(sub.max())
            assert np.all(sub <= 1e-9)
            sub_checked += int(live.sum())
        dump = s.dump_scores(cells.astype(np.int32)).cpu().numpy()
        assert np.all(np.abs(dump - ref) <= 1e-9 * np.maximum(1.0, np.abs(ref)))
        say(f"c5 full size: split/merge {step}")
        ls.split_merge()
    ls.finish(sub_scores_checked=sub_checked, **worst)
    assert sub_checked > 4000
