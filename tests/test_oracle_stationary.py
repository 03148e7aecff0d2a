"""The oracle chain's stationary distribution over partitions, against the
exact posterior p(c | x) enumerated on tiny data (test infrastructure).

Section 2.3 and Section 2.4 rest the sampler's correctness on detailed
balance, i.e. on p(c | x) being the chain's stationary distribution.  Here the
posterior of every set partition of 5 or 6 cells is computed with scipy's
log-gamma (eq. 10 with Gamma(alpha), eq. 12 integrated against eq. 28, no
oracle code), and the final partitions of thousands of independent oracle
chains are compared with it by a chi-square test.

* The exact chain (oracle.EXACT: a sweep that would empty a cluster is undone,
  one atomic chain-B move per call with the Hastings ratio of its own proposal
  probabilities) passes.  Its pass pins together the Dirichlet redraw, the
  Gumbel-max draws, the log-marginals, the partition prior and the ratios.
* The same harness rejects the exact chain's counts against the posterior of a
  different alpha, so a pass is not for lack of power.

The chains built from the paper's own moves (sub-cluster splits, parallel
split and merge passes, the Gibbs step over K + 1) do not pass at this size;
``python -m oracle.stationary`` prints their measured distances.
"""
import numpy as np
import pytest

import oracle
from oracle import stationary as S


@pytest.mark.parametrize("name", ["n5g2", "n6g3"])
def test_exact_chain_visits_partitions_with_their_posterior(name):
    X = S.DATASETS[name]
    parts, p = S.exact_posterior(X, 1.0, 1.0)
    assert len(parts) == {5: 52, 6: 203}[X.shape[0]]          # Bell numbers
    counts = S.final_partitions(X, oracle.EXACT, n_chains=3000, n_iter=150, seed0=7000)
    stat, dof, pv = S.chi_square(counts, p)
    assert pv > 1e-3, (stat, dof, pv)
    assert S.total_variation(counts, p) < 0.08


def test_harness_rejects_a_wrong_posterior():
    X = S.DATASETS["n5g2"]
    counts = S.final_partitions(X, oracle.EXACT, n_chains=3000, n_iter=150, seed0=7000)
    _, p_wrong = S.exact_posterior(X, 3.0, 1.0)
    _, _, pv = S.chi_square(counts, p_wrong)
    assert pv < 1e-6


def test_exact_sweep_never_empties_a_cluster():
    X = S.DATASETS["n6g3"]
    rp, col, val = S.csr(X)
    o = oracle.Oracle(rp, col, val, 3, seed=3, k_max=8, init=False, exact=True)
    o.set_state(0, 6, np.arange(6), np.zeros(6), np.ones(6))        # all singletons
    reverts = 0
    for _ in range(200):
        o.sweep()
        assert o.K == 6 and sorted(o.c) == list(range(6))
        reverts = o.counters()["sweep_reverts"]
    # singletons keep their cell only when every cell draws its own cluster
    assert reverts > 0


def test_exact_moves_carry_their_selection_probabilities():
    """One atomic move per call: a split of cluster k among K has ratio
    logR_c + n log 2 - log(K + 1), a merge of a pair among K clusters
    -logR_c - n log 2 + log K (logR_c the collapsed ratio)."""
    X = S.DATASETS["n6g3"]
    rp, col, val = S.csr(X)
    o = oracle.Oracle(rp, col, val, 3, alpha=0.7, seed=11, k_max=8, init=False, exact=True)
    seen = set()
    lab = np.array([0, 0, 1, 1, 2, 2], dtype=np.int32)
    for t in range(200):
        o.set_state(t, 3, lab, np.zeros(6), np.zeros(3))
        o.split_merge()
        assert o.sm_n == 1
        if np.isnan(o.sm_logr[0]):
            continue
        after = np.array(S.canonical(o.c)) if o.sm_accept[0] else None
        if o.sm_pass == 1:
            # which pair: the merged pair if accepted; else recompute all
            cands = []
            for k2 in range(1, 3):
                for k1 in range(k2):
                    a, b = lab == k1, lab == k2
                    r, _ = oracle.split_logr(X[a].sum(0), X[b].sum(0), a.sum(), b.sum(), np.ones(3), 0.7)
                    cands.append(-r - (a.sum() + b.sum()) * np.log(2.0) + np.log(3.0))
            assert np.min(np.abs(np.array(cands) - o.sm_logr[0])) < 1e-12
            seen.add("merge")
        else:
            assert o.sm_pass == 2
            # the coins of the cells (stream RSPLIT at this step)
            side = np.array([oracle.philox4x32_10(11, [i, 0, t, oracle.ST_RSPLIT << 24])[0] >> 31
                             for i in range(6)])
            cands = []
            for k in range(3):
                a, b = (lab == k) & (side == 0), (lab == k) & (side == 1)
                if a.any() and b.any():
                    r, _ = oracle.split_logr(X[a].sum(0), X[b].sum(0), a.sum(), b.sum(), np.ones(3), 0.7)
                    cands.append(r + (a.sum() + b.sum()) * np.log(2.0) - np.log(4.0))
            assert np.min(np.abs(np.array(cands) - o.sm_logr[0])) < 1e-12
            if after is not None:
                assert after.max() == 3
            seen.add("split")
    assert seen == {"merge", "split"}
