"""Pins for the oracle's sampler steps (test infrastructure).

* Redraw (eq. 4, eq. 19): empirical means of exp(log theta) and exp(log pi)
  over many steps equal the Dirichlet posterior means, row by row; this fixes
  which statistics feed which row.
* Assignment (eq. 4 third line, eq. 8): empirical label frequencies over many
  steps equal the exact categorical probabilities computed here with numpy,
  for the cluster choice, the sub-cluster choice with its n_{r,-i} weights,
  the equal-weight case and the reset coin.
* The split proposal term (SPLIT_Q): the per-cell log p(cbar_i) matches the
  frequency of the draws, and enters the split ratio as -sum over the cluster.
* The Gibbs step over K + 1 clusters (NEW_CLUSTER): the new cluster's weight
  and theta have the Dirichlet means of the alpha component and the prior.
* Random splits (RANDOM_SPLIT): coin halves, ratio = collapsed + (n - 2) log 2 =
  minus the eq. 23 merge ratio of the halves, application along the coins.
* Statistics and compaction: conservation and consistency invariants.
* Split and merge application: acceptance frequency equals min(1, R); moved
  statistics equal statistics recomputed from the moved labels.
* The whole chain: the small four-cluster recipe is recovered; a resumed chain
  is identical to an uninterrupted one.
"""
import math

import numpy as np
import pytest
from scipy import stats
from sklearn.metrics import adjusted_rand_score

import oracle
from paper_1812_10048_amd import synth


# the plain passes (sub-cluster split or merge, one fair coin), for the pins
# of one pass at a time
COLLAPSED = dict(split_q=False, new_cluster=False, random_split=False)


def _dense_oracle(X, k_max=8, beta=1.0, alpha=1.0, seed=0, **flags):
    d = synth.from_dense(X)
    rp, col, val = d.host_arrays()
    return oracle.Oracle(rp, col, val, X.shape[1], alpha=alpha, beta=beta, seed=seed, k_max=k_max, init=False,
                         **{**COLLAPSED, **flags})


def _chi2_ok(counts, probs, min_p=1e-4):
    counts = np.asarray(counts, dtype=float)
    probs = np.asarray(probs, dtype=float)
    exp = probs * counts.sum()
    keep = exp > 5
    chi = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    dof = max(1, keep.sum() - 1)
    return stats.chi2.sf(chi, dof) > min_p, (counts, exp)


# --------------------------------------------------------------------------
# statistics
# --------------------------------------------------------------------------

def test_stats_invariants():
    d = synth.generate("c1", seed=3, n_cells=600)
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, d.n_genes, seed=1, k_max=16, init=False, **COLLAPSED)
    rng = np.random.default_rng(0)
    K = 5
    c = rng.integers(0, K, size=d.n_cells)
    cs = rng.integers(0, 2, size=d.n_cells)
    o.set_state(0, K, c, cs, np.zeros(K))
    colsum = np.bincount(col, weights=val, minlength=d.n_genes)
    assert np.array_equal(o.ssub[: 2 * K].sum(0), colsum)
    assert o.nsub[: 2 * K].sum() == d.n_cells
    lib = np.add.reduceat(val, rp[:-1]) if val.size else np.zeros(d.n_cells)
    grp = 2 * c + cs
    assert np.array_equal(o.ssub[: 2 * K].sum(1), np.bincount(grp, weights=lib, minlength=2 * K))
    assert np.array_equal(o.nsub[: 2 * K], np.bincount(grp, minlength=2 * K))
    assert not o.ssub[2 * K:].any() and not o.nsub[2 * K:].any()


# --------------------------------------------------------------------------
# redraw
# --------------------------------------------------------------------------

def test_redraw_matches_dirichlet_posterior_means():
    rng = np.random.default_rng(4)
    G = 4
    X = rng.integers(0, 9, size=(7, G))
    X[:, 0] += 3
    beta = np.array([0.5, 1.0, 2.0, 0.3])
    o = _dense_oracle(X, k_max=4, beta=beta, alpha=1.7)
    c = np.array([0, 0, 0, 1, 1, 1, 1])
    cs = np.array([0, 1, 1, 0, 0, 1, 0])
    o.set_state(0, 2, c, cs, np.zeros(2))
    T = 6000
    acc_t = np.zeros((3 * 2, G))
    acc_p = np.zeros(2)
    for t in range(T):
        o.step = t
        o.redraw()
        acc_t[:2] += np.exp(o.logtheta[:2])
        acc_t[2:] += np.exp(o.logtheta[4:8])
        acc_p += np.exp(o.logpi[:2])
        np.testing.assert_allclose(np.exp(o.logtheta[:2]).sum(1), 1.0, rtol=1e-12)
    s = np.zeros((4, G))
    for i in range(7):
        s[2 * c[i] + cs[i]] += X[i]
    rows = [s[0] + s[1], s[2] + s[3], s[0], s[1], s[2], s[3]]
    for r, sr in enumerate(rows):
        a = beta + sr
        mean = a / a.sum()
        var = mean * (1 - mean) / (a.sum() + 1)
        np.testing.assert_array_less(np.abs(acc_t[r] / T - mean), 5 * np.sqrt(var / T) + 1e-12)
    n = np.array([3.0, 4.0])
    a = np.concatenate([n, [1.7]])
    mean = (a / a.sum())[:2]
    var = mean * (1 - mean) / (a.sum() + 1)
    np.testing.assert_array_less(np.abs(acc_p / T - mean), 5 * np.sqrt(var / T))


# --------------------------------------------------------------------------
# assignment
# --------------------------------------------------------------------------

def test_cluster_choice_frequencies_are_softmax():
    rng = np.random.default_rng(9)
    N, G, K = 5, 4, 3
    X = rng.integers(0, 4, size=(N, G))
    o = _dense_oracle(X, k_max=4)
    o.set_state(0, K, np.zeros(N), np.zeros(N), np.ones(K))
    logth = np.log(rng.dirichlet(np.ones(G), size=K))
    # scale so that the choices are genuinely random
    logth = logth * 0.3 + np.log(1.0 / G) * 0.7
    logpi = np.log(np.array([0.5, 0.3, 0.2]))
    T = 20000
    counts = np.zeros((N, K))
    for t in range(T):
        o.logtheta[:K] = logth
        o.logpi[:K] = logpi
        o.c[:] = 0
        o.cs[:] = 0
        o.step = t
        o.assign()
        counts[np.arange(N), o.c] += 1
    score = logpi[None, :] + X @ logth.T
    p = np.exp(score - score.max(1, keepdims=True))
    p /= p.sum(1, keepdims=True)
    for i in range(N):
        ok, info = _chi2_ok(counts[i], p[i])
        assert ok, (i, info)


def test_subcluster_choice_uses_counts_without_the_cell():
    rng = np.random.default_rng(12)
    N, G = 5, 3
    X = rng.integers(0, 3, size=(N, G))
    o = _dense_oracle(X, k_max=4)
    c = np.zeros(N, dtype=np.int32)
    cs = np.array([0, 0, 1, 1, 1], dtype=np.uint8)       # nbar = (2, 3)
    o.set_state(0, 2, c, cs, np.zeros(2))
    # cluster 1 is never chosen
    logpi = np.array([0.0, -1e6])
    lsub = np.log(rng.dirichlet(np.ones(G) * 3, size=2))
    T = 20000
    ones = np.zeros(N)
    for t in range(T):
        o.logpi[:2] = logpi
        o.logtheta[:2] = np.log(1.0 / G)
        o.logtheta[4:6] = lsub
        o.c[:] = c
        o.cs[:] = cs
        o.step = t
        o.assign()
        assert np.all(o.c == 0)
        ones += o.cs
    for i in range(N):
        w = np.array([2.0, 3.0])
        w[cs[i]] -= 1.0
        sc = np.log(w) + lsub @ X[i]
        p1 = 1.0 / (1.0 + np.exp(sc[0] - sc[1]))
        ok, info = _chi2_ok([T - ones[i], ones[i]], [1 - p1, p1])
        assert ok, (i, info)


def test_subcluster_equal_weights_and_reset_coin():
    X = np.array([[3, 1, 0], [0, 2, 2]])
    o = _dense_oracle(X, k_max=4)
    # cell 0 alone in cluster 0 (weights (0,0) -> equal), cell 1 in a reset cluster 1
    c = np.array([0, 1], dtype=np.int32)
    cs = np.array([0, 0], dtype=np.uint8)
    o.set_state(0, 2, c, cs, np.array([0, 1]))
    lsub = np.log(np.array([[0.5, 0.3, 0.2], [0.2, 0.3, 0.5]]))
    T = 20000
    ones = np.zeros(2)
    for t in range(T):
        o.logpi[:2] = [0.0, 0.0]
        o.logtheta[0] = np.log([0.998, 0.001, 0.001])
        o.logtheta[1] = np.log([0.001, 0.499, 0.5])
        o.logtheta[4:6] = lsub
        o.c[:] = c
        o.cs[:] = cs
        o.step = t
        o.assign()
        assert list(o.c) == [0, 1]
        ones += o.cs
    sc = lsub @ X[0]
    p1 = 1.0 / (1.0 + np.exp(sc[0] - sc[1]))
    assert _chi2_ok([T - ones[0], ones[0]], [1 - p1, p1])[0]
    assert _chi2_ok([T - ones[1], ones[1]], [0.5, 0.5])[0]


def test_logp_of_the_drawn_subcluster_matches_its_frequency():
    """lpsub (log p(cbar_i), eq. 8) is tied to the draws themselves: with fixed
    parameters, the probability of cbar_i = 1 implied by lpsub is the same at
    every step and equals the empirical frequency of cbar_i = 1; a reset
    cluster's coin carries log p = 0 (no proposal term)."""
    rng = np.random.default_rng(21)
    N, G = 5, 3
    X = rng.integers(0, 3, size=(N, G))
    X[:, 0] += 1
    o = _dense_oracle(X, k_max=4)
    c = np.zeros(N, dtype=np.int32)
    cs = np.array([0, 1, 1, 0, 0], dtype=np.uint8)        # nbar = (3, 2)
    o.set_state(0, 2, c, cs, np.zeros(2))
    assert np.all(o.lpsub == 0.0)
    lsub = np.log(rng.dirichlet(np.ones(G) * 2, size=2))
    T = 20000
    ones = np.zeros(N)
    p1 = np.full((T, N), np.nan)
    for t in range(T):
        o.logpi[:2] = [0.0, -1e6]                          # cluster 1 is never chosen
        o.logtheta[:2] = np.log(1.0 / G)
        o.logtheta[4:6] = lsub
        o.c[:] = c
        o.cs[:] = cs
        o.step = t
        o.assign()
        assert np.all(o.c == 0)
        ones += o.cs
        pd = np.exp(o.lpsub)                               # probability of the drawn label
        assert np.all((pd > 0) & (pd <= 1.0))
        p1[t] = np.where(o.cs == 1, pd, 1.0 - pd)
    for i in range(N):
        assert np.ptp(p1[:, i]) < 1e-12, i
        ok, info = _chi2_ok([T - ones[i], ones[i]], [1 - p1[0, i], p1[0, i]])
        assert ok, (i, info)
    # a reset cluster draws a fair coin and carries no proposal term
    o.reset[0] = 1
    o.c[:] = c
    o.cs[:] = cs
    o.step = T
    o.assign()
    assert np.all(o.lpsub == 0.0)


def test_split_q_adds_minus_the_summed_logp_to_the_split_ratio():
    """With SPLIT_Q the split ratio of every eligible cluster exceeds the plain
    one by -Q_k = -sum_{i in k} log p(cbar_i) (Section 2.3, q(S*|S) = prod p(cbar_i),
    q(S|S*) = 1); merge passes are unchanged, so the two chains agree up to the
    first split pass."""
    d = synth.generate("c1", seed=3)
    rp, col, val = d.host_arrays()
    chains = [oracle.Oracle(rp, col, val, d.n_genes, seed=5, k_max=16, init=False,
                            **{**COLLAPSED, "split_q": q}) for q in (False, True)]
    cs0 = np.random.default_rng(2).integers(0, 2, size=d.n_cells)
    for o in chains:
        o.set_state(0, d.n_true, d.z, cs0, np.ones(d.n_true, dtype=np.uint8))
    for it in range(12):
        for o in chains:
            o.sweep()
        a, b = chains
        assert np.array_equal(a.c, b.c) and np.array_equal(a.lpsub, b.lpsub)
        K = b.K
        Q = np.bincount(b.c, weights=b.lpsub, minlength=K)
        for o in chains:
            o.split_merge()
        if b.sm_pass == 1:
            assert np.array_equal(a.sm_logr[: a.sm_n], b.sm_logr[: b.sm_n], equal_nan=True)
            continue
        plain, withq = a.sm_logr[:K], b.sm_logr[:K]
        live = ~np.isnan(plain)
        assert live.any()
        assert np.array_equal(np.isnan(withq), ~live)
        assert np.allclose(withq[live] - plain[live], -Q[live], rtol=1e-9, atol=1e-9 * b.sm_scale[:K][live].max())
        assert np.all(-Q[live] >= 0)
        return
    pytest.fail("no split pass in 12 iterations")


def test_new_cluster_takes_the_alpha_weight_and_a_prior_theta():
    """NEW_CLUSTER (eq. 4 over K + 1): the appended cluster's weight is the
    alpha component of pi ~ Dir(n_1..n_K, alpha), so its mean is
    alpha / (N + alpha), and its theta is a draw from the prior Dir(beta),
    whose mean is beta_u / sum(beta).  Nothing is appended at k_max."""
    rng = np.random.default_rng(8)
    N, G, alpha = 20, 5, 1.5
    X = rng.integers(0, 4, size=(N, G))
    X[:, 0] += 1
    d = synth.from_dense(X)
    rp, col, val = d.host_arrays()
    beta = np.array([0.5, 1.0, 1.5, 2.0, 3.0])
    o = oracle.Oracle(rp, col, val, G, alpha=alpha, beta=beta, seed=4, k_max=4, init=False,
                      **{**COLLAPSED, "new_cluster": True})
    c = np.zeros(N, dtype=np.int32)
    cs = (np.arange(N) % 2).astype(np.uint8)
    T = 4000
    pin, th = np.zeros(T), np.zeros((T, G))
    for t in range(T):
        o.set_state(t, 1, c, cs, np.zeros(1))
        o.extend()
        assert o.K == 2 and o.has_new and o.reset[1] == 1
        o.redraw()
        pin[t] = np.exp(o.logpi[1])
        th[t] = np.exp(o.logtheta[1])
        assert abs(np.exp(o.logpi[:2]).sum() - 1.0) < 1e-12        # pi_{K+1} is the alpha component itself
    m, v = alpha / (N + alpha), alpha * N / ((N + alpha) ** 2 * (N + alpha + 1))
    assert abs(pin.mean() - m) < 5 * np.sqrt(v / T), (pin.mean(), m)
    pm = beta / beta.sum()
    pv = pm * (1 - pm) / (beta.sum() + 1)
    assert np.all(np.abs(th.mean(axis=0) - pm) < 5 * np.sqrt(pv / T)), (th.mean(axis=0), pm)
    # at capacity nothing is appended
    o.set_state(0, 4, np.arange(N, dtype=np.int32) % 4, cs, np.zeros(4))
    o.extend()
    assert o.K == 4 and not o.has_new


def test_gibbs_over_k_plus_one_opens_clusters_and_keeps_statistics():
    """With NEW_CLUSTER and no split/merge at all, sweeps from one cluster
    open new clusters by the Gibbs step alone (three groups of cells on three
    genes, a sparse prior), and the statistics stay those of the labels."""
    rng = np.random.default_rng(13)
    grp = np.repeat(np.arange(3), 20)
    X = rng.poisson(0.3, size=(60, 3))
    X[np.arange(60), grp] += 8
    d = synth.from_dense(X)
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, 3, alpha=2.0, beta=0.2, seed=9, k_max=16, k_init=1,
                      **{**COLLAPSED, "new_cluster": True})
    assert o.K == 1
    for _ in range(30):
        o.sweep()
        n, s_ = _recomputed_stats(o)
        assert np.array_equal(n, o.nsub[: 2 * o.K]) and np.array_equal(s_, o.ssub[: 2 * o.K])
        assert not o.has_new and n.sum() == 60
        if o.K > 1:
            return
    pytest.fail("no cluster opened in 30 sweeps")


def test_random_split_pass_halves_by_coins_and_reverses_the_merge():
    """RANDOM_SPLIT (chain B of Section 2.4): in a random-split pass each cell's
    half is its Philox coin (stream RSPLIT); each ratio is the collapsed split
    ratio of the coin halves plus (n - 2) log 2, which is exactly minus the
    eq. 23 merge ratio of the two halves; an accepted cluster splits along the
    coins, and the statistics are those of the new labels."""
    d = synth.generate("c1", seed=12)
    rp, col, val = d.host_arrays()
    seed = 31
    o = oracle.Oracle(rp, col, val, d.n_genes, seed=seed, k_max=32, init=False,
                      **{**COLLAPSED, "random_split": True})
    rng = np.random.default_rng(4)
    # the truth with two clusters merged, so that splitting them is attractive
    z = np.where(d.z == 3, 2, d.z).astype(np.int32)
    o.set_state(0, 3, z, rng.integers(0, 2, size=d.n_cells), np.zeros(3, dtype=np.uint8))
    X = np.zeros((d.n_cells, d.n_genes), dtype=np.int64)
    for i in range(d.n_cells):
        X[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    seen = 0
    for it in range(40):
        step, c_before, K = o.step, o.c.copy(), o.K
        o.split_merge()
        if o.sm_pass != 2:
            o.sweep()
            continue
        seen += 1
        bits = np.array([oracle.philox4x32_10(seed, [i, 0, step, (oracle.ST_RSPLIT << 24)])[0] >> 31
                         for i in range(d.n_cells)], dtype=np.int64)
        accepted = [k for k in range(K) if o.sm_accept[k]]
        for k in range(K):
            h = [(c_before == k) & (bits == b) for b in (0, 1)]
            n0, n1 = int(h[0].sum()), int(h[1].sum())
            if n0 < 1 or n1 < 1:
                assert np.isnan(o.sm_logr[k])
                continue
            s0, s1 = X[h[0]].sum(axis=0), X[h[1]].sum(axis=0)
            ref, scale = oracle.split_logr(s0, s1, n0, n1, o.beta, o.alpha)
            ref += (n0 + n1 - 2) * np.log(2.0)
            assert abs(o.sm_logr[k] - ref) <= 1e-9 * max(1.0, scale), (k, o.sm_logr[k], ref)
            back, bscale = oracle.merge_logr(s0, s1, n0, n1, o.beta, o.alpha)
            assert abs(o.sm_logr[k] + back) <= 1e-9 * max(1.0, bscale)
        for j, k in enumerate(accepted):
            moved = (c_before == k) & (bits == 1)
            assert np.all(o.c[moved] == K + j) and np.all(o.c[(c_before == k) & (bits == 0)] == k)
            assert o.reset[k] == 1 and o.reset[K + j] == 1
        n, s_ = _recomputed_stats(o)
        assert np.array_equal(n, o.nsub[: 2 * o.K]) and np.array_equal(s_, o.ssub[: 2 * o.K])
        if seen >= 3:
            break
        o.sweep()
    assert seen >= 3


def test_accepted_random_split_follows_the_coins():
    """A tiny cluster under a large alpha: random splits are accepted, the new
    cluster holds exactly the coin-1 cells, both parts re-draw their
    sub-labels, and the statistics are those of the labels."""
    rng = np.random.default_rng(3)
    X = rng.integers(1, 4, size=(8, 3))
    d = synth.from_dense(X)
    rp, col, val = d.host_arrays()
    seed = 5
    o = oracle.Oracle(rp, col, val, 3, alpha=200.0, seed=seed, k_max=8, init=False,
                      **{**COLLAPSED, "random_split": True})
    o.set_state(0, 1, np.zeros(8, dtype=np.int32), np.zeros(8, dtype=np.uint8), np.zeros(1, dtype=np.uint8))
    for it in range(60):
        step, c_before, K = o.step, o.c.copy(), o.K
        o.split_merge()
        if o.sm_pass != 2 or not o.sm_accept[:K].any():
            o.set_state(o.step, 1, np.zeros(8, dtype=np.int32), np.zeros(8, dtype=np.uint8), np.zeros(1, dtype=np.uint8))
            continue
        bits = np.array([oracle.philox4x32_10(seed, [i, 0, step, (oracle.ST_RSPLIT << 24)])[0] >> 31
                         for i in range(8)])
        assert K == 1 and o.K == 2
        assert np.array_equal(o.c, bits) and np.all(o.cs == 0)
        assert o.reset[0] == 1 and o.reset[1] == 1
        n, s_ = _recomputed_stats(o)
        assert np.array_equal(n, o.nsub[:4]) and np.array_equal(s_, o.ssub[:4])
        return
    pytest.fail("no accepted random split in 60 calls")


# --------------------------------------------------------------------------
# sweep bookkeeping
# --------------------------------------------------------------------------

def _recomputed_stats(o):
    K = o.K
    s = np.zeros((2 * K, o.G), dtype=np.int64)
    n = np.zeros(2 * K, dtype=np.int64)
    for i in range(o.N):
        g = 2 * o.c[i] + o.cs[i]
        n[g] += 1
        s[g, o.col[o.row_ptr[i]:o.row_ptr[i + 1]]] += o.val[o.row_ptr[i]:o.row_ptr[i + 1]]
    return n, s


def test_sweeps_keep_statistics_and_flags_consistent():
    d = synth.generate("c1", seed=5, n_cells=400)
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, d.n_genes, seed=2, k_max=32, k_init=6)
    total = np.bincount(col, weights=val, minlength=d.n_genes)
    for it in range(12):
        o.sweep()
        K = o.K
        n, s = _recomputed_stats(o)
        assert np.array_equal(n, o.nsub[: 2 * K]) and np.array_equal(s, o.ssub[: 2 * K])
        nk = n[0::2] + n[1::2]
        assert np.all(nk > 0)
        flag = (nk >= 2) & ((n[0::2] == 0) | (n[1::2] == 0))
        assert np.array_equal(o.reset[:K].astype(bool), flag)
        assert np.array_equal(o.ssub[: 2 * K].sum(0), total)
        o.split_merge()
        K = o.K
        n, s = _recomputed_stats(o)
        assert np.array_equal(n, o.nsub[: 2 * K]) and np.array_equal(s, o.ssub[: 2 * K])
        assert np.all(n[0::2] + n[1::2] > 0)
        assert o.c.max() < K


def test_split_acceptance_frequency_is_min_one_r():
    rng = np.random.default_rng(21)
    G = 3
    X = rng.integers(0, 3, size=(6, G))
    c = np.zeros(6, dtype=np.int32)
    cs = np.array([0, 1, 0, 1, 0, 1], dtype=np.uint8)
    o = _dense_oracle(X, k_max=4, alpha=1.0)
    o.set_state(0, 1, c, cs, np.zeros(1))
    # choose alpha so that log R = -1 (log R is linear in log alpha)
    logr1, _ = oracle.split_logr(o.ssub[0], o.ssub[1], 3, 3, o.beta, 1.0)
    alpha = math.exp(-1.0 - logr1)
    o = _dense_oracle(X, k_max=4, alpha=alpha)
    o.set_state(0, 1, c, cs, np.zeros(1))
    logr, _ = oracle.split_logr(o.ssub[0], o.ssub[1], 3, 3, o.beta, alpha)
    assert abs(logr + 1.0) < 1e-9
    splits = accepted = 0
    for t in range(6000):
        o.set_state(t, 1, c, cs, np.zeros(1))
        o.split_merge()
        if o.sm_pass == 0:
            splits += 1
            assert abs(o.sm_logr[0] - logr) < 1e-12
            if o.K == 2:
                accepted += 1
                # sub-cluster 1 became cluster 1, both flagged for reset
                assert np.array_equal(o.c, cs.astype(np.int32)) and not o.cs.any()
                assert list(o.reset[:2]) == [1, 1]
        else:
            assert o.K == 1
    p = math.exp(logr)
    assert abs(splits / 6000 - 0.5) < 5 * math.sqrt(0.25 / 6000)
    assert abs(accepted / splits - p) < 5 * math.sqrt(p * (1 - p) / splits)


def test_merge_pass_merges_disjoint_pairs():
    rng = np.random.default_rng(5)
    G = 4
    X = rng.integers(1, 4, size=(12, G))
    # a tiny alpha makes every merge attractive
    o = _dense_oracle(X, k_max=8, alpha=1e-30)
    c = np.repeat(np.arange(4), 3).astype(np.int32)
    cs = np.tile([0, 1, 0], 4).astype(np.uint8)
    seen_merge = False
    for t in range(40):
        o.set_state(t, 4, c, cs, np.zeros(4))
        o.split_merge()
        if o.sm_pass != 1:
            continue
        seen_merge = True
        assert o.K == 2
        # each new cluster is the union of two old clusters, with the old
        # clusters as its sub-clusters
        for k in range(2):
            members = np.nonzero(o.c == k)[0]
            old = sorted(set(c[members]))
            assert len(old) == 2
            assert np.array_equal(o.cs[members], (c[members] == old[1]).astype(np.uint8))
        n, s = _recomputed_stats(o)
        assert np.array_equal(n, o.nsub[:4]) and np.array_equal(s, o.ssub[:4])
        assert np.sum(o.sm_accept[:6]) == 2
    assert seen_merge


# --------------------------------------------------------------------------
# whole chain
# --------------------------------------------------------------------------

def test_small_recipe_recovers_its_clusters():
    d = synth.generate("c1", seed=0)
    rp, col, val = d.host_arrays()
    o = oracle.Oracle(rp, col, val, d.n_genes, alpha=1.0, beta=1.0, seed=0, k_max=64)
    o.iterate(100)
    assert o.K == d.n_true
    assert adjusted_rand_score(d.z, o.c) > 0.95


def test_resumed_chain_is_identical():
    d = synth.generate("c1", seed=1, n_cells=500)
    rp, col, val = d.host_arrays()
    a = oracle.Oracle(rp, col, val, d.n_genes, seed=4, k_max=32, beta=0.7)
    a.iterate(6)
    b = oracle.Oracle(rp, col, val, d.n_genes, seed=4, k_max=32, beta=0.7)
    b.iterate(3)
    snap = b.snapshot()
    r = oracle.Oracle(rp, col, val, d.n_genes, seed=4, k_max=32, beta=snap["beta"], init=False)
    r.set_state(snap["step"], snap["K"], snap["c"], snap["cs"], snap["reset"])
    r.iterate(3)
    assert r.K == a.K and r.step == a.step
    assert np.array_equal(r.c, a.c) and np.array_equal(r.cs, a.cs)
