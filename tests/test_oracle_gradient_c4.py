"""The oracle's Dirichlet-multinomial gradient (the beta gradient, eq. 12
integrated against eq. 28) at the 100,000 x 2,000 scale with 12 clusters
and 24 sub-clusters, against central finite differences evaluated in mpmath.

The objective is sum_j g_j logDM(s_j; beta).  Only the terms that depend on
beta_u are differentiated: lgamma(B) - lgamma(B + S_j) (B = sum of beta) and
lgamma(beta_u + s_ju) - lgamma(beta_u).  With 40 digits and h = 1e-6 the
central difference is accurate to ~1e-12 relative, so the target 1e-6 has
ample room.  The genes are chosen with Philox draws.
"""
import mpmath
import numpy as np
import pytest

import oracle
from paper_1812_10048_amd import synth

mpmath.mp.dps = 40
H = mpmath.mpf("1e-6")


@pytest.fixture(scope="module")
def c4_stats():
    d = synth.generate("c4", seed=0, device="cpu")
    rp, col, val = d.host_arrays()
    rng = np.random.default_rng(7)
    sub = rng.integers(0, 2, size=d.n_cells)
    K = d.n_true
    # rows 2k + r: the sub-cluster statistics of a random halving of each true cluster
    grp = np.repeat(2 * d.z.astype(np.int64) + sub, np.diff(rp))
    ssub = np.zeros((2 * K, d.n_genes), dtype=np.int64)
    np.add.at(ssub, (grp, col), val)
    clusters = ssub[0::2] + ssub[1::2]
    return np.concatenate([clusters, ssub]), K, d.n_genes


def _philox_genes(G, n, key=0x5EED):
    genes = []
    i = 0
    while len(genes) < n:
        w = oracle.philox4x32_10(key, [i, 0, 0, 0])
        g = int(w[0]) % G
        if g not in genes:
            genes.append(g)
        i += 1
    return genes


def _fd(s, beta, g, u):
    """Central difference of sum_j g_j logDM(s_j; beta) in beta_u (beta_u-dependent terms)."""
    S = s.sum(axis=1)
    B0 = mpmath.fsum(mpmath.mpf(float(b)) for b in beta)
    bu = mpmath.mpf(float(beta[u]))
    h = H * min(1, bu)          # beta_u may sit at the 1e-6 floor of the EB clamp

    def f(delta):
        B = B0 + delta
        b = bu + delta
        return mpmath.fsum(mpmath.mpf(float(gj)) * (mpmath.loggamma(B) - mpmath.loggamma(B + int(Sj)) +
                                                     mpmath.loggamma(b + int(sj[u])) - mpmath.loggamma(b))
                           for sj, Sj, gj in zip(s, S, g))

    return float((f(h) - f(-h)) / (2 * h))


@pytest.mark.parametrize("weights", ["all", "clusters"])
@pytest.mark.parametrize("beta_kind", ["flat", "per_gene"])
def test_gradient_at_c4_scale_matches_mpmath_differences(c4_stats, weights, beta_kind):
    s, K, G = c4_stats
    J = s.shape[0]
    assert J == 3 * K == 36
    if beta_kind == "flat":
        beta = np.full(G, 0.5)
    else:
        beta = 0.5 * np.exp(0.3 * np.random.default_rng(3).normal(size=G))
    g = np.ones(J) if weights == "all" else np.r_[np.ones(K), np.zeros(2 * K)]
    got = oracle.dm_grad(s, beta, g)
    for u in _philox_genes(G, 50):
        ref = _fd(s, beta, g, u)
        assert abs(got[u] - ref) <= 1e-6 * max(1.0, abs(ref)), (u, got[u], ref)
