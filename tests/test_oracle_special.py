"""Pins for the oracle's model quantities (test infrastructure).

* lgamma / digamma differences against exact finite sums, scipy and mpmath.
* The Dirichlet-multinomial marginal (eq. 28 integrated against eq. 12):
  the beta = 1 closed form in exact integer arithmetic, normalisation over all
  count vectors of a given total, and the beta-binomial special case.
* The partition prior of eq. 10 (with Gamma(alpha)): sums to one over every
  set partition of N <= 8 points (Bell(8) = 4140) and agrees with the Chinese-restaurant
  sequential rule.
* The split and merge Hastings ratios against the collapsed joint computed
  independently in mpmath.
* The gradient of the summed log-marginal against central finite differences
  at 40 digits, and the empirical-Bayes fixed point.
"""
import itertools
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from scipy import special, stats

import oracle

mpmath.mp.dps = 40


# --------------------------------------------------------------------------
# special functions
# --------------------------------------------------------------------------

@pytest.mark.parametrize("beta", [0.5, 1.0, 2.3, 1e-3])
@pytest.mark.parametrize("s", [1, 5, 100, 3000])
def test_lgamma_difference_is_log_rising_factorial(beta, s):
    exact = math.fsum(math.log(beta + j) for j in range(s))
    got = oracle.lgamma(beta + s) - oracle.lgamma(beta)
    assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)) + 1e-12


def test_digamma_against_references():
    assert abs(oracle.digamma(1.0) + float(mpmath.euler)) < 1e-15
    xs = np.concatenate([np.geomspace(1e-6, 1e8, 400), [0.5, 1.4616321449683623, 2.0, 9.99, 10.0, 10.01]])
    for x in xs:
        ref = float(mpmath.digamma(mpmath.mpf(float(x))))
        got = oracle.digamma(float(x))
        assert abs(got - ref) <= 2e-15 * max(1.0, abs(ref)), x
        assert abs(got - special.digamma(x)) <= 1e-13 * max(1.0, abs(ref))
    for beta in (0.5, 1e-4, 3.0):
        for s in (1, 7, 500):
            exact = math.fsum(1.0 / (beta + j) for j in range(s))
            got = oracle.digamma(beta + s) - oracle.digamma(beta)
            assert abs(got - exact) <= 1e-12 * exact


# --------------------------------------------------------------------------
# Dirichlet-multinomial marginal
# --------------------------------------------------------------------------

def _log_fraction(fr: Fraction) -> float:
    return math.log(fr.numerator) - math.log(fr.denominator)


def test_logdm_beta_one_closed_form():
    # with beta = 1: integral of prod theta^s over the uniform simplex
    # = (G-1)! prod s_u! / (G-1+S)!
    rng = np.random.default_rng(3)
    for _ in range(40):
        G = int(rng.integers(2, 9))
        s = rng.integers(0, 12, size=G)
        S = int(s.sum())
        exact = Fraction(math.factorial(G - 1) * math.prod(math.factorial(int(v)) for v in s),
                         math.factorial(G - 1 + S))
        got = oracle.logdm(s, np.ones(G))
        assert abs(got - _log_fraction(exact)) < 1e-11 * max(1.0, abs(got))


def _compositions(total, parts):
    if parts == 1:
        yield (total,)
        return
    for first in range(total + 1):
        for rest in _compositions(total - first, parts - 1):
            yield (first,) + rest


@pytest.mark.parametrize("G,L", [(2, 9), (3, 6), (4, 4)])
def test_logdm_normalises_over_count_vectors(G, L):
    rng = np.random.default_rng(G * 10 + L)
    beta = rng.uniform(0.2, 3.0, size=G)
    tot = math.fsum(
        math.exp(math.lgamma(L + 1) - sum(math.lgamma(v + 1) for v in x) + oracle.logdm(np.array(x), beta))
        for x in _compositions(L, G))
    assert abs(tot - 1.0) < 1e-12


def test_logdm_two_genes_is_beta_binomial():
    for a, b in [(0.3, 2.0), (1.0, 1.0), (5.0, 0.7)]:
        for n in (1, 10, 250):
            for k in (0, 1, n // 2, n):
                ref = stats.betabinom.logpmf(k, n, a, b) - (special.gammaln(n + 1) - special.gammaln(k + 1)
                                                            - special.gammaln(n - k + 1))
                got = oracle.logdm(np.array([k, n - k]), np.array([a, b]))
                assert abs(got - ref) < 1e-9 * max(1.0, abs(ref))


def test_logdm_is_an_integral_over_theta():
    # direct numerical integration over the 2-simplex of theta^s Dir(theta|beta)
    from scipy import integrate
    beta = np.array([0.7, 1.9])
    s = np.array([3, 5])
    f = lambda t: t ** s[0] * (1 - t) ** s[1] * stats.beta(beta[0], beta[1]).pdf(t)
    val, _ = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13)
    assert abs(oracle.logdm(s, beta) - math.log(val)) < 1e-10


# --------------------------------------------------------------------------
# partition prior
# --------------------------------------------------------------------------

def _set_partitions(n):
    def rec(i, blocks):
        if i == n:
            yield [list(b) for b in blocks]
            return
        for b in blocks:
            b.append(i)
            yield from rec(i + 1, blocks)
            b.pop()
        blocks.append([i])
        yield from rec(i + 1, blocks)
        blocks.pop()
    yield from rec(0, [])


@pytest.mark.parametrize("alpha", [0.3, 1.0, 2.5])
@pytest.mark.parametrize("n", [1, 3, 5, 7, 8])
def test_partition_prior_sums_to_one(alpha, n):
    tot = math.fsum(math.exp(oracle.log_partition_prior([len(b) for b in p], alpha))
                    for p in _set_partitions(n))
    assert abs(tot - 1.0) < 1e-12


def test_partition_prior_matches_sequential_crp():
    # Chinese restaurant: point i joins block b with prob n_b/(alpha+i), opens one with alpha/(alpha+i)
    alpha = 0.8
    for p in itertools.islice(_set_partitions(6), 0, 203, 7):
        label = {}
        for bi, b in enumerate(p):
            for i in b:
                label[i] = bi
        counts, logp, order = {}, 0.0, {}
        for i in range(6):
            b = label[i]
            if b not in counts:
                logp += math.log(alpha / (alpha + i))
                counts[b] = 1
            else:
                logp += math.log(counts[b] / (alpha + i))
                counts[b] += 1
        assert abs(oracle.log_partition_prior([len(b) for b in p], alpha) - logp) < 1e-12


# --------------------------------------------------------------------------
# split / merge ratios against the collapsed joint in mpmath
# --------------------------------------------------------------------------

def _mp_logdm(s, beta):
    B = mpmath.fsum(beta)
    S = int(sum(s))
    t = mpmath.loggamma(B) - mpmath.loggamma(B + S)
    for v, b in zip(s, beta):
        t += mpmath.loggamma(b + int(v)) - mpmath.loggamma(b)
    return t


def _mp_log_joint(blocks, X, beta, alpha):
    """log p(c) + sum_k logDM(s_k) with p(c) from the sequential CRP rule."""
    N = X.shape[0]
    label = np.empty(N, dtype=int)
    for bi, b in enumerate(blocks):
        label[list(b)] = bi
    counts, lp = {}, mpmath.mpf(0)
    for i in range(N):
        b = label[i]
        if b not in counts:
            lp += mpmath.log(mpmath.mpf(alpha) / (alpha + i))
            counts[b] = 1
        else:
            lp += mpmath.log(mpmath.mpf(counts[b]) / (alpha + i))
            counts[b] += 1
    for b in blocks:
        lp += _mp_logdm(X[list(b)].sum(axis=0), [mpmath.mpf(float(v)) for v in beta])
    return lp


def test_split_and_merge_ratios_match_collapsed_joint():
    rng = np.random.default_rng(11)
    for trial in range(30):
        N = int(rng.integers(2, 8))
        G = int(rng.integers(2, 6))
        X = rng.integers(0, 6, size=(N, G))
        beta = rng.uniform(0.2, 2.0, size=G)
        alpha = float(rng.uniform(0.1, 3.0))
        # a random 2-way split of all points (both sides non-empty)
        side = rng.integers(0, 2, size=N)
        side[0], side[-1] = 0, 1
        A = [i for i in range(N) if side[i] == 0]
        B = [i for i in range(N) if side[i] == 1]
        before = _mp_log_joint([list(range(N))], X, beta, alpha)
        after = _mp_log_joint([A, B], X, beta, alpha)
        ref = float(after - before)
        got, scale = oracle.split_logr(X[A].sum(0), X[B].sum(0), len(A), len(B), beta, alpha)
        assert abs(got - ref) <= 1e-12 * max(1.0, scale), trial
        mref = -ref + (N - 2) * math.log(0.5)
        mgot, _ = oracle.merge_logr(X[A].sum(0), X[B].sum(0), len(A), len(B), beta, alpha)
        assert abs(mgot - mref) <= 1e-12 * max(1.0, scale), trial


# --------------------------------------------------------------------------
# gradient and empirical Bayes
# --------------------------------------------------------------------------

def _mp_objective(s, beta, g):
    return mpmath.fsum(gj * _mp_logdm(sj, beta) for sj, gj in zip(s, g))


def test_dm_logmarginal_matches_mpmath():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 40, size=(5, 7))
    s[1, :3] = 0
    beta = rng.uniform(0.05, 3.0, size=7)
    got = oracle.dm_logmarginal(s, beta)
    for j in range(5):
        ref = _mp_logdm(s[j], [mpmath.mpf(float(b)) for b in beta])
        assert abs(got[j] - float(ref)) < 1e-12 * max(1.0, abs(float(ref)))


def test_dm_gradient_matches_central_differences():
    rng = np.random.default_rng(8)
    J, G = 6, 9
    s = rng.integers(0, 300, size=(J, G))
    s[rng.random((J, G)) < 0.3] = 0
    beta = rng.uniform(0.05, 2.5, size=G)
    g = rng.normal(size=J)
    got = oracle.dm_grad(s, beta, g)
    h = mpmath.mpf("1e-6")
    bmp = [mpmath.mpf(float(b)) for b in beta]
    gmp = [mpmath.mpf(float(v)) for v in g]
    for u in range(G):
        up = list(bmp)
        dn = list(bmp)
        up[u] += h
        dn[u] -= h
        fd = (_mp_objective(s, up, gmp) - _mp_objective(s, dn, gmp)) / (2 * h)
        assert abs(got[u] - float(fd)) <= 1e-9 * max(1.0, abs(float(fd))), u


def test_eb_update_climbs_to_a_stationary_point():
    # statistics of three clusters; EB treats the cluster vectors as the data
    rng = np.random.default_rng(2)
    G = 6
    X = np.zeros((3, G), dtype=np.int64)
    for k in range(3):
        X[k] = rng.multinomial(400, rng.dirichlet(np.full(G, 0.8)))
    # a tiny "dataset": one cell per cluster carrying its whole count vector
    rows = [np.nonzero(X[k])[0] for k in range(3)]
    row_ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])])
    col = np.concatenate(rows).astype(np.int32)
    val = np.concatenate([X[k][rows[k]] for k in range(3)]).astype(np.int32)
    o = oracle.Oracle(row_ptr, col, val, G, alpha=1.0, beta=0.5, seed=1, k_max=8, init=False)
    o.set_state(0, 3, np.arange(3), np.zeros(3), np.zeros(3))
    obj = lambda: float(np.sum(oracle.dm_logmarginal(X, o.beta)))
    prev = obj()
    for _ in range(5000):
        o.eb_update()
        cur = obj()
        assert cur >= prev - 1e-9 * abs(prev)
        prev = cur
    # at the fixed point the gradient of the summed log-marginal vanishes
    grad = oracle.dm_grad(X, o.beta, np.ones(3))
    assert np.max(np.abs(grad)) < 1e-6
