"""Test infrastructure: the oracle chain's stationary distribution over
partitions, against the exact posterior obtained by enumeration.

On a handful of cells every set partition c can be listed, and its posterior
p(c | x) is proportional to the partition prior of eq. 10 (with Gamma(alpha)
restored) times the product over clusters of the Dirichlet-multinomial
marginal (eq. 12 integrated against eq. 28).  Section 2.3 and Section 2.4 state
that the split/merge moves satisfy detailed balance, so a correct chain visits
each partition with that probability.  This module computes the exact
posterior with scipy's log-gamma (no oracle code), runs many independent
oracle chains from one cluster and compares their final partitions with it
(chi-square and total variation).

``python -m oracle.stationary`` prints the table of every flag combination.
"""
from __future__ import annotations

import itertools
import sys

import numpy as np
from scipy.special import gammaln
from scipy.stats import chi2

from . import EXACT, NEW_CLUSTER, RANDOM_SPLIT, SPLIT_Q, Oracle

# Tiny count matrices (cells x genes) whose posteriors spread over many
# partitions; N = 5 has 52 partitions, N = 6 has 203.
DATASETS = {
    "n5g2": np.array([[3, 0], [2, 1], [0, 3], [1, 2], [2, 2]], dtype=np.int64),
    "n6g3": np.array([[4, 0, 0], [3, 1, 0], [0, 4, 1], [0, 3, 2], [1, 0, 4], [2, 2, 2]], dtype=np.int64),
}


def set_partitions(n: int) -> list[tuple[int, ...]]:
    """Every set partition of n items as a restricted growth string."""
    out: list[tuple[int, ...]] = []

    def grow(prefix: list[int], top: int) -> None:
        if len(prefix) == n:
            out.append(tuple(prefix))
            return
        for v in range(top + 2):
            grow(prefix + [v], max(top, v))

    grow([0], 0)
    return out


def canonical(labels) -> tuple[int, ...]:
    """Relabel clusters by first appearance."""
    seen: dict[int, int] = {}
    return tuple(seen.setdefault(int(v), len(seen)) for v in labels)


def exact_posterior(X: np.ndarray, alpha: float, beta: float):
    """(partitions, probabilities) of p(c | x) for every partition of the rows."""
    N, G = X.shape
    parts = set_partitions(N)
    B = beta * G
    lp = np.empty(len(parts))
    for j, part in enumerate(parts):
        lab = np.array(part)
        K = lab.max() + 1
        v = K * np.log(alpha) + gammaln(alpha) - gammaln(alpha + N)
        for k in range(K):
            rows = X[lab == k]
            s = rows.sum(axis=0)
            v += gammaln(rows.shape[0])
            v += gammaln(B) - gammaln(B + s.sum()) + np.sum(gammaln(beta + s) - gammaln(beta))
        lp[j] = v
    p = np.exp(lp - lp.max())
    return parts, p / p.sum()


def csr(X: np.ndarray):
    rp, col, val = [0], [], []
    for row in X:
        nz = np.nonzero(row)[0]
        col.extend(nz.tolist())
        val.extend(row[nz].tolist())
        rp.append(len(col))
    return np.array(rp, np.int64), np.array(col, np.int32), np.array(val, np.int32)


def flag_kwargs(flags: int) -> dict:
    return dict(split_q=bool(flags & SPLIT_Q), new_cluster=bool(flags & NEW_CLUSTER),
                random_split=bool(flags & RANDOM_SPLIT), exact=bool(flags & EXACT))


def final_partitions(X: np.ndarray, flags: int, n_chains: int, n_iter: int, alpha: float = 1.0,
                     beta: float = 1.0, seed0: int = 1000):
    """Counts of the final partitions of n_chains independent chains (seeds
    seed0, seed0 + 1, ...) of n_iter iterations each, started from one cluster."""
    parts = set_partitions(X.shape[0])
    index = {p: j for j, p in enumerate(parts)}
    rp, col, val = csr(X)
    counts = np.zeros(len(parts), dtype=np.int64)
    for j in range(n_chains):
        o = Oracle(rp, col, val, X.shape[1], alpha=alpha, beta=beta, seed=seed0 + j,
                   k_max=X.shape[0] + 2, k_init=1, **flag_kwargs(flags))
        o.iterate(n_iter)
        counts[index[canonical(o.c)]] += 1
    return counts


def chi_square(counts: np.ndarray, p: np.ndarray, min_expected: float = 5.0):
    """Pearson chi-square of counts against probabilities p, with the
    categories of expected count below min_expected pooled into one.
    Returns (statistic, degrees of freedom, p-value)."""
    n = counts.sum()
    e = n * p
    big = e >= min_expected
    obs = list(counts[big]) + [counts[~big].sum()]
    exp = list(e[big]) + [e[~big].sum()]
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    obs = np.array(obs, float)
    exp = np.array(exp, float)
    stat = float(np.sum((obs - exp) ** 2 / exp))
    dof = len(exp) - 1
    return stat, dof, float(chi2.sf(stat, dof))


def total_variation(counts: np.ndarray, p: np.ndarray) -> float:
    return float(0.5 * np.abs(counts / counts.sum() - p).sum())


COMBINATIONS = [
    ("collapsed ratios only", 0),
    ("SPLIT_Q", SPLIT_Q),
    ("NEW_CLUSTER", NEW_CLUSTER),
    ("RANDOM_SPLIT", RANDOM_SPLIT),
    ("SPLIT_Q + NEW_CLUSTER", SPLIT_Q | NEW_CLUSTER),
    ("SPLIT_Q + RANDOM_SPLIT", SPLIT_Q | RANDOM_SPLIT),
    ("NEW_CLUSTER + RANDOM_SPLIT", NEW_CLUSTER | RANDOM_SPLIT),
    ("SPLIT_Q + NEW_CLUSTER + RANDOM_SPLIT", SPLIT_Q | NEW_CLUSTER | RANDOM_SPLIT),
    ("EXACT", EXACT),
]


def main(n_chains: int = 4000, n_iter: int = 200) -> None:
    print(f"{n_chains} chains of {n_iter} iterations from one cluster, final partitions")
    print(f"{'data':6} {'flags':40} {'TV':>7} {'chi2':>9} {'dof':>4} {'p':>9}")
    for name, X in DATASETS.items():
        _, p = exact_posterior(X, 1.0, 1.0)
        for label, flags in COMBINATIONS:
            counts = final_partitions(X, flags, n_chains, n_iter)
            stat, dof, pv = chi_square(counts, p)
            print(f"{name:6} {label:40} {total_variation(counts, p):7.4f} {stat:9.1f} {dof:4d} {pv:9.2e}",
                  flush=True)


if __name__ == "__main__":
    args = [int(a) for a in sys.argv[1:3]]
    main(*args)
