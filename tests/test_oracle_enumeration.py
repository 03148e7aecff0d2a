"""Exhaustive pins of the oracle's Hastings ratios and log joint on N <= 8
cells, in exact rational arithmetic (test infrastructure).

With beta = 1 and two genes the Dirichlet-multinomial marginal (eq. 12
integrated against eq. 28, multinomial coefficient dropped as in eq. 26) is
s0! s1! / (S + 1)!, and the partition prior of eq. 10 with Gamma(alpha)
restored is alpha^K Gamma(alpha) prod_k Gamma(n_k) / Gamma(alpha + N); both
are exact rationals for integer alpha.  Every 2-way split of every block of
8 cells is checked against the ratio of these joints (the collapsed split
ratio; the merge of eq. 23 is its inverse times (1/2)^(n - 2)), and the
oracle's log joint is checked on every set partition of 7 cells.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

X8 = np.array([[3, 0], [2, 1], [0, 4], [1, 2], [2, 2], [5, 1], [0, 1], [1, 0]], dtype=np.int64)


def _fact(n: int) -> int:
    return math.factorial(n)


def _dm(s) -> Fraction:
    """Dirichlet-multinomial marginal, beta = 1, G = 2."""
    s0, s1 = int(s[0]), int(s[1])
    return Fraction(_fact(s0) * _fact(s1), _fact(s0 + s1 + 1))


def _prior(sizes, alpha: int) -> Fraction:
    N = sum(sizes)
    num = alpha ** len(sizes) * _fact(alpha - 1)
    for n in sizes:
        num *= _fact(n - 1)
    return Fraction(num, _fact(alpha + N - 1))


def _log(q: Fraction) -> float:
    return math.log(q.numerator) - math.log(q.denominator)


@pytest.mark.parametrize("alpha", [1, 3])
def test_every_two_way_split_of_every_block_of_eight(alpha):
    beta = np.ones(2)
    cells = range(X8.shape[0])
    checked = 0
    for size in range(2, 9):
        for block in itertools.combinations(cells, size):
            first, rest = block[0], block[1:]
            s = X8[list(block)].sum(0)
            for r in range(0, len(rest)):          # side A holds the first cell
                for extra in itertools.combinations(rest, r):
                    A = [first, *extra]
                    B = [i for i in block if i not in A]
                    sA, sB = X8[A].sum(0), X8[B].sum(0)
                    ratio = (Fraction(alpha) * Fraction(_fact(len(A) - 1) * _fact(len(B) - 1), _fact(size - 1))
                             * _dm(sA) * _dm(sB) / _dm(s))
                    ref = _log(ratio)
                    got, scale = oracle.split_logr(sA, sB, len(A), len(B), beta, float(alpha))
                    assert abs(got - ref) <= 1e-13 * max(1.0, scale), (block, A)
                    mgot, _ = oracle.merge_logr(sA, sB, len(A), len(B), beta, float(alpha))
                    mref = -ref + (size - 2) * math.log(0.5)
                    assert abs(mgot - mref) <= 1e-13 * max(1.0, scale), (block, A)
                    checked += 1
    assert checked == (3 ** 8 - 2 ** 9 + 1) // 2      # sum_b C(8, b) (2^(b-1) - 1)


def _partitions(n):
    def grow(prefix, top):
        if len(prefix) == n:
            yield list(prefix)
            return
        for v in range(top + 2):
            yield from grow(prefix + [v], max(top, v))
    yield from grow([0], 0)


@pytest.mark.parametrize("alpha", [1, 2])
def test_log_joint_on_every_partition_of_seven(alpha):
    X = X8[:7]
    rp = np.concatenate([[0], np.cumsum((X > 0).sum(1))]).astype(np.int64)
    col = np.concatenate([np.nonzero(r)[0] for r in X]).astype(np.int32)
    val = np.concatenate([r[r > 0] for r in X]).astype(np.int32)
    o = oracle.Oracle(rp, col, val, 2, alpha=float(alpha), beta=1.0, seed=0, k_max=8, init=False)
    n = 0
    for lab in _partitions(7):
        lab = np.array(lab)
        K = int(lab.max()) + 1
        o.set_state(0, K, lab, np.zeros(7, np.uint8), np.zeros(K, np.uint8))
        joint = _prior([int((lab == k).sum()) for k in range(K)], alpha)
        for k in range(K):
            joint *= _dm(X[lab == k].sum(0))
        assert abs(o.log_joint() - _log(joint)) <= 1e-13 * max(1.0, abs(_log(joint))), lab
        n += 1
    assert n == 877                                   # Bell(7)
