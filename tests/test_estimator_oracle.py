"""Pins for the sample-statistics oracle (oracle/estimators.py): the unbiased
click-cumulant estimator and the Pearson coefficient of App. F.

References: textbook unbiased estimators for orders 1-3 (sample mean,
covariance with N - 1, third central co-moment with N / ((N-1)(N-2))); the
literal average over tuples of distinct samples; exact expectations over every
data set of a small distribution (unbiasedness, in rational arithmetic); and
numpy's correlation coefficient.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import estimators as E


def _bits(N, M, seed, p=0.4):
    rng = np.random.default_rng(seed)
    base = rng.random((N, 1)) < 0.3  # a shared cause makes the bits correlated
    return ((rng.random((N, M)) < p) | (base & (rng.random((N, M)) < 0.5))).astype(np.uint8)


def test_order_one_is_the_sample_mean():
    b = _bits(50, 4, 1)
    for a in range(4):
        assert float(E.k_statistic(b, (a,))) == pytest.approx(b[:, a].mean(), abs=1e-15)


def test_order_two_is_the_unbiased_covariance():
    b = _bits(60, 4, 2)
    for a, c in itertools.combinations(range(4), 2):
        ref = np.cov(b[:, a].astype(float), b[:, c].astype(float), ddof=1)[0, 1]
        assert float(E.k_statistic(b, (a, c))) == pytest.approx(ref, abs=1e-15)


def test_order_three_is_the_unbiased_third_comoment():
    b = _bits(40, 5, 3).astype(float)
    N = len(b)
    for S in itertools.combinations(range(5), 3):
        d = [b[:, k] - b[:, k].mean() for k in S]
        ref = N / ((N - 1) * (N - 2)) * float(np.sum(d[0] * d[1] * d[2]))
        assert float(E.k_statistic(b.astype(np.uint8), S)) == pytest.approx(ref, abs=1e-14)


@pytest.mark.parametrize("S", [(0, 1), (0, 1, 2), (0, 1, 2, 3), (1, 2, 3, 4)])
def test_power_sum_form_matches_distinct_tuple_average(S):
    b = _bits(7, 5, 4, p=0.5)
    for pi in O.set_partitions(len(S)):
        blocks = [tuple(S[k] for k in blk) for blk in pi]
        if len(blocks) > 7:
            continue
        assert E.u_statistic(b, blocks) == E.u_statistic_literal(b, blocks)


def _exact_cumulant(probs, M, S):
    """kappa~(S) of an explicit distribution over {0,1}^M (rational)."""
    def mu(B):
        return sum((pr for x, pr in enumerate(probs) if all((x >> k) & 1 for k in B)), Fraction(0))
    total = Fraction(0)
    for pi in O.set_partitions(len(S)):
        term = Fraction((-1) ** (len(pi) - 1) * math.factorial(len(pi) - 1))
        for blk in pi:
            term *= mu([S[k] for k in blk])
        total += term
    return total


@pytest.mark.parametrize("M,N", [(3, 3), (4, 4)])
def test_unbiased_over_every_data_set(M, N):
    """E[k(S)] over all data sets of N independent samples equals kappa~(S)."""
    rng = np.random.default_rng(10 + M)
    w = rng.integers(1, 9, size=1 << M)
    probs = [Fraction(int(v), int(w.sum())) for v in w]
    S = tuple(range(M))
    expect = Fraction(0)
    outcomes = range(1 << M)
    for multiset in itertools.combinations_with_replacement(outcomes, N):
        counts = np.bincount(multiset, minlength=1 << M)
        weight = Fraction(math.factorial(N))
        for x, c in enumerate(counts):
            weight *= probs[x] ** int(c) / math.factorial(int(c))
        bits = np.array([[(x >> k) & 1 for k in range(M)] for x in multiset], dtype=np.uint8)
        expect += weight * E.k_statistic(bits, S)
    assert expect == _exact_cumulant(probs, M, S)


def test_sample_cumulant_layout():
    b = _bits(30, 6, 5)
    full = E.sample_cumulants(b, 3)
    assert len(full) == O.total_outputs(6, 3)
    ranks = np.array([0, 7, 19])
    part = E.sample_cumulants(b, 3, last_ranks=ranks)
    off = O.order_offset(6, 3)
    assert np.array_equal(part[:off], full[:off])
    assert np.array_equal(part[off:], full[off + ranks])


def test_pearson():
    rng = np.random.default_rng(6)
    x = rng.normal(size=500)
    y = 0.3 * x + rng.normal(size=500)
    assert E.pearson(x, y) == pytest.approx(np.corrcoef(x, y)[0, 1], abs=1e-14)
    assert E.pearson(x, 2.5 * x - 1.0) == pytest.approx(1.0, abs=1e-14)
    assert E.pearson(x, -0.5 * x + 3.0) == pytest.approx(-1.0, abs=1e-14)
    assert E.pearson(x, y) == pytest.approx(E.pearson(y, x), abs=1e-15)


def _battery():
    ok = []
    b = _bits(60, 4, 2)
    for a, c in itertools.combinations(range(4), 2):
        ref = np.cov(b[:, a].astype(float), b[:, c].astype(float), ddof=1)[0, 1]
        ok.append(abs(float(E.k_statistic(b, (a, c))) - ref) < 1e-15)
    b7 = _bits(7, 5, 4, p=0.5)
    for pi in O.set_partitions(3):
        blocks = [tuple((0, 1, 2)[k] for k in blk) for blk in pi]
        ok.append(E.u_statistic(b7, blocks) == E.u_statistic_literal(b7, blocks))
    return all(ok)


@pytest.mark.parametrize("mutation", ["power", "mobius_sign", "weight_sign"])
def test_planted_mistakes_are_caught(mutation, monkeypatch):
    if mutation == "power":
        monkeypatch.setattr(E, "falling", lambda N, p: N ** p)
    elif mutation == "mobius_sign":
        monkeypatch.setattr(E, "lattice_mobius",
                            lambda sigma: math.prod(math.factorial(len(C) - 1) for C in sigma))
    else:
        orig = E.k_statistic

        def k(bits, S, counts=None):
            S = tuple(sorted(S))
            total = Fraction(0)
            for pi in O.set_partitions(len(S)):
                blocks = [tuple(S[i] for i in blk) for blk in pi]
                total += math.factorial(len(pi) - 1) * E.u_statistic(bits, blocks, counts)
            return total
        monkeypatch.setattr(E, "k_statistic", k)
    assert not _battery()
