"""CPU oracle of the sample-side validation statistics (TEST INFRASTRUCTURE).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use
this module; it shares no code with the GPU library.

Click cumulants estimated from N samples (App. F, "Click cumulants, Pearson
and Spearman coefficients", Eq. cumulants_test_def): the population cumulant
  kappa~(S) = sum_{pi in P(S)} w(pi) prod_{B in pi} mu(B),  w(pi) = (-1)^(|pi|-1) (|pi|-1)!
with mu(B) the probability that every mode of B clicks.  The paper estimates
it without bias (k-statistics); this module uses the U-statistic form of that
estimator: every product of |pi| expectations is replaced by its average over
ordered tuples of |pi| distinct samples,
  U_pi = (1 / (N)_p) sum_{s_1 .. s_p distinct} prod_j X_{B_j}(s_j),   p = |pi|,
X_B(s) = prod_{k in B} x_k(s), (N)_p = N (N-1) ... (N-p+1), so that E[U_pi] =
prod_j mu(B_j) for independent samples and E[k(S)] = kappa~(S).  The sum over
distinct tuples follows from power sums s_B = sum_s X_B(s) (the number of
samples in which all of B clicked) by Moebius inversion on the lattice of
partitions of the p blocks:
  sum_{distinct} prod_j f_j(s_j) = sum_{sigma in P([p])} prod_{C in sigma}
                                     (-1)^(|C|-1) (|C|-1)! sum_s prod_{j in C} f_j(s).
Everything here is exact rational arithmetic (fractions) until the final
conversion to float.

The Pearson coefficient (Eq. pearson_correlation) is written out in FP64 with
compensated sums.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

from . import colex_rank, order_offset, set_partitions, subsets_colex


def power_sum(bits: np.ndarray, B) -> int:
    """s_B: the number of samples in which every mode of B clicked."""
    if len(B) == 0:
        return len(bits)
    return int(np.count_nonzero(np.all(bits[:, list(B)] == 1, axis=1)))


def falling(N: int, p: int) -> int:
    out = 1
    for i in range(p):
        out *= N - i
    return out


def lattice_mobius(sigma) -> int:
    """prod_{C in sigma} (-1)^(|C|-1) (|C|-1)!"""
    out = 1
    for C in sigma:
        out *= (-1) ** (len(C) - 1) * math.factorial(len(C) - 1)
    return out


def u_statistic(bits: np.ndarray, blocks, counts=None) -> Fraction:
    """U_pi for the blocks of pi (tuples of modes), exactly."""
    p = len(blocks)
    N = len(bits)
    s = counts or (lambda B: power_sum(bits, B))
    total = 0
    for sigma in set_partitions(p):
        term = lattice_mobius(sigma)
        for C in sigma:
            union = tuple(sorted(set().union(*(blocks[j] for j in C))))
            term *= s(union)
        total += term
    return Fraction(total, falling(N, p))


def k_statistic(bits: np.ndarray, S, counts=None) -> Fraction:
    """Unbiased estimate of the click cumulant kappa~(S) from the samples."""
    S = tuple(sorted(S))
    total = Fraction(0)
    for pi in set_partitions(len(S)):
        blocks = [tuple(S[k] for k in b) for b in pi]
        w = (-1) ** (len(pi) - 1) * math.factorial(len(pi) - 1)
        total += w * u_statistic(bits, blocks, counts)
    return total


def u_statistic_literal(bits: np.ndarray, blocks) -> Fraction:
    """U_pi by its definition: the average over all ordered tuples of distinct
    samples (tiny N only)."""
    N = len(bits)
    p = len(blocks)
    total = 0
    for tup in itertools.permutations(range(N), p):
        prod = 1
        for j, s in enumerate(tup):
            prod *= int(np.all(bits[s, list(blocks[j])] == 1))
        total += prod
    return Fraction(total, falling(N, p))


def sample_cumulants(bits: np.ndarray, K: int, last_ranks=None) -> np.ndarray:
    """k(S) for all S of orders 1..K-1 and, at order K, all subsets or those
    with the given colex ranks (in that order): the library's layout."""
    bits = np.asarray(bits, dtype=np.uint8)
    M = bits.shape[1]
    cache = {}

    def counts(B):
        if B not in cache:
            cache[B] = power_sum(bits, B)
        return cache[B]

    out = []
    for d in range(1, K + 1):
        if d == K and last_ranks is not None:
            from . import colex_unrank
            subsets = [colex_unrank(d, int(r)) for r in last_ranks]
        else:
            subsets = subsets_colex(M, d)
        for S in subsets:
            out.append(float(k_statistic(bits, S, counts)))
    return np.array(out)


def pearson(x, y) -> float:
    """Eq. pearson_correlation: centered cross and square sums."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mx = math.fsum(x) / len(x)
    my = math.fsum(y) / len(y)
    sxy = math.fsum((x - mx) * (y - my))
    sxx = math.fsum((x - mx) ** 2)
    syy = math.fsum((y - my) ** 2)
    return sxy / math.sqrt(sxx * syy)
