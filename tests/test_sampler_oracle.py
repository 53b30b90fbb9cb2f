"""Pins for the sampler oracle (oracle/sampler.py): the chain-rule sampler of
Sec. II with the single-elision (K = 3, Methods) and double-elision (K = 5,
App. C.1) marginal approximations.

Nothing here checks the oracle against itself.  The references are:
* the Torontonian pattern probabilities (App. F, independent of cumulants)
  for Gaussian states small enough that the expansion and every marginal the
  method uses are exact (M <= 3 single, M <= 5 double);
* closed-form distributions of independent consecutive bit pairs, for which
  every cumulant of order >= 3 vanishes and every product of marginals the
  method forms factorises exactly, at any M;
* the exact conditionals of those distributions, and a chi-square test of
  sampled frequencies.
"""
import itertools
import math

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from oracle import sampler as S


def _gauss(M, seed):
    inst = G.make_instance("m144_k5", M=M, seed=seed)
    _, cum = O.correlators_and_cumulants(inst.sigma, M, O.PARITY)
    return inst.sigma, cum


def _patterns(M):
    for x in range(1 << M):
        yield x, [(x >> k) & 1 for k in range(M)]


@pytest.mark.parametrize("method,M", [(S.SINGLE, 2), (S.SINGLE, 3), (S.DOUBLE, 2),
                                      (S.DOUBLE, 3), (S.DOUBLE, 4), (S.DOUBLE, 5)])
def test_exact_for_small_gaussian_states(method, M):
    sigma, cum = _gauss(M, 11 + M)
    ref = O.pattern_probabilities(sigma)
    for x, bits in _patterns(M):
        assert abs(S.pattern_probability(cum, M, method, bits) - ref[x]) < 1e-13


@pytest.mark.parametrize("method,M", [(S.SINGLE, 4), (S.DOUBLE, 6)])
def test_truncation_error_is_small_but_present(method, M):
    """One mode beyond the exact range, the truncated expansion (order K) and
    the factorised marginals are approximations: close, not equal."""
    sigma, cum = _gauss(M, 31)
    ref = O.pattern_probabilities(sigma)
    err = max(abs(S.pattern_probability(cum, M, method, bits) - ref[x])
              for x, bits in _patterns(M))
    assert 1e-8 < err < 1e-2


def _pair_distribution(M, seed):
    """Independent consecutive pairs (1,2), (3,4), ... (a single last bit when M
    is odd), each with a random joint distribution."""
    rng = np.random.default_rng(seed)
    blocks, k = [], 0
    while k < M:
        size = 2 if k + 1 < M else 1
        blocks.append((list(range(k, k + size)), rng.dirichlet(np.full(1 << size, 2.0))))
        k += size
    return blocks


def _block_prob(blocks, bits):
    p = 1.0
    for modes, w in blocks:
        p *= w[sum(bits[m] << i for i, m in enumerate(modes))]
    return p


def _block_cumulants(blocks, M, K):
    """Parity cumulants of the pair distribution in closed form: E[z_k] for
    single bits, Cov(z_k, z_k') within a pair (z = (-1)^x), zero otherwise."""
    cum = np.zeros(O.total_outputs(M, K))
    for modes, w in blocks:
        def ez(sub):
            return sum(w[i] * math.prod(-1.0 if (i >> s) & 1 else 1.0 for s in sub)
                       for i in range(len(w)))
        for i, m in enumerate(modes):
            cum[O.order_offset(M, 1) + O.colex_rank((m,))] = ez([i])
        if len(modes) == 2:
            cum[O.order_offset(M, 2) + O.colex_rank(tuple(modes))] = ez([0, 1]) - ez([0]) * ez([1])
    return cum


@pytest.mark.parametrize("method", [S.SINGLE, S.DOUBLE])
@pytest.mark.parametrize("M", [6, 7, 8])
def test_exact_for_independent_pairs(method, M):
    blocks = _pair_distribution(M, 100 + M)
    cum = _block_cumulants(blocks, M, method)
    total = []
    for x, bits in _patterns(M):
        p = S.pattern_probability(cum, M, method, bits)
        assert abs(p - _block_prob(blocks, bits)) < 1e-15
        total.append(p)
    assert abs(math.fsum(total) - 1.0) < 1e-14


@pytest.mark.parametrize("method", [S.SINGLE, S.DOUBLE])
def test_conditionals_of_independent_pairs(method):
    M = 7
    blocks = _pair_distribution(M, 77)
    cum = _block_cumulants(blocks, M, method)
    rng = np.random.default_rng(5)
    for _ in range(10):
        bits = list(rng.integers(0, 2, size=M))
        _, cond, _ = S.sample(cum, M, method, forced=bits)
        for n in range(M):
            prev = bits[:n]
            num = sum(_block_prob(blocks, prev + [1] + list(rest))
                      for rest in itertools.product([0, 1], repeat=M - n - 1))
            den = sum(_block_prob(blocks, prev + list(rest))
                      for rest in itertools.product([0, 1], repeat=M - n))
            assert abs(cond[n] - num / den) < 1e-13


def test_sampled_frequencies_follow_the_distribution():
    """Chi-square goodness of fit of 4000 samples (single elision, M = 4, a
    distribution it represents exactly)."""
    M = 4
    blocks = _pair_distribution(M, 9)
    cum = _block_cumulants(blocks, M, S.SINGLE)
    u = np.random.default_rng(12).random((4000, M))
    counts = np.zeros(1 << M)
    for row in u:
        bits, _, _ = S.sample(cum, M, S.SINGLE, u=row)
        counts[sum(int(b) << k for k, b in enumerate(bits))] += 1
    expect = np.array([_block_prob(blocks, [(x >> k) & 1 for k in range(M)]) for x in range(1 << M)])
    expect *= len(u)
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    from scipy.stats import chi2 as dist
    assert dist.sf(chi2, (1 << M) - 1) > 1e-3


def test_decision_rule():
    """x_n = 1 exactly when u_n < p(x_n = 1 | x_<n)."""
    M = 6
    sigma, cum = _gauss(M, 3)
    _, cum5 = O.correlators_and_cumulants(sigma, 5, O.PARITY)
    rng = np.random.default_rng(4)
    for _ in range(20):
        u = rng.random(M)
        bits, cond, p = S.sample(cum5, M, S.DOUBLE, u=u)
        assert np.array_equal(bits, (u < cond).astype(np.uint8))
        assert 0.0 < p < 1.0


# ---------------------------------------------------------------------------
# planted mistakes: each must make the battery below fail


def _battery():
    ok = []
    for method, M in ((S.SINGLE, 3), (S.DOUBLE, 5)):
        sigma, cum = _gauss(M, 11 + M)
        ref = O.pattern_probabilities(sigma)
        ok.append(all(abs(S.pattern_probability(cum, M, method, bits) - ref[x]) < 1e-13
                      for x, bits in _patterns(M)))
    for method in (S.SINGLE, S.DOUBLE):
        blocks = _pair_distribution(7, 107)
        cum = _block_cumulants(blocks, 7, method)
        ok.append(all(abs(S.pattern_probability(cum, 7, method, bits) - _block_prob(blocks, bits))
                      < 1e-15 for x, bits in _patterns(7)))
    return ok


def _run(mut, monkeypatch):
    mut(monkeypatch)
    try:
        return all(_battery())
    except (AssertionError, KeyError, IndexError, ZeroDivisionError):
        return False


def test_battery_passes_unmutated():
    assert all(_battery())


def _drop_parity(mp):
    mp.setattr(S._Step, "gamma", lambda self, *b: self.kap(*b))


def _drop_order(k):
    def mut(mp):
        orig = S._Step.gamma
        mp.setattr(S._Step, "gamma", lambda self, *b: 0.0 if len(b) == k else orig(self, *b))
    mut.__name__ = f"_drop_order_{k}"
    return mut


def _mode_shift(mp):
    orig = S.kappa_lookup

    def look(cum, M, K):
        kap = orig(cum, M, K)
        return lambda *bits: kap(*[(b % M) + 1 for b in bits])
    mp.setattr(S, "kappa_lookup", look)


def _top_elision_wrong(mp):
    orig = S._Tables.p1
    mp.setattr(S._Tables, "p1", lambda self, a, e: self.p(a) if e == a else orig(self, a, e))


def _empty_partial_zero(mp):
    orig = S._Tables.pp
    mp.setattr(S._Tables, "pp", lambda self, b, a: 0.0 if b < a else orig(self, b, a))


def _ord_increasing(mp):
    mp.setattr(S, "_ord", lambda *idx: tuple(sorted(idx)))


def _conditional_undivided(mp):
    mp.setattr(S, "conditional_one", lambda p_one, p_prev: p_one)


MUTATIONS = [_drop_parity, _drop_order(2), _drop_order(3), _drop_order(4), _drop_order(5),
             _mode_shift, _top_elision_wrong, _empty_partial_zero, _ord_increasing]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=lambda f: f.__name__)
def test_mutation_is_caught(mutation, monkeypatch):
    assert not _run(mutation, monkeypatch), f"no pin caught {mutation.__name__}"


def test_conditional_mutation_is_caught(monkeypatch):
    _conditional_undivided(monkeypatch)
    blocks = _pair_distribution(5, 3)
    cum = _block_cumulants(blocks, 5, S.SINGLE)
    bits = [1, 0, 1, 1, 0]
    _, cond, _ = S.sample(cum, 5, S.SINGLE, forced=bits)
    exact = []
    for n in range(5):
        prev = bits[:n]
        num = sum(_block_prob(blocks, prev + [1] + list(r))
                  for r in itertools.product([0, 1], repeat=4 - n))
        den = sum(_block_prob(blocks, prev + list(r)) for r in itertools.product([0, 1], repeat=5 - n))
        exact.append(num / den)
    assert not np.allclose(cond, exact, rtol=0, atol=1e-13)


@pytest.mark.parametrize("method,M", [(S.SINGLE, 10), (S.DOUBLE, 9)])
def test_c_tier_matches_python(c_oracle, method, M):
    inst = G.make_instance("m144_k5", M=M, seed=19)
    _, cum = O.correlators_and_cumulants(inst.sigma, method, O.PARITY)
    u = np.random.default_rng(8).random((M, 5))
    bits, prob, cond = S.c_sample(cum, M, method, u=u)
    for s in range(5):
        b, c, p = S.sample(cum, M, method, u=u[:, s])
        assert np.array_equal(b, bits[s])
        assert np.allclose(c, cond[:, s], rtol=1e-13, atol=1e-15)
        assert abs(p - prob[s]) <= 1e-13 * p
    fb, fprob, fcond = S.c_sample(cum, M, method, forced=bits)
    assert np.array_equal(fb, bits) and np.array_equal(fprob, prob)
