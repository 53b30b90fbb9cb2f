"""Planted mistakes: each mutation of the oracle (a dropped term, a wrong sign, a
wrong index, a transposed operand, a missing vacuum term) must make at least one
pin of the battery below fail.  Mutations are applied to the oracle on the CPU
with monkeypatch and undone after each case."""
import math

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O


def _pin_single_mode():
    r, eta = 0.9, 0.6
    sigma = G.product_state_covariance(np.array([r]), np.array([eta]))
    det = (1 - eta * (1 - math.exp(-2 * r)) / 2) * (1 + eta * (math.exp(2 * r) - 1) / 2)
    corr, _ = O.correlators_and_cumulants(sigma, 1)
    return abs(corr[0] - (1 - det ** -0.5)) < 1e-12


def _pin_product_state():
    sigma = G.product_state_covariance(np.array([0.5, 1.0, 0.7]), np.array([0.4, 0.8, 0.6]))
    corr, cum = O.correlators_and_cumulants(sigma, 3)
    ok = np.all(np.abs(cum[3:]) < 1e-14)
    ok &= abs(corr[-1] - corr[0] * corr[1] * corr[2]) < 1e-14
    return bool(ok)


def _pin_tmsv():
    r = 0.7
    sigma = G.tmsv_covariance(r, M=3, i=0, j=2)
    corr, cum = O.correlators_and_cumulants(sigma, 2)
    t2 = math.tanh(r) ** 2
    i02 = 3 + O.colex_rank((0, 2))
    return abs(corr[i02] - t2) < 1e-12 and abs(cum[i02] - t2 / math.cosh(r) ** 2) < 1e-12


_BRUTE = {}


def _pin_brute_force():
    inst = G.make_instance("m16_k3", M=4, seed=3)
    if "p" not in _BRUTE:
        _BRUTE["p"] = O.pattern_probabilities(inst.sigma)
    probs = _BRUTE["p"]
    corr, _ = O.correlators_and_cumulants(inst.sigma, 4)
    pos = 0
    for d in range(1, 5):
        for S in O.subsets_colex(4, d):
            mask = sum(1 << k for k in S)
            ref = sum(probs[x] for x in range(16) if x & mask == mask)
            if abs(corr[pos] - ref) > 1e-11:
                return False
            pos += 1
    return True


def _pin_roundtrip():
    inst = G.make_instance("m16_k3", M=5, seed=8)
    corr, cum = O.correlators_and_cumulants(inst.sigma, 4)
    m, k = {}, {}
    pos = 0
    for d in range(1, 5):
        for S in O.subsets_colex(5, d):
            m[S], k[S] = corr[pos], cum[pos]
            pos += 1
    for S in m:
        tot = sum(math.prod(k[tuple(S[i] for i in b)] for b in pi) for pi in O.set_partitions(len(S)))
        if abs(tot - m[S]) > 1e-12:
            return False
    return True


def _pin_phase_rotation():
    inst = G.make_instance("m16_k3", M=4, seed=6)
    rot = G.local_phase_rotation(inst.sigma, np.array([0.3, 1.9, 2.5, 4.0]))
    a = O.correlators_and_cumulants(inst.sigma, 3)
    b = O.correlators_and_cumulants(rot, 3)
    return bool(np.allclose(a[0], b[0], rtol=1e-10, atol=1e-14))


BATTERY = [_pin_single_mode, _pin_product_state, _pin_tmsv, _pin_brute_force, _pin_roundtrip,
           _pin_phase_rotation]


def test_battery_passes_unmutated():
    assert all(pin() for pin in BATTERY)


def _mut_weight_sign(mp):
    mp.setattr(O, "partition_weight", lambda nb: math.factorial(nb - 1))


def _mut_weight_factorial(mp):
    mp.setattr(O, "partition_weight", lambda nb: (-1) ** (nb - 1) * nb)


def _mut_drop_full_term(mp):
    orig = O.all_subsets

    def drop(S):
        S = tuple(S)
        for T in orig(S):
            if len(S) > 1 and len(T) == len(S):
                continue
            yield T
    mp.setattr(O, "all_subsets", drop)


def _mut_inclusion_sign(mp):
    def wrong(Q, S, p=None):
        p = p or (lambda T: O.vacuum_probability(Q, T))
        return math.fsum((-1) ** (len(T) + 1) * p(T) for T in O.all_subsets(tuple(S))) + 0.0
    mp.setattr(O, "click_correlator", wrong)


def _mut_wrong_index(mp):
    def block(Q, T):
        M = Q.shape[0] // 2
        idx = [t for t in T] + [(t + M + 1) % (2 * M) for t in T]
        return Q[np.ix_(idx, idx)]
    mp.setattr(O, "principal_block", block)


def _mut_transposed_block(mp):
    def block(Q, T):
        M = Q.shape[0] // 2
        xi = [t for t in T]
        pi = [t + M for t in T]
        A = Q[np.ix_(xi + pi, xi + pi)].copy()
        n = len(T)
        A[:n, n:] = A[:n, n:].T  # x-p coupling block transposed
        A[n:, :n] = A[:n, n:].T
        return A
    mp.setattr(O, "principal_block", block)


def _mut_missing_vacuum(mp):
    mp.setattr(O, "q_matrix", lambda s: np.asarray(s, dtype=np.float64) + 0.25 * np.eye(s.shape[0]))


def _mut_sqrt_missing(mp):
    def vp(Q, T):
        if len(T) == 0:
            return 1.0
        L = np.linalg.cholesky(O.principal_block(Q, T))
        return 1.0 / float(np.prod(np.diag(L))) ** 2
    mp.setattr(O, "vacuum_probability", vp)


def _mut_partition_drop_singletons(mp):
    orig = O.set_partitions

    def parts(n):
        out = orig(n)
        return tuple(pi for pi in out if not (n > 2 and len(pi) == n))
    mp.setattr(O, "set_partitions", parts)


MUTATIONS = [_mut_weight_sign, _mut_weight_factorial, _mut_drop_full_term, _mut_inclusion_sign,
             _mut_wrong_index, _mut_transposed_block, _mut_missing_vacuum, _mut_sqrt_missing,
             _mut_partition_drop_singletons]


@pytest.mark.parametrize("mutation", MUTATIONS, ids=lambda f: f.__name__)
def test_mutation_is_caught(mutation, monkeypatch):
    mutation(monkeypatch)
    results = []
    for pin in BATTERY:
        try:
            results.append(bool(pin()))
        except (AssertionError, np.linalg.LinAlgError, ValueError, ZeroDivisionError):
            results.append(False)
    assert not all(results), f"no pin caught {mutation.__name__}"
