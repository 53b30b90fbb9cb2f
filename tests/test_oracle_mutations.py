"""Planted mistakes: each mutation of the oracle (a dropped term, a wrong sign, a
wrong index, a transposed operand, a missing vacuum term) must make at least one
pin of the battery below fail.  Mutations are applied to the oracle on the CPU
with monkeypatch and undone after each case."""
import math

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from fock import FockState, fock_cumulant, two_mode_state


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
    def vp(Q, T, mu=None):
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


def _run_battery(battery):
    results = []
    for pin in battery:
        try:
            results.append(bool(pin()))
        except (AssertionError, np.linalg.LinAlgError, ValueError, ZeroDivisionError):
            results.append(False)
    return results


@pytest.mark.parametrize("mutation", MUTATIONS, ids=lambda f: f.__name__)
def test_mutation_is_caught(mutation, monkeypatch):
    mutation(monkeypatch)
    assert not all(_run_battery(BATTERY)), f"no pin caught {mutation.__name__}"


# ---------------------------------------------------------------------------
# displaced states (Eq. vacuum_gaussian_prob with mu != 0)


def _pin_coherent_product():
    M = 4
    rng = np.random.default_rng(5)
    U = G.haar_unitary(M, rng)
    alpha = rng.normal(size=M) + 1j * rng.normal(size=M)
    mu = G.interferometer_symplectic(U) @ (math.sqrt(2.0) * np.concatenate([alpha.real, alpha.imag]))
    corr, cum = O.correlators_and_cumulants(G.vacuum_covariance(M), 3, O.CLICK, mu)
    f = 1.0 - np.exp(-np.abs(U @ alpha) ** 2)
    ok = np.all(np.abs(cum[M:]) < 1e-13)
    ok &= np.allclose(corr[:M], f, rtol=0, atol=1e-13)
    return bool(ok)


def _pin_fock_single():
    st = FockState(1, 100)
    st.squeeze(0, 0.6)
    st.displace(0, 0.7 - 0.6j)
    sigma, mu = st.moments()
    corr, _ = O.correlators_and_cumulants(sigma, 1, O.CLICK, mu)
    return abs(corr[0] - st.click_correlator((0,))) < 1e-12


_FOCK = {}


def _pin_fock_two_mode():
    if "st" not in _FOCK:
        _FOCK["st"] = two_mode_state()
    st = _FOCK["st"]
    sigma, mu = st.moments()
    corr, cum = O.correlators_and_cumulants(sigma, 2, O.CLICK, mu)
    pos = 0
    for d in (1, 2):
        for S in O.subsets_colex(2, d):
            if abs(corr[pos] - st.click_correlator(S)) > 1e-12:
                return False
            if abs(cum[pos] - fock_cumulant(S, st.click_correlator)) > 1e-12:
                return False
            pos += 1
    return True


BATTERY_DISPLACED = [_pin_coherent_product, _pin_fock_single, _pin_fock_two_mode]


def test_displaced_battery_passes_unmutated():
    assert all(_run_battery(BATTERY_DISPLACED))


def _mut_mean_xp_swapped(mp):
    def pm(mu, T):
        M = len(mu) // 2
        return np.asarray(mu)[[t + M for t in T] + [t for t in T]]
    mp.setattr(O, "principal_mean", pm)


def _mut_mean_wrong_mode(mp):
    def pm(mu, T):
        M = len(mu) // 2
        return np.asarray(mu)[[(t + 1) % M for t in T] + [(t + 1) % M + M for t in T]]
    mp.setattr(O, "principal_mean", pm)


def _mut_mean_missing_half(mp):
    orig = O.mean_quadratic_form
    mp.setattr(O, "mean_quadratic_form", lambda Q, mu, T: 2.0 * orig(Q, mu, T))


def _mut_mean_sign(mp):
    orig = O.mean_quadratic_form
    mp.setattr(O, "mean_quadratic_form", lambda Q, mu, T: -orig(Q, mu, T))


def _mut_mean_uses_sigma(mp):
    def qf(Q, mu, T):
        m = O.principal_mean(mu, T)
        A = O.principal_block(Q, T) - 0.5 * np.eye(2 * len(T))
        return float(m @ np.linalg.solve(A, m))
    mp.setattr(O, "mean_quadratic_form", qf)


def _mut_mean_diagonal_only(mp):
    def qf(Q, mu, T):
        m = O.principal_mean(mu, T)
        return float(np.sum(m * m / np.diag(O.principal_block(Q, T))))
    mp.setattr(O, "mean_quadratic_form", qf)


def _mut_mean_not_inverted(mp):
    def qf(Q, mu, T):
        m = O.principal_mean(mu, T)
        return float(m @ O.principal_block(Q, T) @ m)
    mp.setattr(O, "mean_quadratic_form", qf)


MUTATIONS_DISPLACED = [_mut_mean_xp_swapped, _mut_mean_wrong_mode, _mut_mean_missing_half,
                       _mut_mean_sign, _mut_mean_uses_sigma, _mut_mean_diagonal_only,
                       _mut_mean_not_inverted]


@pytest.mark.parametrize("mutation", MUTATIONS_DISPLACED, ids=lambda f: f.__name__)
def test_displaced_mutation_is_caught(mutation, monkeypatch):
    mutation(monkeypatch)
    assert not all(_run_battery(BATTERY_DISPLACED)), f"no pin caught {mutation.__name__}"
