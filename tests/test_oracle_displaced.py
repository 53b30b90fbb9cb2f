"""Pins for the displaced-state oracle (first moments mu != 0; App. D.1, Eq.
vacuum_gaussian_prob with hbar = 1).

The references here do not use the Gaussian formula at all: small pure states
are prepared in a truncated Fock basis by exponentiating the generators of
displacement, squeezing and beam-splitter gates; their first and second
quadrature moments give (sigma, mu), and the vacuum, click and parity
probabilities are summed directly from the Fock amplitudes.  A coherent
product state adds a closed form, and the high-precision arbiter, the C tier
and the zero-mean case tie the rest together.
"""
import math

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from fock import FockState, fock_cumulant, three_mode_state, two_mode_state


@pytest.fixture(scope="module")
def two_mode():
    st = two_mode_state()
    assert st.tail_weight() < 1e-15
    return st


@pytest.fixture(scope="module")
def three_mode():
    st = three_mode_state()
    assert st.tail_weight() < 1e-14
    return st


# ---------------------------------------------------------------------------
# closed form: coherent product states


def test_coherent_product_state_closed_form():
    # sigma = I/2 (every mode coherent, also after a passive interferometer):
    # p(T) = exp(-sum_{k in T} |beta_k|^2), |beta_k|^2 = (mu_k^2 + mu_{k+M}^2)/2,
    # so click correlators factorise as prod (1 - e^{-|beta_k|^2}), parity
    # correlators as prod (2 e^{-|beta_k|^2} - 1), and every cumulant of order >= 2
    # vanishes.
    M = 6
    rng = np.random.default_rng(11)
    U = G.haar_unitary(M, rng)
    alpha = rng.normal(size=M) + 1j * rng.normal(size=M)
    mu_in = math.sqrt(2.0) * np.concatenate([alpha.real, alpha.imag])
    mu = G.interferometer_symplectic(U) @ mu_in
    sigma = G.vacuum_covariance(M)
    beta2 = np.abs(U @ alpha) ** 2
    assert np.allclose(beta2, 0.5 * (mu[:M] ** 2 + mu[M:] ** 2))
    p1 = np.exp(-beta2)
    for conv, f in ((O.CLICK, 1.0 - p1), (O.PARITY, 2.0 * p1 - 1.0)):
        corr, cum = O.correlators_and_cumulants(sigma, 4, conv, mu)
        pos = 0
        for d in range(1, 5):
            for S in O.subsets_colex(M, d):
                ref = float(np.prod(f[list(S)]))
                assert abs(corr[pos] - ref) < 1e-14
                if d == 1:
                    assert abs(cum[pos] - ref) < 1e-14
                else:
                    assert abs(cum[pos]) < 1e-14
                pos += 1


# ---------------------------------------------------------------------------
# Fock-basis references


@pytest.mark.parametrize("r,alpha", [(0.5, 0.8 + 0.3j), (-0.7, -0.2 + 0.9j), (0.0, 1.2 - 0.5j),
                                     (0.8, 0.0)])
def test_single_mode_displaced_squeezed_vacuum(r, alpha):
    st = FockState(1, 120)
    st.squeeze(0, r)
    st.displace(0, alpha)
    assert st.tail_weight() < 1e-16
    sigma, mu = st.moments()
    Q = O.q_matrix(sigma)
    assert abs(O.vacuum_probability(Q, (0,), mu) - st.vacuum_probability((0,))) < 1e-13
    corr, _ = O.correlators_and_cumulants(sigma, 1, O.CLICK, mu)
    assert abs(corr[0] - st.click_correlator((0,))) < 1e-13


def test_two_mode_vacuum_probabilities(two_mode):
    sigma, mu = two_mode.moments()
    assert abs(mu).min() > 0.05 and abs(sigma[0, 1]) > 0.05 and abs(sigma[0, 3]) > 0.01
    Q = O.q_matrix(sigma)
    for T in [(0,), (1,), (0, 1)]:
        assert abs(O.vacuum_probability(Q, T, mu) - two_mode.vacuum_probability(T)) < 1e-13


@pytest.mark.parametrize("conv", [O.CLICK, O.PARITY])
def test_two_mode_correlators_and_cumulants(two_mode, conv):
    sigma, mu = two_mode.moments()
    corr, cum = O.correlators_and_cumulants(sigma, 2, conv, mu)
    fock = two_mode.click_correlator if conv == O.CLICK else two_mode.parity_correlator
    pos = 0
    for d in (1, 2):
        for S in O.subsets_colex(2, d):
            assert abs(corr[pos] - fock(S)) < 1e-12
            assert abs(cum[pos] - fock_cumulant(S, fock)) < 1e-12
            pos += 1
    assert abs(cum[2]) > 1e-3  # the state is correlated: a real check


@pytest.mark.parametrize("conv", [O.CLICK, O.PARITY])
def test_three_mode_correlators_and_cumulants(three_mode, conv):
    sigma, mu = three_mode.moments()
    corr, cum = O.correlators_and_cumulants(sigma, 3, conv, mu)
    fock = three_mode.click_correlator if conv == O.CLICK else three_mode.parity_correlator
    pos = 0
    for d in (1, 2, 3):
        for S in O.subsets_colex(3, d):
            assert abs(corr[pos] - fock(S)) < 1e-12, (S, corr[pos], fock(S))
            assert abs(cum[pos] - fock_cumulant(S, fock)) < 1e-12
            pos += 1
    assert abs(cum[-1]) > 1e-5


def test_displacement_changes_the_answer(three_mode):
    # the same covariance without the mean gives different probabilities, so
    # the Fock checks above really exercise the exponential factor
    sigma, mu = three_mode.moments()
    Q = O.q_matrix(sigma)
    for T in [(0,), (1, 2), (0, 1, 2)]:
        assert abs(O.vacuum_probability(Q, T) - three_mode.vacuum_probability(T)) > 1e-3


# ---------------------------------------------------------------------------
# invariances and cross-checks


def test_zero_mean_is_the_undisplaced_oracle():
    inst = G.make_instance("m16_k3", M=7, seed=5)
    a = O.correlators_and_cumulants(inst.sigma, 3)
    b = O.correlators_and_cumulants(inst.sigma, 3, O.CLICK, np.zeros(14))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_mean_sign_and_phase_rotation_invariance():
    # p(T) depends on mu only through a quadratic form (even in mu), and a
    # local phase rotation applied to both sigma and mu leaves every vacuum
    # probability unchanged
    inst = G.make_instance("m16_k3", M=5, seed=9)
    mu = G.input_displacement(inst, seed=3)
    base = O.correlators_and_cumulants(inst.sigma, 3, O.CLICK, mu)
    flip = O.correlators_and_cumulants(inst.sigma, 3, O.CLICK, -mu)
    assert np.allclose(base[0], flip[0], rtol=1e-13, atol=1e-15)
    theta = np.array([0.4, 2.2, 5.0, 1.3, 3.3])
    M = 5
    c, s = np.cos(theta), np.sin(theta)
    mu_rot = np.concatenate([c * mu[:M] - s * mu[M:], s * mu[:M] + c * mu[M:]])
    rot = O.correlators_and_cumulants(G.local_phase_rotation(inst.sigma, theta), 3, O.CLICK,
                                      mu_rot)
    assert np.allclose(base[0], rot[0], rtol=1e-10, atol=1e-14)
    assert np.allclose(base[1], rot[1], rtol=1e-8, atol=1e-14)


def test_displaced_oracle_against_high_precision_arbiter():
    inst = G.make_instance("m144_k5", M=12, seed=21)
    mu = G.input_displacement(inst, seed=22)
    for S in [(0,), (3, 7), (1, 5, 11), (0, 2, 4, 9), (2, 3, 6, 8, 10)]:
        for conv in (O.CLICK, O.PARITY):
            m, k = O.subset_values(inst.sigma, S, conv, mu)
            am, ak = O.arbiter_values(inst.sigma, S, conv, mu=mu)
            vmu, vk = O.c_error_floor(inst.sigma, len(S), [O.colex_rank(S)], conv, mu=mu)
            assert abs(m - am) <= 1e-12 * abs(am) + 64 * O.U64 * vmu[0]
            assert abs(k - ak) <= 1e-10 * abs(ak) + 64 * O.U64 * vk[0]


@pytest.mark.parametrize("conv", [O.CLICK, O.PARITY])
def test_c_oracle_displaced_matches_python(c_oracle, conv):
    inst = G.make_instance("m16_k3", M=9, seed=2)
    mu = G.input_displacement(inst, seed=7)
    a = O.correlators_and_cumulants(inst.sigma, 3, conv, mu)
    b = O.c_forward(inst.sigma, 3, conv, mu=mu)
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=1e-15)
    assert np.allclose(a[1], b[1], rtol=1e-10, atol=1e-15)
    ranks = np.array([0, 5, 17, 83])
    c = O.c_forward_sample(inst.sigma, 3, ranks, conv, mu=mu)
    off = O.order_offset(9, 3)
    assert np.array_equal(c[0], b[0][off + ranks]) and np.array_equal(c[1], b[1][off + ranks])
