"""Pins of the FP64 parity tolerance (tests/parity.py) against a 40-digit
evaluation of the same definitions.

At the M = 144, K = 5 workload, for every order and both conventions, on
sampled subsets:
* the FP64 oracle's own error against the 40-digit arbiter stays inside half
  of the stated tolerance 1e-10 max(|ref|, 1e-4 S_pi) + 4 u V, leaving the
  other half for a second FP64 evaluation (the GPU path) rounding the other
  way;
* the tolerance is not inflated: its median is at most SLACK times the largest
  error the arbiter measures, per order (the error floor used before, 64 u V
  alone, was about 6,000 times the measured error of the order-5 click
  cumulants and fails this);
* for weakly illuminated modes (click probabilities of a few percent) the
  partition-sum term alone is not a valid bound: the FP64 oracle misses it,
  and the carried-in term 4 u V restores it;
* the scales the C oracle reports equal the Python tier's.
"""
import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from parity import fp64_scales, fp64_tolerance

pytestmark = pytest.mark.skipif(not O.c_oracle_available(), reason="C oracle not built")

U = 2.0 ** -53
SLACK = 1000.0
NSAMPLE = 16


@pytest.fixture(scope="module")
def inst():
    return G.make_instance("m144_k5")


def _arbiter(sigma, d, ranks, conv, mu=None):
    return np.array([O.arbiter_values(sigma, O.colex_unrank(d, int(r)), conv, mu=mu)
                     for r in ranks])


@pytest.mark.parametrize("d", [2, 3, 4, 5])
@pytest.mark.parametrize("conv", [O.CLICK, O.PARITY], ids=["click", "parity"])
def test_tolerance_against_arbiter(inst, conv, d):
    ranks = G.random_ranks(O.num_subsets(144, d), NSAMPLE, seed=7100 + 10 * d + conv)
    rc, rk = O.c_forward_sample(inst.sigma, d, ranks, conv)
    smu, skap = fp64_scales(inst.sigma, d, ranks, conv)
    arb = _arbiter(inst.sigma, d, ranks, conv)
    ec, ek = np.abs(rc - arb[:, 0]), np.abs(rk - arb[:, 1])
    tc, tk = fp64_tolerance(arb[:, 0], smu), fp64_tolerance(arb[:, 1], skap)
    # one FP64 evaluation uses at most half of the tolerance
    assert np.all(ec <= 0.5 * tc), (ec / tc).max()
    assert np.all(ek <= 0.5 * tk), (ek / tk).max()
    # the cumulant tolerance stays within SLACK of the measured error
    assert ek.max() > 0.0
    assert np.median(tk) <= SLACK * ek.max(), (np.median(tk), ek.max())


def test_old_floor_fails_the_slack_pin(inst):
    """Planted: the previous floor (64 u times the propagated magnitude of the
    cancelling terms) is far looser than the measured error at order 5."""
    d = 5
    ranks = G.random_ranks(O.num_subsets(144, d), NSAMPLE, seed=7150)
    _, rk = O.c_forward_sample(inst.sigma, d, ranks)
    _, vkap = O.c_error_floor(inst.sigma, d, ranks)
    arb = _arbiter(inst.sigma, d, ranks, O.CLICK)
    ek = np.abs(rk - arb[:, 1])
    assert np.median(64 * U * vkap) > SLACK * ek.max()


def _weak_light(M, seed=1):
    """Independent lossy squeezed modes with click probabilities of a few
    percent, coupled by a weak random symmetric perturbation (Q stays SPD)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.3, 1.0, M)
    eta = rng.uniform(0.3, 0.6, M)
    sigma = G.product_state_covariance(r, eta)
    B = rng.standard_normal((2 * M, 2 * M)) * 5e-4
    return sigma + 0.5 * (B + B.T)


@pytest.mark.parametrize("d", [2, 3])
def test_weak_light_needs_the_carried_term(d):
    """Cumulants of weakly illuminated modes are high-order differences of
    probabilities near one: the rounding of the correlators dominates, so the
    partition-sum bound alone is missed by the FP64 oracle itself, while the
    full tolerance holds with room for the second evaluation."""
    M = 64
    sigma = _weak_light(M)
    ranks = G.random_ranks(O.num_subsets(M, d), 40, seed=7300 + d)
    _, rk = O.c_forward_sample(sigma, d, ranks)
    _, skap = fp64_scales(sigma, d, ranks)
    arb = _arbiter(sigma, d, ranks, O.CLICK)
    ek = np.abs(rk - arb[:, 1])
    partition_only = 1e-10 * np.maximum(np.abs(arb[:, 1]), 1e-4 * skap[0])
    assert np.any(ek > partition_only), (ek / partition_only).max()
    assert np.all(ek <= 0.5 * fp64_tolerance(arb[:, 1], skap)), \
        (ek / fp64_tolerance(arb[:, 1], skap)).max()


def test_displaced_tolerance_against_arbiter(inst):
    mu = G.input_displacement(inst)
    for d in (3, 5):
        ranks = G.random_ranks(O.num_subsets(144, d), 8, seed=7200 + d)
        rc, rk = O.c_forward_sample(inst.sigma, d, ranks, mu=mu)
        smu, skap = fp64_scales(inst.sigma, d, ranks, mu=mu)
        arb = _arbiter(inst.sigma, d, ranks, O.CLICK, mu=mu)
        assert np.all(np.abs(rc - arb[:, 0]) <= 0.5 * fp64_tolerance(arb[:, 0], smu))
        assert np.all(np.abs(rk - arb[:, 1]) <= 0.5 * fp64_tolerance(arb[:, 1], skap))


def test_c_scales_match_python_tier():
    inst = G.make_instance("m144_k5", M=12, seed=3)
    for conv in (O.CLICK, O.PARITY):
        for d in (1, 3, 5):
            ranks = np.arange(0, O.num_subsets(12, d), 37, dtype=np.int64)
            smu, skap = O.c_tolerance_scale(inst.sigma, d, ranks, conv)
            for i, r in enumerate(ranks):
                S = O.colex_unrank(d, int(r))
                assert skap[i] == pytest.approx(O.cumulant_scale(inst.sigma, S, conv), rel=1e-13)
                if conv == O.CLICK:
                    assert smu[i] == pytest.approx(O.vacuum_mass(inst.sigma, S), rel=1e-13)


def test_range_entry_matches_sampled_entry():
    inst = G.make_instance("m144_k5", M=20, seed=4)
    for conv in (O.CLICK, O.PARITY):
        r0, cnt = 1000, 2345
        c, k, smu, skap = O.c_forward_range(inst.sigma, 4, r0, cnt, conv, scales=True)
        ranks = np.arange(r0, r0 + cnt, dtype=np.int64)
        c2, k2 = O.c_forward_sample(inst.sigma, 4, ranks, conv)
        s2, t2 = O.c_tolerance_scale(inst.sigma, 4, ranks, conv)
        assert np.array_equal(c, c2) and np.array_equal(k, k2)
        assert np.array_equal(smu, s2) and np.array_equal(skap, t2)
    with pytest.raises(RuntimeError):
        O.c_forward_range(inst.sigma, 4, O.num_subsets(20, 4) - 5, 6)
