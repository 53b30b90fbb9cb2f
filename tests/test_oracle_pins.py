"""Pins for the CPU oracle: every check here is fixed by the paper's mathematics or
by an independent route, never by the oracle's own formula retyped.

Citations name the paper's sections and equations.
"""
import itertools
import math

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O


# ---------------------------------------------------------------------------
# layout


def test_colex_rank_unrank_roundtrip():
    for M, d in [(7, 1), (7, 3), (9, 4), (10, 5)]:
        seen = []
        for S in O.subsets_colex(M, d):
            r = O.colex_rank(S)
            assert O.colex_unrank(d, r) == S
            seen.append(r)
        assert seen == list(range(math.comb(M, d)))


def test_colex_order_is_sorted_by_reversed_tuple():
    subs = list(O.subsets_colex(8, 3))
    assert subs == sorted(itertools.combinations(range(8), 3), key=lambda s: s[::-1])


def test_output_counts():
    # C(144,5) order-5 correlators (caption of Fig. 1) and the K<=5 total
    assert O.num_subsets(144, 5) == 481_008_528
    assert O.total_outputs(144, 5) == 498_685_188
    assert O.total_outputs(16, 3) == 696
    assert O.total_outputs(100, 4) == 4_087_975
    assert O.order_offset(144, 5) == 144 + 10_296 + 487_344 + 17_178_876


def test_partition_counts_and_weights():
    # Bell numbers B_d (cost discussion after Eq. corre_cov_main)
    assert [len(O.set_partitions(d)) for d in range(1, 6)] == [1, 2, 5, 15, 52]
    # sum of weights vanishes for |S| >= 2: the cumulant of a constant variable
    for d in range(2, 6):
        assert sum(O.partition_weight(len(pi)) for pi in O.set_partitions(d)) == 0
    # block-count profile of the 52 partitions of a 5-set: Stirling numbers S(5,k)
    prof = [0] * 6
    for pi in O.set_partitions(5):
        prof[len(pi)] += 1
    assert prof[1:] == [1, 15, 25, 10, 1]


# ---------------------------------------------------------------------------
# closed forms


@pytest.mark.parametrize("r,eta", [(0.3, 1.0), (0.7, 0.4), (1.1, 0.9), (1.5, 0.25)])
def test_single_mode_click_probability(r, eta):
    """mu({k}) = 1 - det(Q_k)^(-1/2) with, for an x-squeezed lossy mode,
    det Q_k = [1 - eta(1 - e^{-2r})/2][1 + eta(e^{2r} - 1)/2]."""
    sigma = G.product_state_covariance(np.array([r]), np.array([eta]))
    det = (1 - eta * (1 - math.exp(-2 * r)) / 2) * (1 + eta * (math.exp(2 * r) - 1) / 2)
    corr, cum = O.correlators_and_cumulants(sigma, 1)
    assert corr[0] == pytest.approx(1 - det ** -0.5, rel=1e-14)
    assert cum[0] == corr[0]
    if eta == 1.0:
        # pure squeezed vacuum: vacuum probability sech r
        assert 1 - corr[0] == pytest.approx(1 / math.cosh(r), rel=1e-14)


def test_vacuum_state():
    sigma = G.vacuum_covariance(5)
    corr, cum = O.correlators_and_cumulants(sigma, 4)
    assert np.all(corr == 0.0) and np.all(np.abs(cum) < 1e-15)
    c, k = O.correlators_and_cumulants(sigma, 4, O.PARITY)
    assert np.allclose(c, 1.0, atol=1e-15)
    assert np.allclose(k[:5], 1.0, atol=1e-15) and np.all(np.abs(k[5:]) < 1e-14)


def test_product_state_factorises_and_cumulants_vanish():
    """Independent modes: joint moments factorise and every cumulant of order >= 2
    vanishes (App. A.2, cumulants of independent variables)."""
    rng = np.random.default_rng(3)
    M = 6
    r = rng.uniform(0.4, 1.4, M)
    eta = rng.uniform(0.2, 0.9, M)
    sigma = G.product_state_covariance(r, eta)
    corr, cum = O.correlators_and_cumulants(sigma, 4)
    single = corr[:M]
    pos = 0
    for d in range(1, 5):
        for S in O.subsets_colex(M, d):
            assert corr[pos] == pytest.approx(np.prod(single[list(S)]), rel=1e-12)
            if d >= 2:
                assert abs(cum[pos]) < 1e-15
            pos += 1


@pytest.mark.parametrize("r", [0.3, 0.8, 1.3])
def test_two_mode_squeezed_vacuum(r):
    """Pure TMSV (the input block of Eq. jiuzhang_input_cov): both modes are
    thermal with mean photon number sinh^2 r and perfectly photon-number
    correlated, so mu_1 = mu_2 = mu_12 = tanh^2 r and kappa~_12 = tanh^2 r sech^2 r.
    Embedded on non-adjacent modes (1, 3) of M = 5 to exercise the xxpp indexing."""
    M = 5
    sigma = G.tmsv_covariance(r, M=M, i=1, j=3)
    corr, cum = O.correlators_and_cumulants(sigma, 3)
    t2 = math.tanh(r) ** 2
    idx1 = O.colex_rank((1,))
    idx3 = O.colex_rank((3,))
    idx13 = O.order_offset(M, 2) + O.colex_rank((1, 3))
    assert corr[idx1] == pytest.approx(t2, rel=1e-13)
    assert corr[idx3] == pytest.approx(t2, rel=1e-13)
    assert corr[idx13] == pytest.approx(t2, rel=1e-13)
    assert cum[idx13] == pytest.approx(t2 / math.cosh(r) ** 2, rel=1e-12)
    # vacuum modes never click; every other cumulant vanishes
    for S, pos in zip(itertools.chain(*(O.subsets_colex(M, d) for d in (1, 2, 3))), range(len(corr))):
        if not set(S) <= {1, 3}:
            assert corr[pos] == 0.0 and abs(cum[pos]) < 1e-15


# ---------------------------------------------------------------------------
# independent brute force: Torontonian pattern probabilities (App. F)


@pytest.fixture(scope="module")
def small_instance():
    return G.make_instance("m16_k3", M=6, seed=11)


@pytest.fixture(scope="module")
def small_patterns(small_instance):
    return O.pattern_probabilities(small_instance.sigma)


def test_torontonian_is_a_distribution(small_patterns):
    assert small_patterns.sum() == pytest.approx(1.0, abs=1e-12)
    assert small_patterns.min() > 0


def test_click_correlators_match_brute_force(small_instance, small_patterns):
    """mu(S) = P(every mode of S clicks) = sum of p(x) over patterns with x_S = 1
    (Eq. joint_moments_def)."""
    M = small_instance.M
    corr, _ = O.correlators_and_cumulants(small_instance.sigma, M)
    pos = 0
    for d in range(1, M + 1):
        for S in O.subsets_colex(M, d):
            mask = sum(1 << k for k in S)
            ref = math.fsum(small_patterns[x] for x in range(1 << M) if x & mask == mask)
            assert corr[pos] == pytest.approx(ref, rel=1e-11, abs=1e-14)
            pos += 1


def test_parity_correlators_match_brute_force(small_instance, small_patterns):
    """c(S) = E[prod (-1)^{x_k}] (Eq. correlators_def_bitstrings)."""
    M = small_instance.M
    corr, _ = O.correlators_and_cumulants(small_instance.sigma, 4, O.PARITY)
    pos = 0
    for d in range(1, 5):
        for S in O.subsets_colex(M, d):
            mask = sum(1 << k for k in S)
            ref = math.fsum(small_patterns[x] * (-1) ** bin(x & mask).count("1")
                            for x in range(1 << M))
            assert corr[pos] == pytest.approx(ref, rel=1e-11, abs=1e-13)
            pos += 1


def test_fourier_reconstruction():
    """p(x) = 2^-M sum_S chi_S(x) c(S) (Eq. prob_dist_corr) with all orders
    (K = M = 5) reproduces the Torontonian pattern probabilities."""
    inst = G.make_instance("m144_k5", M=5, seed=21)
    probs = O.pattern_probabilities(inst.sigma)
    corr, _ = O.correlators_and_cumulants(inst.sigma, 5, O.PARITY)
    c = {(): 1.0}
    pos = 0
    for d in range(1, 6):
        for S in O.subsets_colex(5, d):
            c[S] = corr[pos]
            pos += 1
    for x in range(32):
        rec = math.fsum((-1) ** sum((x >> k) & 1 for k in S) * v for S, v in c.items()) / 32
        assert rec == pytest.approx(probs[x], rel=1e-10, abs=1e-14)


# ---------------------------------------------------------------------------
# identities between the two conventions and the partition sums (App. A.2, B)


@pytest.fixture(scope="module")
def mid_instance():
    return G.make_instance("m144_k5", M=7, seed=31)


def _as_dict(M, K, arr):
    out = {}
    pos = 0
    for d in range(1, K + 1):
        for S in O.subsets_colex(M, d):
            out[S] = arr[pos]
            pos += 1
    return out


def test_parity_click_bridge(mid_instance):
    """kappa(S) = (-2)^|S| kappa~(S) for |S| > 1, kappa({k}) = 1 - 2 E[x_k]
    (Eq. cumulant_exponential); both sides computed by separate routes."""
    M, K = mid_instance.M, 5
    mu, kt = O.correlators_and_cumulants(mid_instance.sigma, K, O.CLICK)
    c, kp = O.correlators_and_cumulants(mid_instance.sigma, K, O.PARITY)
    pos = 0
    for d in range(1, K + 1):
        for _ in O.subsets_colex(M, d):
            if d == 1:
                assert kp[pos] == pytest.approx(1 - 2 * mu[pos], rel=1e-14)
            else:
                assert kp[pos] == pytest.approx((-2) ** d * kt[pos], rel=1e-6, abs=1e-14)
            pos += 1


def test_moments_from_cumulants_roundtrip(mid_instance):
    """mu(S) = sum_pi prod_B kappa~(B) (Eq. moments_cumulants_rel) and
    c(S) = sum_pi prod_B kappa(B) (Eq. correlators_cumulants_rel)."""
    M, K = mid_instance.M, 5
    for conv in (O.CLICK, O.PARITY):
        corr, cum = O.correlators_and_cumulants(mid_instance.sigma, K, conv)
        m = _as_dict(M, K, corr)
        k = _as_dict(M, K, cum)
        for S in m:
            tot = math.fsum(math.prod(k[tuple(S[i] for i in b)] for b in pi)
                            for pi in O.set_partitions(len(S)))
            assert tot == pytest.approx(m[S], rel=1e-12, abs=1e-15)


def test_fixed_element_recursion(mid_instance):
    """c(S' + {n}) = sum_{R subset S'} kappa(R + {n}) c(S' minus R)
    (Eq. correlators_expanded_2), with c(empty) = 1."""
    M, K = mid_instance.M, 5
    corr, cum = O.correlators_and_cumulants(mid_instance.sigma, K, O.PARITY)
    c = _as_dict(M, K, corr)
    c[()] = 1.0
    k = _as_dict(M, K, cum)
    for S in (s for s in c if len(s) >= 2):
        n, Sp = S[-1], S[:-1]
        tot = []
        for R in O.all_subsets(Sp):
            rest = tuple(x for x in Sp if x not in R)
            tot.append(k[tuple(sorted(R + (n,)))] * c[rest])
        assert math.fsum(tot) == pytest.approx(c[S], rel=1e-12, abs=1e-14)


# ---------------------------------------------------------------------------
# symmetries


def test_local_phase_rotation_invariance(mid_instance):
    """Threshold detectors are phase insensitive (POVM of App. D.1): rotating each
    mode's quadratures by its own phase changes no output.  A wrong x/p pairing of
    rows k and k+M breaks this."""
    rng = np.random.default_rng(5)
    rot = G.local_phase_rotation(mid_instance.sigma, rng.uniform(0, 2 * np.pi, mid_instance.M))
    a = O.correlators_and_cumulants(mid_instance.sigma, 4)
    b = O.correlators_and_cumulants(rot, 4)
    assert np.allclose(a[0], b[0], rtol=1e-11, atol=1e-15)
    assert np.allclose(a[1], b[1], rtol=1e-6, atol=1e-15)


def test_mode_permutation_equivariance(mid_instance):
    M = mid_instance.M
    perm = np.random.default_rng(9).permutation(M)
    sp = G.mode_permutation(mid_instance.sigma, perm)
    corr, cum = O.correlators_and_cumulants(mid_instance.sigma, 3)
    corr_p, cum_p = O.correlators_and_cumulants(sp, 3)
    m = _as_dict(M, 3, corr)
    mp = _as_dict(M, 3, corr_p)
    for S, v in mp.items():
        assert v == pytest.approx(m[tuple(sorted(perm[list(S)]))], rel=1e-12)


# ---------------------------------------------------------------------------
# FP64 accuracy against a 40-digit evaluation at the full M = 144 workload


def test_oracle_against_high_precision_arbiter():
    inst = G.make_instance("m144_k5")
    ranks = G.random_ranks(math.comb(144, 5), 6, seed=7)
    for r in ranks:
        S = O.colex_unrank(5, int(r))
        mu, kt = O.subset_values(inst.sigma, S)
        mu_a, kt_a = O.arbiter_values(inst.sigma, S)
        assert mu == pytest.approx(mu_a, rel=1e-12)
        scale = O.cumulant_scale(inst.sigma, S)
        assert abs(kt - kt_a) <= 1e-14 * scale


# ---------------------------------------------------------------------------
# C tier against the Python tier


@pytest.mark.parametrize("conv", [O.CLICK, O.PARITY])
def test_c_oracle_matches_python(c_oracle, conv):
    inst = G.make_instance("m16_k3")
    a = O.correlators_and_cumulants(inst.sigma, 3, conv)
    b = O.c_forward(inst.sigma, 3, conv, threads=2)
    assert np.allclose(a[0], b[0], rtol=1e-13, atol=1e-15)
    assert np.allclose(a[1], b[1], rtol=1e-8, atol=1e-14)
    m = G.make_instance("m144_k5", M=9, seed=2)
    a = O.correlators_and_cumulants(m.sigma, 5, conv)
    b = O.c_forward(m.sigma, 5, conv, threads=2)
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=1e-15)
    assert np.allclose(a[1], b[1], rtol=1e-7, atol=1e-14)


def test_c_oracle_sampled_matches_full(c_oracle):
    inst = G.make_instance("m144_k5", M=20, seed=4)
    corr, cum = O.c_forward(inst.sigma, 4, threads=2)
    ranks = G.random_ranks(math.comb(20, 4), 300, seed=1)
    sc, sk = O.c_forward_sample(inst.sigma, 4, ranks, threads=2)
    off = O.order_offset(20, 4)
    assert np.array_equal(sc, corr[off + ranks]) and np.array_equal(sk, cum[off + ranks])


# ---------------------------------------------------------------------------
# gradient of the cumulant-matching loss


def _loss(sigma, K, target):
    _, cum = O.correlators_and_cumulants(sigma, K)
    return math.fsum((cum - target) ** 2)


def test_gradient_against_finite_differences():
    inst = G.make_instance("grad_m144_k3", M=5, seed=41)
    K = 3
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.correlators_and_cumulants(sig_t, K)
    loss, grad = O.cumulant_loss_and_grad(inst.sigma, K, target)
    assert loss == pytest.approx(_loss(inst.sigma, K, target), rel=1e-13)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(4):
        D = rng.standard_normal(inst.sigma.shape)
        D = 0.5 * (D + D.T)
        fd = (_loss(inst.sigma + h * D, K, target) - _loss(inst.sigma - h * D, K, target)) / (2 * h)
        an = float(np.sum(grad * D))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_parameter_chain_against_finite_differences():
    inst = G.make_instance("grad_m144_k3", M=5, seed=43)
    K = 3
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.correlators_and_cumulants(sig_t, K)
    _, grad = O.cumulant_loss_and_grad(inst.sigma, K, target)
    d_eta, d_r = O.covariance_param_grad(inst.U, inst.r, inst.eta, grad)
    h = 1e-6
    for k in range(inst.M):
        e = np.zeros(inst.M)
        e[k] = h
        f = lambda r, eta: _loss(G.lossy_squeezed_covariance(inst.U, r, eta), K, target)
        fd_eta = (f(inst.r, inst.eta + e) - f(inst.r, inst.eta - e)) / (2 * h)
        fd_r = (f(inst.r + e, inst.eta) - f(inst.r - e, inst.eta)) / (2 * h)
        assert d_eta[k] == pytest.approx(fd_eta, rel=1e-6, abs=1e-11)
        assert d_r[k] == pytest.approx(fd_r, rel=1e-6, abs=1e-11)


def test_product_state_gradient_closed_form():
    """Product state, loss = (mu_k - t)^2 over order 1 only: dL/deta_k =
    2 (mu_k - t) d mu_k/d eta_k with mu_k = 1 - det(Q_k)^{-1/2} in closed form."""
    r = np.array([0.6, 1.0, 0.8])
    eta = np.array([0.3, 0.5, 0.7])
    U = np.eye(3, dtype=complex)
    sigma = G.lossy_squeezed_covariance(U, r, eta)
    target = np.array([0.1, 0.2, 0.3])
    _, grad = O.cumulant_loss_and_grad(sigma, 1, target)
    d_eta, d_r = O.covariance_param_grad(U, r, eta, grad)
    for k in range(3):
        a = 1 - eta[k] * (1 - math.exp(-2 * r[k])) / 2
        b = 1 + eta[k] * (math.exp(2 * r[k]) - 1) / 2
        mu = 1 - (a * b) ** -0.5
        dmu_deta = 0.5 * (a * b) ** -1.5 * (-(1 - math.exp(-2 * r[k])) / 2 * b
                                             + a * (math.exp(2 * r[k]) - 1) / 2)
        assert d_eta[k] == pytest.approx(2 * (mu - target[k]) * dmu_deta, rel=1e-12)


def test_c_gradient_matches_python(c_oracle):
    inst = G.make_instance("grad_m144_k3", M=7, seed=45)
    K = 3
    _, _, sig_t = G.make_grad_target(inst)
    _, target = O.correlators_and_cumulants(sig_t, K)
    loss_p, grad_p = O.cumulant_loss_and_grad(inst.sigma, K, target)
    loss_c, grad_c = O.c_loss_grad(inst.sigma, K, target, threads=2)
    assert loss_c == pytest.approx(loss_p, rel=1e-12)
    assert np.allclose(grad_c, grad_p, rtol=1e-9, atol=1e-14 * np.abs(grad_p).max())


# ---------------------------------------------------------------------------
# stored closed-form values (tests/golden/closed_forms.txt)


def test_golden_closed_forms():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert rows
    for kind, r, eta, mu, kap in rows:
        r, eta, mu, kap = float(r), float(eta), float(mu), float(kap)
        if kind == "tmsv":
            corr, cum = O.correlators_and_cumulants(G.tmsv_covariance(r, M=2), 2)
            assert corr[2] == pytest.approx(mu, rel=1e-13)
            assert cum[2] == pytest.approx(kap, rel=1e-12)
        else:
            sigma = G.product_state_covariance(np.array([r]), np.array([eta]))
            corr, cum = O.correlators_and_cumulants(sigma, 1)
            assert corr[0] == pytest.approx(mu, rel=1e-14) and cum[0] == pytest.approx(kap, rel=1e-14)


def test_golden_m16_matches_oracle():
    import os
    inst = G.make_instance("m16_k3")
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "m16_k3_click.npz"))
    assert np.array_equal(g["sigma"], inst.sigma)
    corr, cum = O.correlators_and_cumulants(inst.sigma, 3)
    assert np.array_equal(g["corr"], corr) and np.array_equal(g["cum"], cum)
