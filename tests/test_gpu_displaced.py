"""GPU parity of gbs_cumulants_displaced (first moments mu != 0; App. D.1, Eq.
vacuum_gaussian_prob) against the CPU oracle, element by element, through the
C ABI."""
import math
import sys

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from parity import assert_within, fp64_scales, fp64_tolerance

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2511_14923_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.lib()
    return P


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def _run(P, sigma, mu, K, flags=0):
    import torch
    M = sigma.shape[0] // 2
    corr, cum = P.gbs_cumulants_displaced(M, _dev(sigma), _dev(mu), K, flags)
    torch.cuda.synchronize()
    return corr.cpu().numpy(), cum.cpu().numpy()


def _check_full(P, sigma, mu, K, conv, flags_extra=0, what=""):
    M = sigma.shape[0] // 2
    corr, cum = _run(P, sigma, mu, K, conv | flags_extra)
    rc, rk = O.c_forward(sigma, K, conv, mu=mu)
    for d in range(1, K + 1):
        a, b = O.order_offset(M, d), O.order_offset(M, d + 1)
        ranks = np.arange(b - a, dtype=np.int64)
        smu, skap = fp64_scales(sigma, d, ranks, conv, mu=mu)
        assert_within(corr[a:b], rc[a:b], fp64_tolerance(rc[a:b], smu), f"{what} corr d={d}")
        assert_within(cum[a:b], rk[a:b], fp64_tolerance(rk[a:b], skap), f"{what} cum d={d}")
    return corr, cum


KERNELS = [0, 16]  # order-recursive (default), GBS_ALL_MINORS
KERNEL_IDS = ["recursive", "all_minors"]


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
@pytest.mark.parametrize("conv", [0, 1], ids=["click", "parity"])
def test_displaced_m12_k5_full(P, conv, kernel):
    _say("case: displaced M=12 K=5 full", conv, kernel)
    inst = G.make_instance("m144_k5", M=12, seed=41)
    mu = G.input_displacement(inst, seed=42)
    _check_full(P, inst.sigma, mu, 5, conv, kernel, "M=12")


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
def test_displaced_m40_k5_full(P, kernel):
    """658,008 order-5 subsets: thousands of workgroups and a ragged last one."""
    _say("case: displaced M=40 K=5 full", kernel)
    inst = G.make_instance("m144_k5", M=40, seed=43)
    mu = G.input_displacement(inst, seed=44, amp2_range=(0.2, 1.0))
    _check_full(P, inst.sigma, mu, 5, 0, kernel, "M=40")


def _picks(M, K, n, seed, tail=200):
    picks = {}
    for d in range(1, K + 1):
        cnt = math.comb(M, d)
        r = G.random_ranks(cnt, min(n, cnt), seed=seed + d)
        t = np.arange(max(0, cnt - tail), cnt, dtype=np.int64)
        picks[d] = np.unique(np.concatenate([r, t]))
    return picks


def _check_sampled(P, sigma, mu, K, picks, conv, what):
    import torch
    M = sigma.shape[0] // 2
    corr, cum = P.gbs_cumulants_displaced(M, _dev(sigma), _dev(mu), K, conv)
    torch.cuda.synchronize()
    for d, ranks in picks.items():
        idx = torch.from_numpy(O.order_offset(M, d) + ranks).to("cuda:0")
        gc, gk = corr[idx].cpu().numpy(), cum[idx].cpu().numpy()
        rc, rk = O.c_forward_sample(sigma, d, ranks, conv, mu=mu)
        smu, skap = fp64_scales(sigma, d, ranks, conv, mu=mu)
        assert_within(gc, rc, fp64_tolerance(rc, smu), f"{what} corr d={d}")
        assert_within(gk, rk, fp64_tolerance(rk, skap), f"{what} cum d={d}")


@pytest.mark.parametrize("conv", [0, 1], ids=["click", "parity"])
def test_displaced_m144_k5_sampled(P, conv):
    """The M = 144, K = 5 workload with seeded input displacements, in the
    launch configuration the benchmark times; sampled ranks of every order
    plus the ragged end of each order."""
    _say("case: displaced M=144 K=5 sampled", conv)
    inst = G.make_instance("m144_k5")
    mu = G.input_displacement(inst)
    picks = _picks(144, 5, 4000 if conv == 0 else 1500, 50)
    _check_sampled(P, inst.sigma, mu, 5, picks, conv, "M=144")


def test_displaced_beyond_group_kernel(P):
    """M = 160, K = 4: orders 3 and 4 need more (T, a) records than the group
    kernel holds, so displaced calls take the order-recursive kernel there."""
    _say("case: displaced M=160 K=4 sampled")
    inst = G.make_instance("m144_k5", M=160, seed=45)
    mu = G.input_displacement(inst, seed=46)
    _check_sampled(P, inst.sigma, mu, 4, _picks(160, 4, 4000, 70, tail=300), 0, "M=160")


def test_displaced_64bit_ranks(P):
    """M = 1500, K = 3: more than 2^29 order-3 subsets (64-bit rank arithmetic)."""
    _say("case: displaced M=1500 K=3 sampled")
    inst = G.make_instance("m144_k5", M=1500, seed=47)
    mu = G.input_displacement(inst, seed=48)
    _check_sampled(P, inst.sigma, mu, 3, _picks(1500, 3, 2000, 60, tail=300), 0, "M=1500")


@pytest.mark.parametrize("kernel", KERNELS, ids=KERNEL_IDS)
@pytest.mark.parametrize("M,K", [(1, 1), (2, 2), (5, 5), (6, 5), (17, 3), (257, 2)])
def test_displaced_edge_sizes(P, M, K, kernel):
    _say("case: displaced edge", M, K, kernel)
    inst = G.make_instance("m144_k5", M=M, seed=100 + M)
    mu = G.input_displacement(inst, seed=200 + M)
    _check_full(P, inst.sigma, mu, K, 0, kernel, f"M={M}")


def test_zero_mean_matches_undisplaced(P):
    import torch
    _say("case: displaced zero mean")
    inst = G.make_instance("m144_k5", M=30, seed=51)
    s = _dev(inst.sigma)
    c0, k0 = P.gbs_cumulants(30, s, 4, 0)
    c1, k1 = P.gbs_cumulants_displaced(30, s, torch.zeros(60, dtype=torch.float64,
                                                          device="cuda:0"), 4, 0)
    torch.cuda.synchronize()
    c0, k0, c1, k1 = (x.cpu().numpy() for x in (c0, k0, c1, k1))
    for d in range(1, 5):
        a, b = O.order_offset(30, d), O.order_offset(30, d + 1)
        smu, skap = fp64_scales(inst.sigma, d, np.arange(b - a, dtype=np.int64))
        assert_within(c1[a:b], c0[a:b], 2 * fp64_tolerance(c0[a:b], smu), f"corr d={d}")
        assert_within(k1[a:b], k0[a:b], 2 * fp64_tolerance(k0[a:b], skap), f"cum d={d}")


def test_coherent_product_state_closed_form(P):
    """sigma = I/2: click correlators factorise as prod (1 - e^{-|beta_k|^2}) and
    cumulants of order >= 2 vanish (no oracle involved)."""
    _say("case: displaced coherent closed form")
    M = 20
    rng = np.random.default_rng(53)
    mu = rng.normal(scale=0.8, size=2 * M)
    f = 1.0 - np.exp(-0.5 * (mu[:M] ** 2 + mu[M:] ** 2))
    corr, cum = _run(P, G.vacuum_covariance(M), mu, 4, 0)
    pos = 0
    for d in range(1, 5):
        for S in O.subsets_colex(M, d):
            ref = float(np.prod(f[list(S)]))
            assert abs(corr[pos] - ref) <= 1e-13, (S, corr[pos], ref)
            assert abs(cum[pos] - (ref if d == 1 else 0.0)) <= 1e-13, (S, cum[pos])
            pos += 1


def test_displaced_mixed_is_unsupported(P):
    import torch
    inst = G.make_instance("m144_k5", M=8, seed=3)
    with pytest.raises(P.GBSError) as e:
        P.gbs_cumulants_displaced(8, _dev(inst.sigma), torch.zeros(16, dtype=torch.float64,
                                                                    device="cuda:0"), 3, P.GBS_MIXED)
    assert e.value.status == P.GBS_E_UNSUPPORTED
