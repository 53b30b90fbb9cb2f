"""GPU parity of gbs_cumulants_shard (one colex rank range of one order, from Q
alone) against the oracle, at M = 40 and at the pseudo-photon-number-resolving
size M = 1152 (C(1152, 5) = 1.7e13 order-5 subsets, 64-bit ranks)."""
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
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("conv", [0, 1], ids=["click", "parity"])
def test_shard_is_a_slice_of_the_full_pass(P, conv):
    """Ranges at the start, inside and at the end of order 5 (partial B runs at
    both ends): with GBS_ALL_MINORS the shard runs the all-minors kernel of the
    full pass and its outputs are the same bits; the default T-shared kernel
    agrees with the full pass to FP64 rounding and with the oracle."""
    import torch
    _say("case: shard slice M=40", conv)
    inst = G.make_instance("m144_k5", M=40, seed=71)
    s = _dev(inst.sigma)
    c_all, k_all = P.gbs_cumulants(40, s, 5, conv | P.GBS_ALL_MINORS)
    c_def, k_def = P.gbs_cumulants(40, s, 5, conv)
    off = P.gbs_order_offset(40, 5)
    for r0, cnt in ((0, 1), (0, 70_001), (123_457, 99_999), (math.comb(40, 5) - 513, 513)):
        c, k = P.gbs_cumulants_shard(40, s, 5, r0, cnt, conv | P.GBS_ALL_MINORS)
        torch.cuda.synchronize()
        assert torch.equal(c, c_all[off + r0:off + r0 + cnt])
        assert torch.equal(k, k_all[off + r0:off + r0 + cnt])
        c, k = P.gbs_cumulants_shard(40, s, 5, r0, cnt, conv)
        torch.cuda.synchronize()
        # two FP64 evaluations: each within the oracle tolerance of the exact value
        ranks = np.arange(r0, r0 + cnt, dtype=np.int64)
        smu, skap = fp64_scales(inst.sigma, 5, ranks, conv)
        cd = c_def[off + r0:off + r0 + cnt].cpu().numpy()
        kd = k_def[off + r0:off + r0 + cnt].cpu().numpy()
        assert_within(c.cpu().numpy(), cd, 2 * fp64_tolerance(cd, smu), f"corr [{r0}, +{cnt})")
        assert_within(k.cpu().numpy(), kd, 2 * fp64_tolerance(kd, skap), f"cum [{r0}, +{cnt})")
    ranks = np.arange(123_457, 123_457 + 2000, dtype=np.int64)
    c, k = P.gbs_cumulants_shard(40, s, 5, 123_457, 2000, conv)
    rc, rk = O.c_forward_sample(inst.sigma, 5, ranks, conv)
    smu, skap = fp64_scales(inst.sigma, 5, ranks, conv)
    assert_within(c.cpu().numpy(), rc, fp64_tolerance(rc, smu), "M=40 corr")
    assert_within(k.cpu().numpy(), rk, fp64_tolerance(rk, skap), "M=40 cum")


@pytest.mark.parametrize("conv", [0, 1], ids=["click", "parity"])
@pytest.mark.parametrize("order", [3, 4, 5])
def test_shard_every_rank_small(P, order, conv):
    """M = 13: every subset of orders 3-5 against the oracle, as one range, as
    many ragged ranges (the same bits), and without the correlator output."""
    import torch
    _say("case: shard M=13", order, conv)
    inst = G.make_instance("m144_k5", M=13, seed=13)
    s = _dev(inst.sigma)
    n = math.comb(13, order)
    ranks = np.arange(n, dtype=np.int64)
    rc, rk = O.c_forward_sample(inst.sigma, order, ranks, conv)
    smu, skap = fp64_scales(inst.sigma, order, ranks, conv)
    c, k = P.gbs_cumulants_shard(13, s, order, 0, n, conv)
    assert_within(c.cpu().numpy(), rc, fp64_tolerance(rc, smu), f"d={order} corr")
    assert_within(k.cpu().numpy(), rk, fp64_tolerance(rk, skap), f"d={order} cum")
    cuts = [0, 1, 2, 7, 30, n // 2, n // 2 + 1, n - 3, n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b <= a:
            continue
        c2, k2 = P.gbs_cumulants_shard(13, s, order, a, b - a, conv)
        torch.cuda.synchronize()
        assert torch.equal(c2, c[a:b]) and torch.equal(k2, k[a:b]), (a, b)
    _, k3 = P.gbs_cumulants_shard(13, s, order, 0, n, conv, want_corr=False)
    assert torch.equal(k3, k)


@pytest.fixture(scope="module")
def pnr():
    return G.pseudo_pnr_covariance(G.make_instance("m144_k5").sigma, 8)


@pytest.mark.parametrize("order,where", [(5, "start"), (5, "middle"), (5, "end"), (3, "end"),
                                         (4, "middle")])
def test_pseudo_pnr_m1152(P, pnr, order, where):
    """Shards of the M = 1152 pseudo-PNR covariance: the first, a middle and the
    last ranks of an order (order-5 ranks beyond 2^32)."""
    import torch
    _say("case: shard M=1152", order, where)
    M = 1152
    total = math.comb(M, order)
    cnt = 262_144
    r0 = {"start": 0, "middle": total // 2 - cnt // 2, "end": total - cnt}[where]
    c, k = P.gbs_cumulants_shard(M, _dev(pnr), order, r0, cnt, 0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(order * 10 + len(where))
    local = np.unique(np.concatenate([rng.integers(0, cnt, size=1500), np.arange(cnt - 100, cnt),
                                      np.arange(0, 50)]))
    ranks = r0 + local
    rc, rk = O.c_forward_sample(pnr, order, ranks)
    smu, skap = fp64_scales(pnr, order, ranks)
    assert_within(c.cpu().numpy()[local], rc, fp64_tolerance(rc, smu), f"M=1152 d={order} corr")
    assert_within(k.cpu().numpy()[local], rk, fp64_tolerance(rk, skap), f"M=1152 d={order} cum")


def test_shard_range_lists_under_threads(P):
    """Two host threads calling with many distinct ranges at once (every call
    builds or reuses a cached T list; the cache keeps eight, so lists are evicted
    while the other thread may hold one): every result equals the same slice of
    a single whole-order call, bit for bit."""
    import threading
    import torch
    _say("case: shard T lists under two threads, M=13 order 5")
    inst = G.make_instance("m144_k5", M=13, seed=13)
    s = _dev(inst.sigma)
    n = math.comb(13, 5)
    c_ref, k_ref = P.gbs_cumulants_shard(13, s, 5, 0, n, 0)
    torch.cuda.synchronize()
    errors = []

    def work(tid):
        try:
            for rnd in range(2):
                for i in range(12):
                    r0 = (37 * i + 11 * tid + rnd) % (n - 40)
                    cnt = 1 + (53 * i + 17 * tid) % (n - r0)
                    c, k = P.gbs_cumulants_shard(13, s, 5, r0, cnt, 0)
                    torch.cuda.synchronize()
                    if not (torch.equal(c, c_ref[r0:r0 + cnt]) and torch.equal(k, k_ref[r0:r0 + cnt])):
                        errors.append((tid, rnd, r0, cnt))
        except Exception as e:  # reported below
            errors.append((tid, repr(e)))

    ts = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors[:5]


def _chunk_starts(M, order, max_t=1 << 16):
    """Ranks at which a whole-order range starts a new chunk of at most max_t T's
    (T in colex order, those with a nonempty triangle a < b_0 < min T)."""
    import itertools
    nt = order - 2
    starts, k = [], 0
    # colex order of the T's: sort by the reversed tuple
    ts = sorted(itertools.combinations(range(M), nt), key=lambda t: t[::-1])
    for t in ts:
        if math.comb(t[0], 2) == 0:
            continue
        if k and k % max_t == 0:
            starts.append(sum(math.comb(t[j], j + 3) for j in range(nt)))
        k += 1
    return starts


def test_shard_in_chunks_m100(P):
    """Order 5 at M = 100 (161,700 T's) runs as three chunks of at most 2^16 T's:
    outputs around both chunk boundaries against the oracle, and ranges that
    straddle a boundary equal to the same slice of the whole-order call, bit
    for bit."""
    import torch
    _say("case: shard in chunks M=100 order 5")
    inst = G.make_instance("m144_k5", M=100, seed=7)
    s = _dev(inst.sigma)
    n = math.comb(100, 5)
    starts = _chunk_starts(100, 5)
    assert len(starts) == 2, starts
    c, k = P.gbs_cumulants_shard(100, s, 5, 0, n, 0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    local = np.unique(np.concatenate([np.arange(b - 300, b + 300) for b in starts] +
                                     [rng.integers(0, n, size=1500), np.arange(n - 50, n)]))
    rc, rk = O.c_forward_sample(inst.sigma, 5, local)
    smu, skap = fp64_scales(inst.sigma, 5, local)
    assert_within(c.cpu().numpy()[local], rc, fp64_tolerance(rc, smu), "M=100 chunks corr")
    assert_within(k.cpu().numpy()[local], rk, fp64_tolerance(rk, skap), "M=100 chunks cum")
    for b in starts:
        r0, cnt = b - 777, 2000
        c2, k2 = P.gbs_cumulants_shard(100, s, 5, r0, cnt, 0)
        torch.cuda.synchronize()
        assert torch.equal(c2, c[r0:r0 + cnt]) and torch.equal(k2, k[r0:r0 + cnt]), b


@pytest.mark.parametrize("case", ["pivot", "coupling"])
def test_shard_not_spd_reported(P, case):
    """A non-physical covariance: GBS_E_NOT_SPD and a failing subset that holds
    the bad modes.  "pivot": mode 2 has negative variances, caught in the
    factors of T, b_0 or a; "coupling": modes 0 and 1 are each physical but
    their x quadratures are coupled beyond positive definiteness, which only the
    main loop's pair leaves (a = 0, b_0 = 1) can see."""
    import torch
    _say("case: shard not SPD", case)
    M = 8
    sigma = G.vacuum_covariance(M)
    if case == "pivot":
        sigma[2, 2] = sigma[2 + M, 2 + M] = -0.9
        bad = {2}
    else:
        sigma[0, 1] = sigma[1, 0] = 1.5  # Q restricted to (x_0, x_1): [[1, 1.5], [1.5, 1]]
        bad = {0, 1}
    s = torch.from_numpy(sigma).to("cuda:0")
    with pytest.raises(P.GBSError) as ei:
        P.gbs_cumulants_shard(M, s, 5, 0, math.comb(M, 5), 0)
    assert ei.value.status == P.GBS_E_NOT_SPD
    st, order, rank = P.gbs_last_error()
    assert st == P.GBS_E_NOT_SPD and order == 5
    assert bad <= set(P.gbs_colex_unrank(5, rank))
    P.gbs_cumulants_shard(M, torch.from_numpy(G.vacuum_covariance(M)).to("cuda:0"), 5, 0,
                          math.comb(M, 5), 0)
    assert P.gbs_last_error()[0] == P.GBS_OK
