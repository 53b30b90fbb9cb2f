"""GPU parity of gbs_cumulants_shard (one colex rank range of one order, from Q
alone) against the oracle, at M = 40 and at the pseudo-photon-number-resolving
size M = 1152 (C(1152, 5) = 1.7e13 order-5 subsets, 64-bit ranks)."""
import math
import sys

import numpy as np
import pytest

import gbs_inputs as G
import oracle as O
from parity import assert_within, fp64_tolerance

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
    import torch
    _say("case: shard slice M=40", conv)
    inst = G.make_instance("m144_k5", M=40, seed=71)
    s = _dev(inst.sigma)
    c_all, k_all = P.gbs_cumulants(40, s, 5, conv | P.GBS_ALL_MINORS)
    off = P.gbs_order_offset(40, 5)
    for r0, cnt in ((0, 1), (0, 70_001), (123_457, 99_999), (math.comb(40, 5) - 513, 513)):
        c, k = P.gbs_cumulants_shard(40, s, 5, r0, cnt, conv)
        torch.cuda.synchronize()
        assert torch.equal(c, c_all[off + r0:off + r0 + cnt])
        assert torch.equal(k, k_all[off + r0:off + r0 + cnt])
    ranks = np.arange(123_457, 123_457 + 2000, dtype=np.int64)
    c, k = P.gbs_cumulants_shard(40, s, 5, 123_457, 2000, conv)
    rc, rk = O.c_forward_sample(inst.sigma, 5, ranks, conv)
    vmu, vkap = O.c_error_floor(inst.sigma, 5, ranks, conv)
    assert_within(c.cpu().numpy(), rc, fp64_tolerance(rc, vmu), "M=40 corr")
    assert_within(k.cpu().numpy(), rk, fp64_tolerance(rk, vkap), "M=40 cum")


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
    vmu, vkap = O.c_error_floor(pnr, order, ranks)
    assert_within(c.cpu().numpy()[local], rc, fp64_tolerance(rc, vmu), f"M=1152 d={order} corr")
    assert_within(k.cpu().numpy()[local], rk, fp64_tolerance(rk, vkap), f"M=1152 d={order} cum")
